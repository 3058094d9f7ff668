"""Plain FP64 CPU oracle of the hybrid lattice-Boltzmann / FENE-P step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.
The HIP library never calls it, and it imports nothing from the library:
the two share no code, tables or helpers.  Their only common input is the
seeded workload module.

Contents
  d3q19       lattice velocities, weights and the BGK equilibrium
  solver      array-at-a-time FP64 solver (explicit ghost layers)
  scalar      node-by-node pure-Python solver for tiny lattices
  observables deformation, orientation, elongation, masses
  components  connected-component count of the droplet phase
  mlp         FP64 forward/backward of the surrogate network

Model: Gupta & Sbragaglia, "Deformation and break-up of viscoelastic droplets
using Lattice Boltzmann Models" (arXiv:1411.2181), Section 2, Eqs. (1)-(4)
(Navier-Stokes with polymer feedback and the FENE-P constitutive law in the
droplet and matrix phases) and the Peterlin factor defined below Eq. (2).
The paper leaves the lattice discretisation to its methods paper; the
discrete readings used here are listed in each module's docstring.
"""
