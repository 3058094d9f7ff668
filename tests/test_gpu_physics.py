"""Physics of the scheme on the GPU FP64 path (which matches the CPU oracle to
1e-10 in the parity tests; the same runs on the oracle would take about half
an hour each).

Taylor's small-deformation law (the paper's Introduction cites Taylor for
the deformation measure D; the formula is Taylor's, not printed in the
paper): a droplet in simple shear at small Ca deforms to
D = Ca (19 lambda + 16)/(16 lambda + 16), oriented at 45 degrees.
The check runs at lambda = 1 with tau = 1.24 in both phases: with the
velocity-shift forcing the coexisting densities depend on tau, and a small
droplet next to a matrix of the same tau swells below tau ~ 1.24 and
dissolves above it, which moves its effective Ca.  At 1.24 its volume holds.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

R = 12.0
BOX = (144, 72, 96)          # 2R/W = 0.25
TAU = 1.24
CAS = (0.025, 0.05)


def test_taylor_small_deformation():
    import torch
    from paper_1411_2181_amd import lbmve, physics
    runs = []
    for ca in CAS:
        p, info = physics.lattice_params(*BOX, R=R, Ca=ca, De=0.0, lam=1.0, phase="N",
                                         tau_matrix=TAU, u_max=0.15)
        assert abs(p["tau"][0] - TAU) < 1e-12 and abs(p["tau"][1] - TAU) < 1e-12
        runs.append(p)
    b = lbmve.Batch(runs, "fp64")
    hist = []
    for _ in range(12):
        b.step(1000)
        hist.append(b.observe(components=True))
    torch.cuda.synchronize()
    b.close()
    d_taylor = [ca * 35.0 / 32.0 for ca in CAS]
    D = [float(np.mean([h[i]["D"] for h in hist[-3:]])) for i in range(len(CAS))]
    for i, ca in enumerate(CAS):
        vol0, vol1 = hist[0][i]["piece_nodes"][0], hist[-1][i]["piece_nodes"][0]
        theta = hist[-1][i]["theta_deg"]
        print(f"Ca {ca}: D {D[i]:.4f} (Taylor {d_taylor[i]:.4f}, ratio {D[i] / d_taylor[i]:.3f}), "
              f"theta {theta:.2f}, droplet nodes {vol0} -> {vol1}")
        assert hist[-1][i]["status"] == 0 and hist[-1][i]["n_components"] == 1
        assert abs(vol1 / vol0 - 1.0) < 0.02            # the droplet keeps its volume
        assert abs(theta - 45.0) < 1.5                    # oriented at 45 degrees
        # finite Re (0.7 and 1.4 here) and the diffuse interface raise D a little
        assert 1.0 < D[i] / d_taylor[i] < 1.25
        # steady: the last three checks agree
        last = [h[i]["D"] for h in hist[-3:]]
        assert max(last) - min(last) < 0.01 * D[i]
    # the slope dD/dCa extrapolated linearly to Ca -> 0 (Re -> 0)
    slope0 = 2.0 * D[0] / CAS[0] - D[1] / CAS[1]
    print(f"slope at Ca -> 0: {slope0:.4f} (Taylor {35.0 / 32.0:.4f})")
    assert abs(slope0 / (35.0 / 32.0) - 1.0) < 0.15


def test_laplace_law_static_spheres():
    """dp = 2 sigma / R for static droplets of radius 10, 12 and 14 (tau 1.25 in
    both phases, G = 0.75, 48^3 boxes, walls at rest): the pressure jump of the
    Shan-Chen bulk pressure times R_eff / 2 is the same sigma for every radius,
    and equals the calibrated sigma the workloads are mapped with."""
    from paper_1411_2181_amd import calibrate, physics
    table = calibrate.calibrate(groups=((0.75, (1.25,)),), precision="fp64")
    (e,) = table["entries"]
    print(f"sigma {e['sigma']:.5f}, spread over radii {e['laplace_spread']:.2%}, "
          f"R_eff {[round(r, 2) for r in e['radii']]}, spurious |u| {e['spurious_umax']:.1e}")
    assert e["usable"] and e["laplace_spread"] < 0.05
    assert e["sigma"] == pytest.approx(physics.sigma_for(1.25, 1.25, 0.75), rel=0.02)
    assert e["spurious_umax"] < 0.05          # Shan-Chen spurious currents at the interface
