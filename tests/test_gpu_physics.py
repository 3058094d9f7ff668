"""Physics of the scheme on the GPU FP64 path (which matches the CPU oracle to
1e-10 in the parity tests; the same runs on the oracle would take about half
an hour each).

Taylor's small-deformation law (the paper's Introduction cites Taylor for
the deformation measure D; the formula is Taylor's, not printed in the
paper): a droplet in simple shear at small Ca deforms to
D = Ca (19 lambda + 16)/(16 lambda + 16), oriented at 45 degrees.  Between
walls the deformation is larger; Shapira and Haber's first-order correction
for a droplet at mid-gap multiplies it by
1 + 5.6993 (1 + 2.5 lambda)/(1 + lambda) (R/d)^3, d = W/2 the distance from
the droplet centre to a wall.

All solvents relax with tau = 1.24: with the velocity-shift forcing the
coexisting densities depend on tau, and a small droplet next to a matrix of
the same tau swells below tau ~ 1.24 and dissolves above it, which moves its
effective Ca; at 1.24 its volume holds, and a droplet whose tau differs from
the matrix's swells or dissolves.  The viscosity ratios 2 and 0.5 are
therefore made with a polymer at negligible Weissenberg number
(Oldroyd-B limit, De = tau_P gamma_dot = 0.02, polymer fraction 0.5): in the
droplet for lambda = 2, in the matrix for lambda = 0.5.  There the polymer
stress is eta_P times the shear rate (Eq. (6) with Wi -> 0), so the phase
behaves as a Newtonian fluid of viscosity eta_s + eta_P.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

R = 12.0
BOX = (144, 72, 96)          # 2R/W = 0.25
TAU = 1.24
CAS = (0.025, 0.05)
LAMBDAS = {0.5: "MV", 1.0: "N", 2.0: "DV"}


def wall_factor(lam, R=R, W=BOX[2]):
    return 1.0 + 5.6993 * (1.0 + 2.5 * lam) / (1.0 + lam) * (R / (0.5 * W)) ** 3


@pytest.fixture(scope="module")
def taylor_runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2181_amd import lbmve, physics
    runs, keys = [], []
    for lam, phase in LAMBDAS.items():
        for ca in CAS:
            if phase == "N":
                p, _ = physics.lattice_params(*BOX, R=R, Ca=ca, De=0.0, lam=lam, phase="N",
                                              tau_matrix=TAU, u_max=0.15)
            else:
                p, _ = physics.lattice_params(*BOX, R=R, Ca=ca, De=0.02, lam=lam, phase=phase,
                                              L2=1e6, fraction=0.5, tau_matrix=TAU, u_max=0.15)
            assert abs(p["tau"][0] - TAU) < 1e-12 and abs(p["tau"][1] - TAU) < 1e-12
            runs.append(p)
            keys.append((lam, ca))
    print(f"case Taylor: {len(runs)} runs of {BOX}, 12000 steps, FP64", flush=True)
    b = lbmve.Batch(runs, "fp64")
    hist = []
    for _ in range(12):
        b.step(1000)
        hist.append(b.observe(components=True))
    torch.cuda.synchronize()
    b.close()
    return keys, hist


@pytest.mark.timeout(900)
@pytest.mark.parametrize("lam", sorted(LAMBDAS))
def test_taylor_small_deformation(taylor_runs, lam):
    keys, hist = taylor_runs
    idx = [i for i, k in enumerate(keys) if k[0] == lam]
    slope_t = (19.0 * lam + 16.0) / (16.0 * lam + 16.0)
    D = []
    for i in idx:
        ca = keys[i][1]
        d_taylor = ca * slope_t
        d_wall = d_taylor * wall_factor(lam)
        Di = float(np.mean([h[i]["D"] for h in hist[-3:]]))
        D.append(Di)
        vol0, vol1 = hist[0][i]["piece_nodes"][0], hist[-1][i]["piece_nodes"][0]
        theta = hist[-1][i]["theta_deg"]
        print(f"lambda {lam} Ca {ca}: D {Di:.4f} (Taylor {d_taylor:.4f}, ratio "
              f"{Di / d_taylor:.3f}; wall-corrected {d_wall:.4f}, ratio {Di / d_wall:.3f}), "
              f"theta {theta:.2f}, droplet nodes {vol0} -> {vol1}", flush=True)
        assert hist[-1][i]["status"] == 0 and hist[-1][i]["n_components"] == 1
        assert abs(vol1 / vol0 - 1.0) < 0.02            # the droplet keeps its volume
        assert abs(theta - 45.0) < 3.0                    # oriented near 45 degrees
        # Taylor's law with the confinement correction, per Ca, within 15 %
        # (finite Re 0.3-1.4 and the diffuse interface remain)
        assert abs(Di / d_wall - 1.0) < 0.15
        # steady: the last three checks agree
        last = [h[i]["D"] for h in hist[-3:]]
        assert max(last) - min(last) < 0.01 * Di
    # the slope dD/dCa extrapolated linearly to Ca -> 0 (Re -> 0) lies
    # between the unbounded and the wall-corrected slopes (within 15 %)
    slope0 = 2.0 * D[0] / CAS[0] - D[1] / CAS[1]
    print(f"lambda {lam}: slope at Ca -> 0 {slope0:.4f} (Taylor {slope_t:.4f}, "
          f"wall-corrected {slope_t * wall_factor(lam):.4f})")
    assert slope_t * 0.85 < slope0 < slope_t * wall_factor(lam) * 1.15


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
