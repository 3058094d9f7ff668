"""Host-side measurements used by the calibration and the precision study,
checked on synthetic fields with known answers."""
import math

import numpy as np
import pytest

from paper_1411_2181_amd import calibrate


def _sphere_fields(n, R, rho_in, rho_out):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = n // 2 - 0.5          # centre between the four central nodes the measure averages
    inside = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 < R * R
    rA = np.where(inside, rho_in[0], rho_out[0])
    rB = np.where(inside, rho_in[1], rho_out[1])
    return np.stack([rA, rB]), int(inside.sum())


@pytest.mark.parametrize("R", [8.0, 12.0])
def test_laplace_measure_on_a_sharp_sphere(R):
    G = 0.75
    rho_in, rho_out = (1.0, 0.04), (0.05, 1.02)
    rho, nodes = _sphere_fields(48, R, rho_in, rho_out)
    dp, reff = calibrate.laplace_measure(rho, G)
    P = lambda a, b: (a + b) / 3.0 + G * a * b
    assert dp == pytest.approx(P(*rho_in) - P(*rho_out), rel=1e-12)
    # the volume of a sharp sphere is its node count
    assert reff == pytest.approx((3.0 * nodes / (4.0 * math.pi)) ** (1.0 / 3.0), rel=1e-12)
    assert reff == pytest.approx(R, rel=0.02)


def test_precision_comparison_arithmetic():
    from paper_1411_2181_amd import precision_study as ps
    u64 = np.ones((3, 2, 2, 2))
    u32 = u64.copy()
    u32[0, 0, 0, 0] += 0.3                       # rel. L2 = 0.3 / sqrt(24)

    def run(D, th, m, m0):
        return dict(hist=[[dict(step=100, D=D, theta=th, mass=m, status=0)]], u={100: [u32]},
                    mass0=[m0], seconds=1.0)
    tw = {"fp64": run(0.20, 40.0, (10.0, 5.0), (10.0, 5.0)),
          "fp32": run(0.21, 41.5, (10.001, 4.999), (10.0, 5.0))}
    tw["fp64"]["u"] = {100: [u64]}
    (row,) = ps.compare(tw, 1)
    assert row["precision"] == "fp32"
    assert row["max_dD"] == pytest.approx(0.01) and row["max_dtheta"] == pytest.approx(1.5)
    assert row["u_rel_l2"][100] == pytest.approx(0.3 / math.sqrt(24.0), rel=1e-12)
    drift = row["checkpoints"][0]["mass_drift"]
    assert drift[0] == pytest.approx(1e-4) and drift[1] == pytest.approx(-2e-4)


def _counter_csv(path, rows):
    import csv
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value",
                    "Start_Timestamp", "End_Timestamp"])
        w.writerows(rows)


def test_traffic_table_scaling_and_launch_decoding(tmp_path):
    from paper_1411_2181_amd import profsum
    box = (64, 32, 16)                     # 32x8 tiles, bz = 8: 2 x 4 columns x 2 z blocks
    nodes = 64 * 32 * 16
    wg, items = 16, 512                    # one workgroup of 2 bx by threads per tile
    name = "void lbm::k_step<float, float, 32, 8>(lbm::StepArgs<float, float>)"
    copy = "void at::native::copy_kernel(float)"
    # counters in KiB: the copy reads 1 GiB and writes 1 GiB; FETCH_SIZE reports half
    fetch = [[copy, 1 << 28, 256, "FETCH_SIZE", (1 << 20) / 2, 0, 1000],
             [name, wg * items, items, "FETCH_SIZE", 100.0, 0, 5000],
             [name, wg * items, items, "FETCH_SIZE", 120.0, 0, 7000]]
    write = [[copy, 1 << 28, 256, "WRITE_SIZE", 1 << 20, 0, 1000],
             [name, wg * items, items, "WRITE_SIZE", 200.0, 0, 5000],
             [name, wg * items, items, "WRITE_SIZE", 200.0, 0, 5000]]
    _counter_csv(tmp_path / "f.csv", fetch)
    _counter_csv(tmp_path / "w.csv", write)
    table, scale = profsum.traffic_table(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), box)
    assert scale["fetch"] == pytest.approx(2.0) and scale["write"] == pytest.approx(1.0)
    (key,) = table
    assert key == "32x8x8"
    e = table[key]["k_step"]
    assert e["fetch"] == round(110.0 * 1024 * 2) and e["write"] == 200 * 1024
    assert e["bytes_per_node"] == pytest.approx((220 + 200) * 1024 / nodes, abs=0.01)
    assert e["us"] == pytest.approx(5.5)
