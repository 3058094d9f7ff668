"""Host logic of the Ca_cr search (sweep.bisect) against a known threshold:
a stand-in run function marks a run broken iff Ca > Ca_cr(De, lambda, c)."""
import pytest

from paper_1411_2181_amd import sweep

TOL = 0.02


def ca_cr(De, lam, c):
    return 0.17 + 0.02 * De + 0.1 * (lam - 0.75) + 0.2 * (c - 0.5)


def threshold_runner(calls):
    def run(specs):
        calls.append(len(specs))
        return [(sp.Ca > ca_cr(sp.De, sp.lam, sp.c), 0) for sp in specs], 0.0
    return run


def search(lo, hi, De=0.5, lam=0.7, c=0.5, hard=(0.10, 0.26)):
    return sweep.Search(De, lam, c, 24.0, lo, hi, hard_lo=hard[0], hard_hi=hard[1])


@pytest.mark.parametrize("De,lam,c", [(0.0, 0.6, 0.45), (1.0, 0.75, 0.5), (2.0, 0.9, 0.55)])
def test_plain_bisection_brackets_the_threshold(De, lam, c):
    calls = []
    s = search(0.10, 0.26, De, lam, c)
    (s,), _, rounds = sweep.bisect([s], tol=TOL, run=threshold_runner(calls))
    t = ca_cr(De, lam, c)
    assert s.outside == ""
    assert s.lo_ok and s.hi_ok and s.lo <= t < s.hi and s.hi - s.lo <= TOL * 1.000001
    assert abs(s.ca_cr - t) <= TOL / 2 * 1.000001
    assert rounds == len(calls) and s.runs == sum(calls)


def test_threshold_above_and_below_the_window():
    calls = []
    above = search(0.10, 0.20, De=2.0, lam=0.9, c=0.6, hard=(0.10, 0.20))   # ca_cr = 0.265
    below = search(0.10, 0.26, hard=(0.22, 0.26))                              # ca_cr ~ 0.18
    res, _, _ = sweep.bisect([above, below], tol=TOL, run=threshold_runner(calls))
    assert res[0].outside == "above" and res[0].runs == 2      # hi check + speculative midpoint
    # the bottom of the window is taken as stable while the search narrows;
    # once the final bracket rests on it, it is run, breaks, and the search
    # reports the threshold below the window
    assert res[1].outside == "below" and res[1].lo == 0.22


def test_bottom_of_the_window_is_verified_when_the_bracket_rests_on_it():
    # threshold just above the window's bottom: the bracket ends on hard_lo,
    # which is then run once and holds
    t = ca_cr(0.5, 0.7, 0.5)
    calls = []
    s = search(t - 0.005, t + 0.2, hard=(t - 0.005, t + 0.2))
    (s,), _, _ = sweep.bisect([s], tol=TOL, run=threshold_runner(calls))
    assert s.outside == "" and s.lo == pytest.approx(t - 0.005) and s.lo_ok and not s.lo_assumed
    assert s.lo <= t < s.hi and s.hi - s.lo <= TOL * 1.000001


def test_exact_proposal_needs_one_round_and_two_runs():
    t = ca_cr(0.5, 0.7, 0.5)
    calls = []
    s = search(t - TOL / 2, t + TOL / 2)
    (s,), _, rounds = sweep.bisect([s], tol=TOL, run=threshold_runner(calls))
    assert rounds == 1 and s.runs == 2 and s.lo <= t < s.hi


@pytest.mark.parametrize("offset", [-0.05, -0.025, 0.025, 0.05])
def test_wrong_proposal_falls_back_outward(offset):
    t = ca_cr(0.5, 0.7, 0.5)
    calls = []
    c = t + offset
    s = search(c - TOL / 2, c + TOL / 2)
    (s,), _, _ = sweep.bisect([s], tol=TOL, run=threshold_runner(calls))
    assert s.outside == "" and s.lo <= t < s.hi and s.hi - s.lo <= TOL * 1.000001


def test_failed_run_ends_the_search():
    def run(specs):
        return [(False, -5) for _ in specs], 0.0
    s = search(0.10, 0.26)
    (s,), _, _ = sweep.bisect([s], tol=TOL, run=run)
    assert s.done and s.outside == "failed"


def test_no_speculation_checks_the_top_alone():
    calls = []
    above = search(0.10, 0.20, De=2.0, lam=0.9, c=0.6, hard=(0.10, 0.20))   # ca_cr = 0.265
    above.speculate = False
    (above,), _, rounds = sweep.bisect([above], tol=TOL, run=threshold_runner(calls))
    assert above.outside == "above" and above.runs == 1 and rounds == 1
    # a wrong "above" prediction goes on as plain bisection
    inside = search(0.10, 0.26)
    inside.speculate = False
    (inside,), _, _ = sweep.bisect([inside], tol=TOL, run=threshold_runner([]))
    t = ca_cr(0.5, 0.7, 0.5)
    assert inside.outside == "" and inside.lo <= t < inside.hi and inside.hi - inside.lo <= TOL * 1.000001


def test_updates_are_accumulated():
    def run(specs):
        return [(sp.Ca > 0.18, 0, 1000) for sp in specs], 0.0
    s = search(0.10, 0.26)
    (s,), _, _ = sweep.bisect([s], tol=TOL, run=run)
    assert s.updates == 1000 * s.runs


def test_runs_carry_the_search_polymer_parameters():
    seen = []

    def run(specs):
        seen.extend((sp.L2, sp.fraction) for sp in specs)
        return [(sp.Ca > 0.18, 0) for sp in specs], 0.0
    s = sweep.Search(1.0, 4 / 3, 0.5, 24.0, 0.10, 0.26, hard_lo=0.10, hard_hi=0.26, L2=400.0, fraction=0.2)
    sweep.bisect([s], tol=TOL, run=run)
    assert seen and all(v == (400.0, 0.2) for v in seen)


def test_lattice_runner_logs_each_round(monkeypatch):
    class Res:
        def __init__(self, sp):
            self.broken, self.status, self.steps = sp.Ca > 0.18, 0, 100
            self.params = dict(nx=4, ny=5, nz=6)

    def fake_simulate(specs, precision, **kw):
        return [Res(sp) for sp in specs], 0.5 * len(specs)
    monkeypatch.setattr(sweep, "simulate", fake_simulate)
    run = sweep.lattice_runner("fp16s")
    (s,), secs, rounds = sweep.bisect([search(0.10, 0.26)], tol=TOL, run=run)
    assert len(run.rounds) == rounds
    assert sum(r[0] for r in run.rounds) == s.runs
    assert all(r[1] == r[0] * 100 * 120 and r[2] == 0.5 * r[0] for r in run.rounds)
    assert secs == sum(r[2] for r in run.rounds)


def test_fp64_reference_search_compares_brackets(monkeypatch, tmp_path):
    import json
    import types
    from paper_1411_2181_amd import study

    class Res:
        def __init__(self, sp):
            self.broken, self.status, self.steps = sp.Ca > 0.185, 0, 100
            self.params = dict(nx=4, ny=5, nz=6)

    def fake_simulate(specs, precision, **kw):
        assert precision == "fp64" and len(specs) == 1      # one run at a time
        return [Res(sp) for sp in specs], 2.0
    monkeypatch.setattr(sweep, "simulate", fake_simulate)
    # the batched search's rows for the same triples: the first agrees, the second not
    qs = study.query_searches(2)
    rows = []
    for k, q in enumerate(qs):
        s, _, _ = sweep.bisect([sweep.Search(q["De"], q["lam"], q["c"], q["R"], *study.window(q),
                                             hard_lo=study.window(q)[0], hard_hi=study.window(q)[1])],
                               tol=study.TOL, run=lambda specs: ([(sp.Ca > 0.185, 0) for sp in specs], 0.0))
        lo, hi = (s[0].lo, s[0].hi) if k == 0 else (s[0].lo + 0.01, s[0].hi + 0.01)
        rows.append(dict(plain=dict(ca_cr=0.5 * (lo + hi), bracket=[lo, hi], outside="")))
    ref = tmp_path / "search.json"
    ref.write_text(json.dumps(dict(search=dict(rows=rows))))
    out = tmp_path / "fp64.json"
    study.cmd_fp64(types.SimpleNamespace(out=str(out), queries=2, compare=str(ref)), lambda m: None)
    d = json.loads(out.read_text())
    assert [r["same_bracket"] for r in d["rows"]] == [True, False]
    assert d["seconds"] == 2.0 * d["runs"]
    assert abs(d["sweeps_per_hour"] - 2 / d["seconds"] * 3600) < 1e-9


def _logistic_surrogate(c0, s):
    """A Surrogate whose break-up probability is a known logistic in Ca
    (the proposal logic only, no network)."""
    import numpy as np
    from paper_1411_2181_amd.surrogate import Surrogate
    sg = Surrogate.__new__(Surrogate)
    sg.breakup_probability = lambda Ca, *a, **k: 1.0 / (1.0 + np.exp(-(np.asarray(Ca) - c0) / s))
    return sg


@pytest.mark.parametrize("c0,s", [(0.18, 0.002), (0.18, 0.02), (0.21, 0.01)])
def test_proposal_brackets_the_predicted_boundary(c0, s):
    import math
    lo, hi = 0.12, 0.26
    b = _logistic_surrogate(c0, s).propose(1.0, 1.0, 0.5, lo, hi, tol=TOL, grid=4096)
    mid, half = 0.5 * (b[0] + b[1]), 0.5 * (b[1] - b[0])
    want_half = max(TOL, s * math.log(3.0))     # quartiles of a logistic: c0 -+ s ln 3
    if c0 + want_half <= hi and c0 - want_half >= lo:
        assert mid == pytest.approx(c0, abs=1e-4) and half == pytest.approx(want_half, abs=1e-4)
    assert lo <= b[0] < c0 < b[1] <= hi


def test_proposal_edges_of_the_window():
    lo, hi = 0.12, 0.26
    assert _logistic_surrogate(0.40, 0.005).propose(1.0, 1.0, 0.5, lo, hi, tol=TOL) is None
    b = _logistic_surrogate(0.05, 0.005).propose(1.0, 1.0, 0.5, lo, hi, tol=TOL)
    assert b[0] == lo and b[1] == pytest.approx(lo + TOL, abs=1e-9)       # breaks everywhere
    b = _logistic_surrogate(0.255, 0.001).propose(1.0, 1.0, 0.5, lo, hi, tol=TOL)
    assert b[1] == hi and b[0] == pytest.approx(0.255 - TOL, abs=1e-3)    # clipped at the top


def test_still_elongating_reads_the_length_history():
    h = lambda steps_lp: [(s, 0.0, 45.0, lp, 1) for s, lp in steps_lp]
    # stretching over the last 4000 steps
    assert sweep.still_elongating(h([(12000, 140), (14000, 142), (16000, 144)]))
    # relaxing or holding its length
    assert not sweep.still_elongating(h([(12000, 98), (14000, 94), (16000, 90)]))
    assert not sweep.still_elongating(h([(12000, 120), (14000, 120), (16000, 120)]))
    # compares with the latest check at or before 4000 steps back (11000, not 12500)
    assert not sweep.still_elongating(h([(11000, 150), (12500, 100), (16000, 110)]))
    assert sweep.still_elongating(h([(11000, 100), (12500, 150), (16000, 110)]))
    assert not sweep.still_elongating(h([(13000, 100), (16000, 110)]))      # no check far enough back
    assert not sweep.still_elongating([])


def test_scan_report(monkeypatch, tmp_path):
    import json
    import types
    from paper_1411_2181_amd import study

    def fake_simulate(specs, precision, t_end=None, every=500, **kw):
        out = []
        for sp in specs:
            r = sweep.RunResult(sp, dict(nx=4, ny=5, nz=6), dict(tau_em=50.0))
            br = sp.Ca > 0.2
            r.history = [(s, 0.1, 45.0, 48.0 + s / 1000.0, 2 if (br and s == 2000) else 1)
                         for s in range(every, (2000 if br else t_end) + 1, every)]
            r.broken, r.step_break = br, (2000 if br else -1)
            r.pieces, r.steps = ([300, 300] if br else []), r.history[-1][0]
            out.append(r)
        return out, 1.0
    monkeypatch.setattr(sweep, "simulate", fake_simulate)
    out = tmp_path / "scan.json"
    args = types.SimpleNamespace(out=str(out), De=1.0, c=0.5, fraction=0.2, L2=100.0, R=24.0,
                                 ca="0.15,0.25", t_end=4000, every=500, precision="fp32")
    study.cmd_scan(args, lambda m: None)
    d = json.loads(out.read_text())
    assert d["lam"] == pytest.approx(1.0) and d["fraction"] == 0.2 and d["t_end"] == 4000
    stable, broken = d["rows"]
    assert not stable["broken"] and stable["t_break_over_tau_em"] is None
    assert broken["broken"] and broken["step_break"] == 2000 and broken["daughter_nodes"] == [300, 300]
    assert broken["t_break_over_tau_em"] == pytest.approx(40.0)
    assert stable["Lp_max_over_2R"] == pytest.approx((48.0 + 4.0) / 48.0)


def test_modes_report_maps_each_mode(monkeypatch, tmp_path):
    """The Newtonian / droplet- / matrix-viscoelastic comparison builds one run
    per mode, Ca and De with lambda = 1 and each mode's matrix solvent tau; the
    lattice parameters of every run lie in the calibrated window."""
    import json
    import types
    from paper_1411_2181_amd import physics, study

    def fake_simulate(specs, precision, t_end=None, every=500, **kw):
        out = []
        for sp in specs:
            p, info = sweep.lattice(sp)
            r = sweep.RunResult(sp, p, info)
            r.history = [(every, 0.1, 45.0, 2 * sp.R, 1)]
            r.steps = every
            out.append(r)
        return out, 1.0
    monkeypatch.setattr(sweep, "simulate", fake_simulate)
    out = tmp_path / "modes.json"
    args = types.SimpleNamespace(out=str(out), c=0.78, R=24.0, ca="0.16,0.24", De="0.2,2",
                                 fraction=0.4, L2=100.0, t_end=1000, extend_to=0, every=500,
                                 precision="fp32")
    study.cmd_modes(args, lambda m: None)
    d = json.loads(out.read_text())
    rows = d["rows"]
    assert [r["mode"] for r in rows[:5]] == ["N", "DV", "MV", "DV", "MV"] and len(rows) == 10
    for r in rows:
        tA, tB = r["tau"]
        physics.sigma_for(tA, tB)                  # raises outside the calibrated window
        assert r["u_wall"] <= sweep.U_MAX * (1 + 1e-9)
        assert tB == pytest.approx(study.MODE_TAU_MATRIX[r["mode"]])   # the matrix is B
        assert r["Lp_max_over_2R"] == pytest.approx(1.0)


def test_paper_scale_mapping_and_bracket():
    """Host logic of the paper-scale Ca_cr driver: lambda on the total
    viscosities with the polymer fraction in the right phase, the wall speed
    from Ca, and the bracket from a scan."""
    from paper_1411_2181_amd import paper_scale as P
    eta = P.eta_of(6.0)
    assert abs(P.eta_of(P.tau_of(0.7)) - 0.7) < 1e-15
    ta, tb, ea, eb = P.viscosities("DV", eta, 1.0, 0.4)
    assert tb == 6.0 and eb == 0.0 and abs(P.eta_of(ta) + ea - eta) < 1e-12
    ta, tb, ea, eb = P.viscosities("MV", eta, 1.0, 0.4)
    assert ta == 6.0 and ea == 0.0 and abs(P.eta_of(tb) + eb - eta) < 1e-12
    p, info = P.run_params("N", 0.3, 32.0, 0.52, 2.0, 1.0, 0.4, 100.0, eta, 1.0, 0.14, 0.75, 0.19)
    assert p["nz"] == 123 and p["tau_minus"] == (1.0, 1.0)
    assert abs(p["u_wall"] - 0.3 * 0.14 / (eta * 32.0) * 123 / 2.0) < 1e-15
    rows = [dict(Ca=0.3, broken=False, status=0), dict(Ca=0.34, broken=False, status=0),
            dict(Ca=0.38, broken=True, status=0), dict(Ca=0.42, broken=True, status=0)]
    assert P.bracket(rows) == (0.34, 0.38)
    assert P.bracket(rows[:2]) == (0.34, None)
    assert P.bracket(rows[2:]) == (None, 0.38)


def test_paper_scale_shape_criterion():
    """A run is steady when L_p moved by at most 2 % over the last 10 tau_em;
    the shape bracket counts broken or still-stretching runs as
    super-critical."""
    from paper_1411_2181_amd import paper_scale as P
    tem = 100.0
    flat = [dict(step=s, Lp_over_2R=v) for s, v in ((0, 1.0), (500, 1.74), (1000, 1.75), (1500, 1.76))]
    grow = [dict(step=s, Lp_over_2R=v) for s, v in ((0, 1.0), (500, 1.5), (1000, 2.0), (1500, 2.5))]
    assert P.steady(flat, tem) and not P.steady(grow, tem)
    assert not P.steady(flat[:1], tem)            # no check a window earlier
    rows = [dict(mode="N", Ca=0.3, broken=False, steady=True, status=0, Re=0.4),
            dict(mode="N", Ca=0.34, broken=False, steady=False, status=0, Re=0.45),
            dict(mode="N", Ca=0.38, broken=True, steady=False, status=0, Re=0.5)]
    b = P.brackets_of(rows, ["N"])["N"]
    assert (b["breakup"]["Ca_cr_lo"], b["breakup"]["Ca_cr_hi"]) == (0.34, 0.38)
    assert (b["shape"]["Ca_cr_lo"], b["shape"]["Ca_cr_hi"]) == (0.3, 0.34)
    assert b["shape"]["Re"] == [0.4, 0.45]


def test_paper_scale_combines_scans(tmp_path):
    """--combine merges the rows of several scans of one set-up and brackets
    them together (here: a stable and a broken Ca from two scans)."""
    import json
    from paper_1411_2181_amd import paper_scale as P
    base = dict(R=32.0, c=0.52, tau_plus_matrix=6.0, tau_minus=1.25, seconds=1.0)
    hist = [dict(step=s, Lp_over_2R=2.0) for s in (0, 2000, 4000)]
    a = dict(base, sigma={"N": dict(sigma=0.16, laplace_residual=0.005)},
             rows=[dict(mode="N", Ca=0.30, broken=False, steady=True, status=0, Re=0.43, history=hist)])
    b = dict(base, sigma={"N": dict(sigma=0.16, laplace_residual=0.005)},
             rows=[dict(mode="N", Ca=0.34, broken=True, steady=False, status=0, Re=0.48, history=hist)])
    pa, pb, out = tmp_path / "a.json", tmp_path / "b.json", tmp_path / "out.json"
    pa.write_text(json.dumps(a))
    pb.write_text(json.dumps(b))
    assert P.main([str(out), "--combine", f"{pa},{pb}"]) == 0
    d = json.loads(out.read_text())
    assert [r["Ca"] for r in d["rows"]] == [0.30, 0.34]
    br = d["brackets"]["N"]["breakup"]
    assert (br["Ca_cr_lo"], br["Ca_cr_hi"], br["Re"]) == (0.30, 0.34, [0.43, 0.48])
    assert "seconds" not in d and d["tau_minus"] == 1.25
