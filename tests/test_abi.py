"""CPU checks of the C ABI: the library loads, exports every function that
include/*.h declares, and rejects invalid parameter sets on the host before
touching any device."""
import ctypes
import glob
import os
import re

import pytest

import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b((?:lbm|sg)_\w+)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_1411_2181_amd import lbmve
    if not os.path.exists(lbmve.LIB_PATH):
        pytest.skip("library not built")
    return lbmve.lib()


def test_header_declares_functions():
    names = _declared_functions()
    for must in ("lbm_init", "lbm_step", "lbm_observe", "lbm_export", "lbm_import",
                 "lbm_batch_init", "lbm_batch_step", "lbm_batch_observe"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror(L):
    from paper_1411_2181_amd import lbmve
    assert lbmve.strerror(0) == "ok"
    assert "invalid" in lbmve.strerror(-1)


def _ws(L, d, precision="fp64"):
    from paper_1411_2181_amd import lbmve
    p = lbmve.make_params(d, precision)
    n = ctypes.c_size_t()
    code = L.lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    return code, n.value


@pytest.mark.parametrize("bad", [
    dict(nx=2), dict(nz=2), dict(tau=(0.5, 1.0)), dict(tau=(1.0, 0.3)),
    dict(u_wall=0.25), dict(radius=16.0), dict(radius=-1.0), dict(rho_minor=0.0),
    dict(eta_P=(0.1, 0.1)), dict(eta_P=(0.1, 0.0), L2=(3.0, 100.0)),
    dict(eta_P=(0.1, 0.0), tau_P=(0.0, 1.0)), dict(chi_lo=0.5, chi_hi=0.4),
    dict(G=float("nan")),
])
def test_invalid_parameters_rejected_on_host(L, bad):
    from paper_1411_2181_amd import lbmve
    d = WL.base_params(**bad)
    assert lbmve.validate(d) == lbmve.LBM_EINVAL
    code, _ = _ws(L, d)
    assert code == lbmve.LBM_EINVAL


def test_valid_parameters_and_workspace_size(L):
    from paper_1411_2181_amd import lbmve
    d = WL.small_droplet_viscoelastic()
    assert lbmve.validate(d) == 0
    n = 32 ** 3
    c64, b64 = _ws(L, d, "fp64")
    c32, b32 = _ws(L, d, "fp32")
    c16, b16 = _ws(L, d, "fp16s")
    assert c64 == c32 == c16 == 0
    # two copies of 38 populations at least
    assert b64 >= 2 * 38 * 8 * n and b32 >= 2 * 38 * 4 * n and b16 >= 2 * 38 * 2 * n
    assert b64 > b32 > b16
    bad = lbmve.make_params(d, "fp64")
    bad.precision = 7
    assert L.lbm_validate(ctypes.byref(bad)) == lbmve.LBM_EINVAL


def test_population_array_must_fit_32bit_offsets(L):
    """The step kernel addresses the population arrays of one run in groups of
    four directions, with 32-bit byte offsets from a group's base: four arrays
    must span less than 4 GiB.  1024 x 1024 x 200 nodes (4 x 0.84 GB in FP32)
    fit in FP32 and FP16 but not in FP64; 1024 x 1024 x 300 only in FP16."""
    from paper_1411_2181_amd import lbmve
    d = WL.base_params(nx=1024, ny=1024, nz=200, radius=8.0)
    assert L.lbm_validate(ctypes.byref(lbmve.make_params(d, "fp32"))) == 0
    assert L.lbm_validate(ctypes.byref(lbmve.make_params(d, "fp16s"))) == 0
    assert L.lbm_validate(ctypes.byref(lbmve.make_params(d, "fp64"))) == lbmve.LBM_EINVAL
    d = WL.base_params(nx=1024, ny=1024, nz=300, radius=8.0)
    assert L.lbm_validate(ctypes.byref(lbmve.make_params(d, "fp32"))) == lbmve.LBM_EINVAL
    assert L.lbm_validate(ctypes.byref(lbmve.make_params(d, "fp16s"))) == 0


def test_batch_requires_one_precision(L):
    from paper_1411_2181_amd import lbmve
    a = lbmve.make_params(WL.small_newtonian(), "fp32")
    b = lbmve.make_params(WL.small_newtonian(), "fp64")
    arr = (lbmve.LbmParams * 2)(a, b)
    n = ctypes.c_size_t()
    assert L.lbm_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == lbmve.LBM_EINVAL
    arr = (lbmve.LbmParams * 2)(a, a)
    assert L.lbm_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == 0
    assert L.lbm_batch_workspace_bytes(arr, 0, ctypes.byref(n)) == lbmve.LBM_EINVAL


def test_null_arguments_rejected(L):
    from paper_1411_2181_amd import lbmve
    assert L.lbm_step(None, 1) == lbmve.LBM_EINVAL
    assert L.lbm_observe(None, 0, None) == lbmve.LBM_EINVAL
    assert L.lbm_export(None, 0, None, 0) == lbmve.LBM_EINVAL
    assert L.lbm_batch_nruns(None) == 0
    n = ctypes.c_size_t()
    assert L.lbm_batch_state_bytes(None, 0, ctypes.byref(n)) == lbmve.LBM_EINVAL
    assert L.lbm_batch_save_state(None, 0, None, 0) == lbmve.LBM_EINVAL
    assert L.lbm_batch_load_state(None, 0, None, 0) == lbmve.LBM_EINVAL
    p = lbmve.make_params(WL.small_newtonian())
    out = ctypes.c_void_p()
    # no workspace -> rejected before any device call
    assert L.lbm_init(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == lbmve.LBM_EINVAL


def test_init_noise_amplitude_is_validated(L):
    """The seeded initial density noise takes a relative amplitude in [0, 0.1)."""
    from paper_1411_2181_amd import lbmve
    d = WL.small_droplet_viscoelastic()
    for a, ok in ((0.0, True), (0.01, True), (0.099, True), (0.1, False), (-0.01, False),
                  (float("nan"), False)):
        p = lbmve.make_params(dict(d, seed=2**64 - 1, init_noise=a), "fp64")
        assert (L.lbm_validate(ctypes.byref(p)) == 0) == ok, a


def test_tau_minus_is_validated(L):
    """The odd-moment relaxation time is 0 (BGK) or a finite value above 1/2."""
    from paper_1411_2181_amd import lbmve
    d = WL.small_droplet_viscoelastic()
    for tm, ok in (((0.0, 0.0), True), ((1.25, 0.0), True), ((0.51, 3.0), True),
                   ((0.5, 1.0), False), ((1.0, -1.0), False), ((float("nan"), 1.0), False),
                   ((1.0, float("inf")), False)):
        p = lbmve.make_params(dict(d, tau_minus=tm), "fp32")
        assert (L.lbm_validate(ctypes.byref(p)) == 0) == ok, tm
