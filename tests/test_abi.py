"""Host-side checks of the C-ABI library (no GPU needed).

* libmtpt.so loads and exports every function include/mtpt.h declares.
* Parameter validation rejects bad input before any device call.
* The buffer plan sizes what the kernels index.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2204_03756_amd import build as lib_build
from paper_2204_03756_amd import mtpt
from paper_2204_03756_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if lib_build.stale():
        lib_build.build()
    return mtpt.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mtpt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mtpt_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 19
    raw = C.CDLL(mtpt.lib_path())
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    assert lib.mtpt_abi_version() == mtpt.MTPT_ABI_VERSION


def test_params_struct_matches_header():
    text = open(os.path.join(ROOT, "include", "mtpt.h")).read()
    body = text[text.index("typedef struct {\n    uint32_t abi_version"):text.index("} mtpt_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(\w+)(?:\[[0-9]\])?[,;]", body)
    names = [f for f, _ in mtpt.mtpt_params._fields_]
    assert [f for f in fields if f in names] == names


def _call_create(lib, p, x, m):
    h = C.c_void_p()
    f64 = C.POINTER(C.c_double)
    rc = lib.mtpt_create(C.byref(p), x.ctypes.data_as(f64), m.ctypes.data_as(f64), None, None,
                         C.byref(h))
    return rc, h


def test_validation_rejects_bad_params(lib):
    w = W.plain2d(n=100)
    x = np.ascontiguousarray(w.x0)
    m = np.ascontiguousarray(w.m0)
    cases = []
    p = mtpt.make_params(w.params); p.abi_version = 99; cases.append((p, mtpt.MTPT_E_ABI))
    p = mtpt.make_params(w.params); p.dim = 4; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.n = -1; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.n_species = 2; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.precision = 5; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.dt = 0.0; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.d_mt = -1.0; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.d_rw = float("nan"); cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.beta = 1.5; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.hi[1] = p.lo[1]; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.start_step = -3; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.vel[0] = float("inf"); cases.append((p, mtpt.MTPT_E_ARG))
    # dispersion tensor: not symmetric, not positive definite, not finite
    p = mtpt.make_params(w.params); p.disp[0] = 1.0; p.disp[4] = 1.0; p.disp[1] = 0.3; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.disp[0] = 1.0; p.disp[4] = -1.0; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.disp[0] = 1.0; p.disp[4] = 1.0; p.disp[1] = p.disp[3] = 1.0; cases.append((p, mtpt.MTPT_E_ARG))
    p = mtpt.make_params(w.params); p.disp[8] = float("nan"); cases.append((p, mtpt.MTPT_E_ARG))
    for p, code in cases:
        rc, h = _call_create(lib, p, x, m)
        assert rc == code and not h.value
        assert lib.mtpt_last_error().decode()
    # a position outside the box
    xb = x.copy(); xb[7, 1] = w.params.hi[1] + 1e-9
    rc, h = _call_create(lib, mtpt.make_params(w.params), xb, m)
    assert rc == mtpt.MTPT_E_ARG and b"outside" in lib.mtpt_last_error()
    mb = m.copy(); mb[0, 3] = np.inf
    rc, h = _call_create(lib, mtpt.make_params(w.params), x, mb)
    assert rc == mtpt.MTPT_E_ARG


def test_null_handles_are_errors_or_noops(lib):
    assert lib.mtpt_destroy(None) == 0
    assert lib.mtpt_pool_destroy(None) == 0
    assert lib.mtpt_step(None, 1) == mtpt.MTPT_E_ARG
    assert lib.mtpt_masses(None, None) == mtpt.MTPT_E_ARG


def test_plan_bytes_scale_with_n(lib):
    small = mtpt.mtpt_sim_bytes(W.rw2d(n=40_000).params)
    big = W.rw2d(n=400_000).params
    big_b = mtpt.mtpt_sim_bytes(big)
    # FP32 positions, FP64 masses: ~5 position arrays, 2 mass arrays, 6 u32
    # arrays and ~2 u32 per cell per particle
    per = big_b / big.n
    assert 40 < per < 120
    assert big_b > 8 * small
    p64 = W.with_precision(W.rw2d(n=400_000), W.FP64).params
    assert mtpt.mtpt_sim_bytes(p64) > big_b
    # a dispersion tensor stretches the cells along its long axis: fewer,
    # larger cells, so fewer bytes of per-cell tables
    pt = W.replace(big, disp=W.rotated_tensor([4.0, 1.0], [0.3]))
    assert mtpt.mtpt_sim_bytes(pt) < big_b


def test_minimum_tile_count_from_the_environment(lib, monkeypatch):
    # the 1e4-particle plain 2-d sim (2704 cells) has 16 throughput-sized
    # transfer tiles; the default minimum cuts it into at least 256, whose
    # per-tile partial sums (3 x 8 B each) the plan then holds
    p = W.plain2d().params
    monkeypatch.setenv("MTPT_MIN_TILES", "1")
    few = mtpt.mtpt_sim_bytes(p)
    monkeypatch.delenv("MTPT_MIN_TILES")
    dflt = mtpt.mtpt_sim_bytes(p)
    assert dflt > few
    monkeypatch.setenv("MTPT_MIN_TILES", "256")
    assert mtpt.mtpt_sim_bytes(p) == dflt
    # anything but a whole number in [1, 2^20] keeps the default
    for bad in ("", "0", "-4", "abc", "12x", str(2 ** 20 + 1)):
        monkeypatch.setenv("MTPT_MIN_TILES", bad)
        assert mtpt.mtpt_sim_bytes(p) == dflt, bad
    # one tile per cell at most
    monkeypatch.setenv("MTPT_MIN_TILES", str(2 ** 20))
    most = mtpt.mtpt_sim_bytes(p)
    monkeypatch.setenv("MTPT_MIN_TILES", "2704")
    assert mtpt.mtpt_sim_bytes(p) == most > dflt
    # a large sim keeps its throughput tiles
    big = W.rw2d().params
    monkeypatch.setenv("MTPT_MIN_TILES", "1")
    b1 = mtpt.mtpt_sim_bytes(big)
    monkeypatch.delenv("MTPT_MIN_TILES")
    assert mtpt.mtpt_sim_bytes(big) == b1


def test_plan_at_the_largest_n(lib):
    """n = 2^31 - 256, the largest the ABI accepts, plans without overflow
    (cells capped at 2^30 and at ~4 per particle; 64-bit offsets), in 2-d
    and in 3-d with three species; one particle more is refused."""
    nmax = 2 ** 31 - 256
    for dim, ns, prec in ((2, 1, W.FP32W_FP64ACC), (3, 3, W.FP64), (3, 1, W.FP32_KAHAN)):
        L = float(nmax) ** (1.0 / dim)
        hi = [L] * dim + [0.0] * (3 - dim)
        p = W.Params(dim=dim, n=nmax, lo=[0.0, 0.0, 0.0], hi=hi, d_rw=0.3, d_mt=0.7, dt=0.05,
                     n_species=ns, k_react=1.0 if ns == 3 else 0.0, precision=prec)
        b = mtpt.mtpt_sim_bytes(p)
        per = b / nmax
        assert 40 < per < 400, (dim, ns, prec, per)
        half = mtpt.mtpt_sim_bytes(W.replace(p, n=nmax // 2))
        assert 1.8 < b / half < 2.2
        # a box far too large for cells of side psi: the grid is coarsened
        sparse = mtpt.mtpt_sim_bytes(W.replace(p, hi=[1e7] * dim + [0.0] * (3 - dim)))
        assert sparse / nmax < 2 * per
        with pytest.raises(mtpt.MtptError):
            mtpt.mtpt_sim_bytes(W.replace(p, n=nmax + 1))
