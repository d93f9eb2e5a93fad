"""The no-allocation neighbour export (mtpt_neighbors_static) through the
C-ABI: the same CSR as mtpt_neighbors on two calls in a row (the second on a
smaller sim of the other dimension, so the static scratch holds the first
call's larger contents), bit for bit, and sizes beyond the scratch rejected
before any device work."""
import ctypes as C

import numpy as np
import pytest

from paper_2204_03756_amd import workloads as W

pytestmark = pytest.mark.gpu

_i64p = C.POINTER(C.c_int64)


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2204_03756_amd import mtpt
    mtpt.load()
    return mtpt


def _static_csr(mt, sim, n):
    lib = mt.load()
    row = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64()
    rc = lib.mtpt_neighbors_static(sim.h, row.ctypes.data_as(_i64p), None, 0, C.byref(nnz))
    assert rc == 0, lib.mtpt_last_error()
    col = np.full(max(nnz.value, 1), -7, dtype=np.int64)
    rc = lib.mtpt_neighbors_static(sim.h, row.ctypes.data_as(_i64p), col.ctypes.data_as(_i64p), nnz.value,
                                   C.byref(nnz))
    assert rc == 0, lib.mtpt_last_error()
    return row, col[:nnz.value]


def test_static_export_equals_allocating_export(mt):
    cases = [W.rw2d(n=200_000 + 77, steps=2, precision=W.FP32W_FP64ACC),
             W.rw3d(n=20_000 + 3, steps=2, precision=W.FP64, n_src=20)]
    for w in cases:
        print(f"  static export: {w.name} n={w.params.n}", flush=True)
        with mt.Sim(w.params, w.x0, w.m0, allocator=mt.TorchAllocator("cuda:0")) as sim:
            sim.step(w.steps)
            row, col = sim.neighbors()
            srow, scol = _static_csr(mt, sim, w.params.n)
        assert np.array_equal(row, srow) and np.array_equal(col, scol)
        assert len(col) > w.params.n


def test_static_export_rejects_sizes_beyond_the_scratch(mt):
    # 16 bytes per row of scratch for 5e6 rows exceed the 64 MiB array
    w = W.plain2d(n=5_000_000, steps=1)
    lib = mt.load()
    with mt.Sim(w.params, w.x0, w.m0, allocator=mt.TorchAllocator("cuda:0")) as sim:
        row = np.zeros(w.params.n + 1, dtype=np.int64)
        nnz = C.c_int64()
        rc = lib.mtpt_neighbors_static(sim.h, row.ctypes.data_as(_i64p), None, 0, C.byref(nnz))
        assert rc == mt.MTPT_E_ARG
        assert b"static scratch" in lib.mtpt_last_error()
        # the sim is untouched: the allocating export still works
        r2, _ = sim.neighbors()
        assert r2[-1] > w.params.n
