"""Shared helpers of the GPU tests: the bars, the runs through the C-ABI and
the comparison with the oracle."""
import sys

import numpy as np
import pytest

from paper_2204_03756_amd import workloads as W

TOL = {W.FP64: 1e-12, W.FP32W_FP64ACC: 1e-5, W.FP32_KAHAN: 1e-5}
PREC_NAMES = {W.FP64: "fp64", W.FP32W_FP64ACC: "fp32w", W.FP32_KAHAN: "kahan"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load_mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2204_03756_amd import mtpt
    mtpt.load()
    return mtpt


def normwise(m, ref):
    out = []
    for c in range(ref.shape[0]):
        den = np.max(np.abs(ref[c]))
        out.append(float(np.max(np.abs(m[c] - ref[c])) / den) if den > 0 else float(np.max(np.abs(m[c]))))
    return max(out)


def gpu_run(mt, w, steps, chunks=None, nb=None):
    """Masses, positions and stats after the steps; with nb a list, the
    neighbour CSR of the final positions is appended to it."""
    say(f"  gpu: {w.name} n={w.params.n} prec={PREC_NAMES[w.params.precision]} steps={steps}")
    alloc = mt.TorchAllocator("cuda:0")
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        for k in (chunks or [steps]):
            sim.step(k)
        if nb is not None:
            nb.append(sim.neighbors())
        return sim.masses(), sim.positions(), sim.stats()


def oracle_run(oracle, w, steps, **kw):
    return oracle.run(w.params, w.x0, w.m0, steps, **kw)


def check_parity(mt, oracle, w, steps, bitwise_pos=True, nb=False):
    csr = [] if nb else None
    m, x, st = gpu_run(mt, w, steps, nb=csr)
    ref = oracle_run(oracle, w, steps)
    if nb:
        orow, ocol = oracle.neighbors(ref.x, w.params.psi_eff, "kdtree", tens=oracle.tensor_of(w.params))
        assert np.array_equal(csr[0][0], orow) and np.array_equal(csr[0][1], ocol)
    err = normwise(m, ref.m)
    say(f"  {w.name} {PREC_NAMES[w.params.precision]}: normwise {err:.3e}, drift {st['drift']:.3e}, "
        f"pairs/step {st['pairs_last']}")
    assert err <= TOL[w.params.precision]
    if bitwise_pos:
        assert np.array_equal(x, ref.x)
    assert st["pairs_last"] == int(ref.pairs[-1])
    assert st["pairs_total"] == int(ref.pairs.sum())
    assert st["steps_done"] == steps
    for c in range(ref.m.shape[0]):
        # the device's FP64 totals against the oracle's compensated totals,
        # at the path's bar
        assert abs(st["mass_total"][c] - ref.totals[-1, c]) <= \
            TOL[w.params.precision] * max(1.0, abs(ref.totals[-1, c]))
    return m, x, st, ref
