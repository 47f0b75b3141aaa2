"""pks_filter_smooth_noalloc (workspace in a static device array) against
pks_filter_smooth (caller workspace), through the C ABI: two calls in a row,
the second with a smaller input, in both precisions; outputs bitwise equal to
the workspace entry point's and within the tolerance of the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1905_13002_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-4}


@pytest.fixture(scope="module")
def pks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_13002_amd import pks as mod
    return mod


def _noalloc(pks, dm, y, prec):
    T, nx = y.shape[0], dm.nx
    rdt = torch.float64 if prec == "fp64" else torch.float32
    outs = [torch.full(s, float("nan"), dtype=rdt, device="cuda") for s in ((T, nx), (T, nx, nx)) * 2]
    st = dm.struct()
    rc = pks.lib.pks_filter_smooth_noalloc(ctypes.byref(st), T, pks._ptr(y), *[pks._ptr(o) for o in outs],
                                           pks._prec(prec), pks._stream())
    pks._check(rc)
    return outs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_workspace_entry_point(pks, prec):
    rdt = torch.float64 if prec == "fp64" else torch.float32
    for T in (262144, 1000):                     # the second call is smaller
        w = wl.workload(1, T=T)
        dm = pks.to_device(w.model)
        y = torch.as_tensor(w.y).to("cuda", rdt)
        got = _noalloc(pks, dm, y, prec)
        ref = pks.filter_smooth(dm, y, prec)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), (prec, T)
        yo = w.y if prec == "fp64" else w.y.astype(np.float32).astype(np.float64)
        o = oracle.kf_rts(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0, w.model.P0, yo)
        for k, a in zip(("m", "P", "ms", "Ps"), got):
            assert wl.max_rel_err(a.double().cpu().numpy(), o[k]) <= TOL[prec], (prec, T, k)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_register_path(pks, prec):
    """nx = 16 (register-resident kernels, whose combined call also keeps
    every step's smoothing element in the scratch): two calls in a row, the
    second smaller, bitwise equal to the workspace entry point."""
    rdt = torch.float64 if prec == "fp64" else torch.float32
    for T in (3000, 1000):
        w = wl.workload(3, T=T)
        dm = pks.to_device(w.model)
        y = torch.as_tensor(w.y).to("cuda", rdt)
        got = _noalloc(pks, dm, y, prec)
        ref = pks.filter_smooth(dm, y, prec)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), (prec, T)


def test_noalloc_rejects_problems_beyond_the_scratch(pks):
    w = wl.workload(1, T=8)
    dm = pks.to_device(w.model)
    T = 1 << 20                                   # needs ~107 MiB in FP64
    assert pks.lib.pks_workspace_bytes(4, 2, T, 1, 0) > pks.lib.pks_noalloc_scratch_bytes()
    st = dm.struct()
    rc = pks.lib.pks_filter_smooth_noalloc(ctypes.byref(st), T, None, None, None, None, None, 0, pks._stream())
    assert rc == pks.PKS_E_UNSUPPORTED
    assert b"static scratch" in pks.lib.pks_last_error()
