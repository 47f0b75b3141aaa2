"""Debug mode with NaN-filled workspaces (pks_set_debug_poison).

With the mode on, every call first fills the floating-point regions of its
workspace with NaN.  Every path must then give bitwise the results it gives
with the mode off: no kernel reads workspace memory that the same call has
not written first (a read of stale workspace data would turn into NaN).
"""
import numpy as np
import pytest

from paper_1905_13002_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PATTERN = np.uint64(0xFFF80000FFF80000)


@pytest.fixture(scope="module")
def pks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_13002_amd import pks as mod
    mod.set_debug_poison(False)
    yield mod
    mod.set_debug_poison(False)


def bits(t):
    t = t.contiguous()
    return t.view(torch.int64 if t.element_size() == 8 else torch.int32)


def same_with_and_without(pks, run):
    """run() -> tuple of output tensors (None entries skipped)."""
    pks.set_debug_poison(False)
    ref = [None if t is None else t.clone() for t in run()]
    torch.cuda.synchronize()
    pks.set_debug_poison(True)
    try:
        out = run()
        torch.cuda.synchronize()
    finally:
        pks.set_debug_poison(False)
    for i, (r, o) in enumerate(zip(ref, out)):
        if r is None:
            continue
        assert not torch.isnan(o).any(), "output %d holds NaN with the workspace filled" % i
        assert torch.equal(bits(r), bits(o)), "output %d differs with the workspace filled" % i


def dev(w, prec):
    return torch.as_tensor(w.y).to("cuda", torch.float64 if prec == "fp64" else torch.float32)


def test_switch_and_fill(pks):
    """The switch round-trips and a call really fills its workspace."""
    w = wl.workload(1, T=300)
    dm = pks.to_device(w.model)
    ws = pks.workspace(4, 2, 300)
    pks.set_debug_poison(True)
    try:
        assert pks.debug_poison()
        pks.filter(dm, dev(w, "fp64"), "fp64", ws=ws)
        torch.cuda.synchronize()
    finally:
        pks.set_debug_poison(False)
    assert not pks.debug_poison()
    words = ws.cpu().numpy()[: ws.numel() // 8 * 8].view(np.uint64)
    # the filter alone leaves the likelihood's arrays untouched: still filled
    assert np.count_nonzero(words == PATTERN) > 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_sequence(pks, prec):
    w = wl.workload(2, T=40000)
    dm = pks.to_device(w.model)
    y = dev(w, prec)
    same_with_and_without(pks, lambda: pks.filter_smooth(dm, y, prec))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_filter_then_smooth_and_loglik(pks, prec):
    """Separate filter, smoother and likelihood calls, each with its own fill."""
    w = wl.workload(2, T=20000)
    dm = pks.to_device(w.model)
    y = dev(w, prec)

    def run():
        m, P = pks.filter(dm, y, prec)
        ms, Ps = pks.smooth(dm, m, P, prec)
        ll, tot = pks.loglik(dm, y, m, P, prec, cumulative=True)
        return m, P, ms, Ps, ll, tot
    same_with_and_without(pks, run)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_per_sequence_models(pks, prec):
    w = wl.workload(4, B=64, T=600)
    dm = pks.to_device(w.model, per_sequence=True)
    y = dev(w, prec)
    off = torch.as_tensor(w.offsets).cuda()

    def run():
        m, P = pks.filter_batched(dm, off, y, prec)
        ms, Ps = pks.smooth_batched(dm, off, m, P, prec)
        ll, tot = pks.loglik_batched(dm, off, y, m, P, prec)
        return m, P, ms, Ps, ll, tot
    same_with_and_without(pks, run)


def test_plan_captured_with_fill(pks):
    """A plan captured while the mode is on fills its workspace at every
    launch; its results equal the eager results without the fill."""
    w = wl.workload(4, B=32, T=500)
    dm = pks.to_device(w.model, per_sequence=True)
    y = dev(w, "fp64")
    off = torch.as_tensor(w.offsets).cuda()
    m, P = pks.filter_batched(dm, off, y, "fp64")
    ms, Ps = pks.smooth_batched(dm, off, m, P, "fp64")
    torch.cuda.synchronize()
    pks.set_debug_poison(True)
    try:
        plan = pks.Plan(dm, y, off, "fp64")
    finally:
        pks.set_debug_poison(False)
    for _ in range(2):
        out = [t.clone() for t in plan.launch()]
        torch.cuda.synchronize()
        for r, o in zip((m, P, ms, Ps), out):
            assert torch.equal(bits(r), bits(o))
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_time_varying(pks, prec):
    w = wl.workload(6, T=10000)
    dm = pks.to_device(w.model, time_varying=True)
    y = dev(w, prec)

    def run():
        m, P, ms, Ps = pks.filter_smooth(dm, y, prec)
        ll, tot = pks.loglik(dm, y, m, P, prec)
        return m, P, ms, Ps, ll, tot
    same_with_and_without(pks, run)


@pytest.mark.parametrize("nx,ny,T", [(16, 8, 700), (64, 32, 70)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_states(pks, nx, ny, T, prec):
    """Large states: block elements and arenas in the workspace."""
    model = wl.random_stable_model(nx, ny, wl.rng_for(900, nx))
    w = wl.single_sequence(model, T, seed=nx)
    dm = pks.to_device(w.model)
    y = dev(w, prec)
    same_with_and_without(pks, lambda: pks.filter_smooth(dm, y, prec))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_batched(pks, prec):
    """Packed sequences with nx = 12 (register-resident kernels)."""
    rng = np.random.default_rng(77)
    lengths = [300, 0, 1, 450, 2, 260]
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    models = [wl.random_stable_model(12, 5, np.random.default_rng(80 + b), radius=0.95) for b in range(6)]
    y = np.concatenate([wl.simulate(mo, L, rng)[0] if L else np.zeros((0, 5)) for mo, L in zip(models, lengths)])
    stack = lambda f: np.stack([getattr(mo, f) for mo in models])
    model = wl.Model(stack("F"), stack("Q"), stack("H"), stack("R"), stack("m0"), stack("P0"))
    dm = pks.to_device(model, per_sequence=True)
    yd = torch.as_tensor(y).to("cuda", torch.float64 if prec == "fp64" else torch.float32)
    off = torch.as_tensor(offsets).cuda()

    def run():
        m, P = pks.filter_batched(dm, off, yd, prec)
        ms, Ps = pks.smooth_batched(dm, off, m, P, prec)
        return m, P, ms, Ps
    same_with_and_without(pks, run)


def test_hmm(pks):
    w = wl.hmm_workload(K=40, T=5000, seed=11)
    dm = pks.hmm_to_device(w.Pi, w.p0)
    L = torch.as_tensor(w.L).cuda()
    same_with_and_without(pks, lambda: pks.hmm_filter_smooth(dm, L))
