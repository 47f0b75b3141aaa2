"""GPU parity of the discrete-state (HMM) filter and smoother against the
sequential forward-backward oracle.

Bars: filtered and smoothed marginals are probabilities in [0, 1], compared
element by element in absolute terms, |alpha - ref| <= 1e-9 and
|gamma - ref| <= 1e-9; the log-likelihood prefixes log p(y_1:k) against the
oracle's running sum, |logp_k - ref_k| <= 1e-9 max(1, sum_j<=k |ll_j|).
"""
import numpy as np
import pytest

import oracle
from paper_1905_13002_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def pks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_13002_amd import pks as mod
    return mod


def run_gpu(pks, Pi, p0, L, smooth=True):
    dm = pks.hmm_to_device(Pi, p0)
    Ld = torch.as_tensor(np.ascontiguousarray(L, dtype=np.float64)).cuda()
    alpha, logp, gamma = pks.hmm_filter_smooth(dm, Ld, smooth=smooth)
    torch.cuda.synchronize()
    f = lambda t: None if t is None else t.cpu().numpy()
    return f(alpha), f(logp), f(gamma)


def check(pks, Pi, p0, L, what=""):
    ref = oracle.hmm_fb(Pi, p0, L)
    alpha, logp, gamma = run_gpu(pks, Pi, p0, L)
    rcum = np.cumsum(ref["ll"])
    acum = np.cumsum(np.abs(ref["ll"]))
    ea = np.max(np.abs(alpha - ref["alpha"]), initial=0.0)
    eg = np.max(np.abs(gamma - ref["gamma"]), initial=0.0)
    el = np.max(np.abs(logp - rcum) / np.maximum(1.0, acum), initial=0.0)
    print(what, "alpha %.2e gamma %.2e logp %.2e" % (ea, eg, el), flush=True)
    assert ea <= TOL and eg <= TOL and el <= TOL, (what, ea, eg, el)
    return alpha, logp, gamma


@pytest.mark.parametrize("K", [1, 2, 3, 5, 16, 17, 31, 33, 48, 64])
@pytest.mark.parametrize("T", [1, 2, 5, 777])
def test_hmm_random_models(pks, K, T):
    """Every padded state count (16, 32, 48, 64 after padding), one to many
    blocks, ragged last block."""
    w = wl.hmm_workload(K=K, T=T, seed=100 + T)
    check(pks, w.Pi, w.p0, w.L, "K=%d T=%d" % (K, T))


@pytest.mark.parametrize("K", [4, 23, 64])
def test_hmm_sparse_transitions(pks, K):
    """Transition matrices with many zeros (states the filter cannot reach
    from others): the smoother's rows of unreachable states carry no weight."""
    w = wl.hmm_workload(K=K, T=3000, seed=200, sparse=True)
    check(pks, w.Pi, w.p0, w.L, "sparse K=%d" % K)


def test_hmm_deterministic_cycle(pks):
    """A cyclic permutation with a known start: filtered = smoothed = the
    indicator of k mod K, log p(y_1:T) = sum of the visited log-likelihoods."""
    K, T = 7, 5000
    Pi = np.roll(np.eye(K), 1, axis=1)
    p0 = np.eye(K)[0]
    L = np.random.default_rng(3).normal(size=(T, K))
    alpha, logp, gamma = check(pks, Pi, p0, L, "cycle")
    ind = np.eye(K)[np.arange(1, T + 1) % K]
    assert np.max(np.abs(alpha - ind)) < 1e-12 and np.max(np.abs(gamma - ind)) < 1e-12


def test_hmm_smoother_alone_and_filter_alone(pks):
    """pks_hmm_smooth from the oracle's filtered marginals, and pks_hmm_filter
    without the smoother, both against the oracle."""
    w = wl.hmm_workload(K=20, T=4000, seed=300)
    ref = oracle.hmm_fb(w.Pi, w.p0, w.L)
    dm = pks.hmm_to_device(w.Pi, w.p0)
    a = torch.as_tensor(ref["alpha"]).cuda()
    g = pks.hmm_smooth(dm, a)
    alpha, logp, none = run_gpu(pks, w.Pi, w.p0, w.L, smooth=False)
    torch.cuda.synchronize()
    assert none is None
    assert np.max(np.abs(g.cpu().numpy() - ref["gamma"])) <= TOL
    assert np.max(np.abs(alpha - ref["alpha"])) <= TOL


def test_hmm_empty_is_noop(pks):
    dm = pks.hmm_to_device(np.eye(3), np.ones(3) / 3)
    alpha, logp, gamma = pks.hmm_filter_smooth(dm, torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    assert alpha.shape == (0, 3) and gamma.shape == (0, 3)


def test_hmm_argument_errors(pks):
    dm = pks.hmm_to_device(np.eye(3), np.ones(3) / 3)
    L = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    ws = pks.hmm_workspace(3, 10)
    with pytest.raises(pks.PksError):
        pks.hmm_filter_smooth(dm, L, ws=ws[:16])                    # workspace too small
    bad = pks.hmm_to_device(np.eye(65), np.ones(65) / 65)
    with pytest.raises(pks.PksError):
        pks.hmm_filter_smooth(bad, torch.zeros((4, 65), dtype=torch.float64, device="cuda"))


def test_hmm_workload_K64_T65536(pks):
    """The benchmark's HMM workload: 64 states, 2^16 steps."""
    w = wl.hmm_workload()
    check(pks, w.Pi, w.p0, w.L, "K=64 T=65536")


def test_hmm_long_sequence(pks):
    """T = 2^20 steps of an 8-state chain (2048 blocks, eleven scan levels)."""
    w = wl.hmm_workload(K=8, T=1 << 20, seed=400)
    check(pks, w.Pi, w.p0, w.L, "K=8 T=2^20")
