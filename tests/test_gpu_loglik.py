"""GPU parity of the marginal likelihood (Section III-C) against the oracle.

The HIP path evaluates every factor log p(y_k | y_1:k-1) from the filtered
moments that its own filter wrote, then sums them (segmented prefix sums);
the oracle takes the same factors from its sequential Kalman recursion.

Bar: per step |ll_k - ll_k^ref| <= tol * b_k, and for the partial sums
log p(y_1:k) and the totals |sum - ref| <= tol * (b_1 + ... + b_k), with
    b_k = s_k + a_k,
    s_k = (ny log(2 pi) + |log det S_k| + r_k^T S_k^-1 r_k) / 2,
    a_k = |v_k|^T (|G| |m_{k-1}| + |y_k| + |e|)
          + sum_ij |S_k^-1 - v_k v_k^T|_ij (|G| |P_{k-1}| |G|^T)_ij / 2,
where S_k, r_k are the oracle's innovation covariance and residual,
v_k = S_k^-1 r_k, G = H F, e = H u + d.  s_k is the size of the terms that
make up the factor; a_k bounds, to first order, how far the factor moves when
m_{k-1}, P_{k-1} and y_k move by a relative amount (the gradient of the factor
is -v_k in the residual and -(S_k^-1 - v_k v_k^T)/2 in S_k).  tol is the bar of
the moments the factors are computed from: 1e-9 in FP64, 1e-4 in the mixed
mode (whose reference is the oracle on the float32-rounded y).  a_k matters
where the residual is a small difference of large numbers (positions of 1e7
stored in float32).
"""
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


def _model_b(model, b, per_sequence):
    if not per_sequence:
        return model
    g = lambda a: None if a is None else a[b]
    return wl.Model(model.F[b], model.Q[b], model.H[b], model.R[b], model.m0[b], model.P0[b],
                    g(model.u), g(model.d))


def oracle_ll(model, y, offsets, per_sequence):
    """Per-step factors, partial sums, totals and the bar's b_k, from the oracle."""
    total = y.shape[0]
    ll = np.empty(total)
    bar = np.empty(total)
    B = offsets.shape[0] - 1
    for b in range(B):
        s, e = int(offsets[b]), int(offsets[b + 1])
        if e == s:
            continue
        mo = _model_b(model, b, per_sequence)
        nx, ny = mo.F.shape[0], mo.H.shape[0]
        out = oracle.kf_rts(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, y[s:e], u=mo.u, d=mo.d, smooth=False,
                            predicted=True, loglik=True)
        ll[s:e] = out["ll"]
        u = np.zeros(nx) if mo.u is None else mo.u
        d = np.zeros(ny) if mo.d is None else mo.d
        G, ev = mo.H @ mo.F, mo.H @ u + d
        mprev = np.concatenate([mo.m0[None], out["m"][:-1]])
        Pprev = np.concatenate([mo.P0[None], out["P"][:-1]])
        S = np.einsum("ij,kjl,ml->kim", mo.H, out["Pp"], mo.H) + mo.R
        r = y[s:e] - out["mp"] @ mo.H.T - d
        Si = np.linalg.inv(S)
        v = np.einsum("kij,kj->ki", Si, r)
        sk = 0.5 * (ny * np.log(2 * np.pi) + np.abs(np.linalg.slogdet(S)[1]) + np.sum(r * v, axis=1))
        aG = np.abs(G)
        ak = np.sum(np.abs(v) * (np.abs(mprev) @ aG.T + np.abs(y[s:e]) + np.abs(ev)), axis=1)
        GPG = np.einsum("ij,kjl,ml->kim", aG, np.abs(Pprev), aG)
        ak += 0.5 * np.sum(np.abs(Si - v[:, :, None] * v[:, None, :]) * GPG, axis=(1, 2))
        bar[s:e] = sk + ak
    cum, tot = oracle.loglik_prefix(ll, offsets)
    cbar, tbar = oracle.loglik_prefix(bar, offsets)
    return ll, cum, tot, bar, cbar, tbar


def gpu_ll(pks, model, y, precision, offsets=None, per_sequence=False):
    """Filter, then the per-step factors + totals, then the partial sums; also
    the totals alone.  Returns numpy arrays."""
    dm = pks.to_device(model, per_sequence=per_sequence)
    dt = torch.float64 if precision == "fp64" else torch.float32
    yd = torch.as_tensor(np.ascontiguousarray(y)).to("cuda", dt)
    if offsets is None:
        m, P = pks.filter(dm, yd, precision)
        steps, tot = pks.loglik(dm, yd, m, P, precision)
        cum, tot2 = pks.loglik(dm, yd, m, P, precision, cumulative=True)
        none, tot3 = pks.loglik(dm, yd, m, P, precision, steps=False)
    else:
        od = torch.as_tensor(np.asarray(offsets, dtype=np.int64)).cuda()
        m, P = pks.filter_batched(dm, od, yd, precision)
        steps, tot = pks.loglik_batched(dm, od, yd, m, P, precision)
        cum, tot2 = pks.loglik_batched(dm, od, yd, m, P, precision, cumulative=True)
        none, tot3 = pks.loglik_batched(dm, od, yd, m, P, precision, steps=False)
    torch.cuda.synchronize()
    assert none is None
    f = lambda t: t.cpu().numpy()
    # the three totals come from the same sums: bitwise equal
    assert np.array_equal(f(tot), f(tot2)) and np.array_equal(f(tot), f(tot3))
    return f(steps), f(cum), f(tot)


def check_ll(pks, model, y, precision, offsets=None, per_sequence=False, what=""):
    yref = y if precision == "fp64" else y.astype(np.float32).astype(np.float64)
    offs = np.array([0, y.shape[0]], dtype=np.int64) if offsets is None else np.asarray(offsets, np.int64)
    ll, cum, tot, s, cs, ts = oracle_ll(model, yref, offs, per_sequence)
    g_ll, g_cum, g_tot = gpu_ll(pks, model, y, precision, offsets, per_sequence)
    tol = TOL[precision]
    e_step = np.max(np.abs(g_ll - ll) / np.maximum(s, 1e-300), initial=0.0)
    e_cum = np.max(np.abs(g_cum - cum) / np.maximum(cs, 1e-300), initial=0.0)
    e_tot = np.max(np.abs(g_tot - tot) / np.maximum(ts, 1e-300), initial=0.0)
    print(what, precision, "step %.2e cum %.2e tot %.2e (max abs step error %.2e)"
          % (e_step, e_cum, e_tot, np.max(np.abs(g_ll - ll), initial=0.0)), flush=True)
    assert e_step <= tol and e_cum <= tol and e_tot <= tol, (what, e_step, e_cum, e_tot)
    # the last partial sum of every non-empty sequence is its total, bitwise
    for b in range(offs.shape[0] - 1):
        if offs[b + 1] > offs[b]:
            assert g_cum[offs[b + 1] - 1] == g_tot[b]
        else:
            assert g_tot[b] == 0.0
    return g_ll, g_cum, g_tot


# ---------------------------------------------------------------------------
# single sequences
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("T", [1, 2, 255, 256, 257, 1023, 1024, 1025, 5000])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_cv_ragged(pks, T, precision):
    """The CV model of Section V across one-, several- and many-block lengths
    (256-step tiles of the factor kernel, 1024-step blocks of the sums)."""
    w = wl.workload(1, T=T)
    check_ll(pks, w.model, w.y, precision, what="cv T=%d" % T)


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (3, 3), (4, 4), (4, 2), (2, 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_random_small_models(pks, nx, ny, precision):
    rng = np.random.default_rng(300 + 10 * nx + ny)
    model = wl.random_small_model(nx, ny, rng)
    y, _ = wl.simulate(model, 3001, rng)
    check_ll(pks, model, y, precision, what="small %dx%d" % (nx, ny))


@pytest.mark.parametrize("nx,ny,T", [(4, 6, 700), (1, 9, 300), (5, 2, 777), (8, 3, 1100), (16, 8, 2000),
                                     (33, 17, 150), (64, 32, 120), (64, 64, 40)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_one_wave_per_step(pks, nx, ny, T, precision):
    """Sizes outside nx, ny <= 4 take the one-wavefront-per-step kernel."""
    rng = np.random.default_rng(400 + nx + 3 * ny)
    model = wl.random_stable_model(nx, ny, rng, radius=0.95)
    y, _ = wl.simulate(model, T, rng)
    check_ll(pks, model, y, precision, what="wave %dx%d" % (nx, ny))


def test_loglik_with_u_and_d(pks):
    """Nonzero u and d enter the prediction (e = H u + d in the residual)."""
    rng = np.random.default_rng(77)
    for nx, ny in ((3, 2), (6, 3)):
        model = wl.random_small_model(nx, ny, rng) if nx <= 4 else wl.random_stable_model(nx, ny, rng)
        model = wl.Model(model.F, model.Q, model.H, model.R, model.m0, model.P0,
                         rng.standard_normal(nx), rng.standard_normal(ny))
        y, _ = wl.simulate(model, 900, rng)
        check_ll(pks, model, y, "fp64", what="u,d %dx%d" % (nx, ny))


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_batched_uneven_cv(pks, precision):
    """Per-sequence CV models, lengths from 0 to several blocks: the sums restart
    at every sequence start and carry across block boundaries inside a sequence."""
    w = wl.workload(4, B=61, T=2600)
    lengths = np.diff(w.offsets).copy()
    lengths[:8] = [1, 0, 2, 1023, 1024, 1025, 0, 3000]
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    y = np.concatenate([w.y, np.zeros((max(0, int(offsets[-1]) - w.total), 2))])[: offsets[-1]]
    check_ll(pks, w.model, y, precision, offsets=offsets, per_sequence=True, what="batched cv")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_batched_shared_large_state(pks, precision):
    rng = np.random.default_rng(5)
    model = wl.random_stable_model(6, 3, rng, radius=0.9)
    lengths = rng.integers(0, 700, size=9)
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    y, _ = wl.simulate(model, int(offsets[-1]), rng)
    check_ll(pks, model, y, precision, offsets=offsets, what="batched shared 6x3")


def test_loglik_many_short_sequences(pks):
    """More sequences than steps in a block: many sequence starts per block."""
    rng = np.random.default_rng(9)
    model = wl.random_small_model(2, 1, rng)
    lengths = rng.integers(0, 9, size=1500)
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    y, _ = wl.simulate(model, int(offsets[-1]), rng)
    check_ll(pks, model, y, "fp64", offsets=offsets, what="1500 short")


# ---------------------------------------------------------------------------
# edge cases, flags, reproducibility, full size
# ---------------------------------------------------------------------------
def test_loglik_empty(pks):
    mo = wl.cv_model()
    dm = pks.to_device(mo)
    y = torch.zeros(0, 2, dtype=torch.float64, device="cuda")
    m = torch.zeros(0, 4, dtype=torch.float64, device="cuda")
    P = torch.zeros(0, 4, 4, dtype=torch.float64, device="cuda")
    ll, tot = pks.loglik(dm, y, m, P, "fp64")
    torch.cuda.synchronize()
    assert ll.shape == (0,) and tot.item() == 0.0
    od = torch.zeros(4, dtype=torch.int64, device="cuda")
    dmb = pks.to_device(wl.Model(*[np.stack([a] * 3) for a in (mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0)]),
                        per_sequence=True)
    _, tots = pks.loglik_batched(dmb, od, y, m, P, "fp64", steps=False)
    torch.cuda.synchronize()
    assert torch.equal(tots.cpu(), torch.zeros(3, dtype=torch.float64))


def test_loglik_numeric_flag_and_nan(pks):
    """A sequence whose innovation covariance is not positive definite: NaN in
    its factors and total, the flag names it; the others are unaffected.  A NaN
    in y gives NaN from that step on without the flag."""
    w = wl.workload(4, B=5, T=300)
    R = w.model.R.copy()
    R[3] = -np.eye(2)
    bad = wl.Model(w.model.F, w.model.Q, w.model.H, R, w.model.m0, w.model.P0)
    dm = pks.to_device(bad, per_sequence=True)
    od = torch.as_tensor(w.offsets).cuda()
    yd = torch.as_tensor(w.y).cuda()
    ws = pks.workspace(4, 2, w.total, w.B)
    m, P = pks.filter_batched(dm, od, yd, "fp64", ws=ws)
    pks.read_numeric_status(ws)                    # the filter's own flag, cleared
    ll, tot = pks.loglik_batched(dm, od, yd, m, P, "fp64", ws=ws)
    ok, first = pks.read_numeric_status(ws)
    assert not ok and first == 3
    assert torch.isnan(ll[w.seq(3)]).all() and torch.isnan(tot[3])
    good = [b for b in range(w.B) if b != 3]
    assert not torch.isnan(tot[good]).any()

    w1 = wl.workload(1, T=3000)
    y = w1.y.copy()
    y[1234, 0] = np.nan
    dm1 = pks.to_device(w1.model)
    yd1 = torch.as_tensor(y).cuda()
    ws1 = pks.workspace(4, 2, 3000)
    m1, P1 = pks.filter(dm1, yd1, "fp64", ws=ws1)
    cum, tot1 = pks.loglik(dm1, yd1, m1, P1, "fp64", cumulative=True, ws=ws1)
    ok, _ = pks.read_numeric_status(ws1)
    assert ok
    assert not torch.isnan(cum[:1234]).any() and torch.isnan(cum[1234:]).all() and torch.isnan(tot1).all()


def test_loglik_reproducible(pks):
    w = wl.workload(4, B=40, T=3000)
    dm = pks.to_device(w.model, per_sequence=True)
    od = torch.as_tensor(w.offsets).cuda()
    yd = torch.as_tensor(w.y).cuda()
    m, P = pks.filter_batched(dm, od, yd, "fp64")
    a = pks.loglik_batched(dm, od, yd, m, P, "fp64", cumulative=True)
    b = pks.loglik_batched(dm, od, yd, m, P, "fp64", cumulative=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_cv_T2pow20(pks, precision):
    """The CV workload at T = 2^20, every factor, partial sum and the total
    against the oracle."""
    w = wl.workload(2)
    check_ll(pks, w.model, w.y, precision, what="cv T=2^20")


def test_loglik_runs_of_empty_sequences(pks):
    """Long runs of zero-length sequences between and inside tiles: the tile
    table brackets a lane's search over hundreds of equal offsets."""
    rng = np.random.default_rng(21)
    model = wl.random_small_model(3, 2, rng)
    lengths = [0] * 700 + [5000] + [0] * 300 + [1] + [0] * 50 + [300] + [0] * 9
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    y, _ = wl.simulate(model, int(offsets[-1]), rng)
    check_ll(pks, model, y, "fp64", offsets=offsets, what="empty runs")
    model6 = wl.random_stable_model(6, 2, rng, radius=0.9)
    y6, _ = wl.simulate(model6, int(offsets[-1]), rng)
    check_ll(pks, model6, y6, "fp64", offsets=offsets, what="empty runs 6x2")


def test_loglik_cv_T2pow23(pks):
    """T = 2^23 (2048 blocks of the prefix sums, so the top-level scan runs
    over several chunks): every partial sum against the oracle's running sum
    (bar: 1e-9 of the running sum of |factors|)."""
    w = wl.workload(1, T=1 << 23)
    ref = oracle.kf_rts(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0, w.model.P0, w.y, smooth=False,
                        loglik=True)["ll"]
    rc = np.cumsum(ref)
    bar = 1e-9 * np.cumsum(np.abs(ref))
    dm = pks.to_device(w.model)
    yd = torch.as_tensor(w.y).cuda()
    m, P = pks.filter(dm, yd, "fp64")
    cum, tot = pks.loglik(dm, yd, m, P, "fp64", cumulative=True)
    steps, tot2 = pks.loglik(dm, yd, m, P, "fp64")
    torch.cuda.synchronize()
    cum, tot, steps = cum.cpu().numpy(), tot.cpu().numpy(), steps.cpu().numpy()
    assert np.all(np.abs(cum - rc) <= bar)
    assert abs(tot[0] - rc[-1]) <= bar[-1] and tot2.item() == tot[0] and cum[-1] == tot[0]
    # the per-step output of the same call path, summed on the host, gives the
    # partial sums (positions reach 4e8 here, so the factors themselves carry
    # the FP64 moments' rounding; their bar is checked at T = 2^20)
    assert np.all(np.abs(np.cumsum(steps) - cum) <= 1e-12 * np.cumsum(np.abs(steps)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loglik_batched_per_sequence_large_state(pks, precision):
    """Per-sequence models through the one-wave kernel (nx = 6, ny = 5): each
    step's G, S, e and, at a sequence start, the prior come from its own model."""
    rng = np.random.default_rng(17)
    B = 7
    models = [wl.random_stable_model(6, 5, rng, radius=0.9, with_offsets=True) for _ in range(B)]
    lengths = [130, 0, 1, 257, 40, 2, 90]
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    ys = [wl.simulate(mo, L, rng)[0] if L else np.zeros((0, 5)) for mo, L in zip(models, lengths)]
    stack = lambda f: np.stack([getattr(mo, f) for mo in models])
    model = wl.Model(stack("F"), stack("Q"), stack("H"), stack("R"), stack("m0"), stack("P0"), stack("u"),
                     stack("d"))
    check_ll(pks, model, np.concatenate(ys), precision, offsets=offsets, per_sequence=True,
             what="per-sequence 6x5")
