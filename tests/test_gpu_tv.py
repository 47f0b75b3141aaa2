"""GPU parity for time-varying models (one row of F, u, Q, H, d, R per step;
Section IV's general model) against the oracle's time-varying recursion.

Same bar as the time-invariant parity tests: per result, per-step normwise
relative error <= 1e-9 in FP64 and <= 1e-4 in the mixed mode (reference: the
oracle on the float32-rounded y; random models' means pass through zero, so
the mixed check floors the denominator at the sequence's RMS norm).
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


def ref_tv(model, y, precision, loglik=False):
    yy = y if precision == "fp64" else y.astype(np.float32).astype(np.float64)
    return oracle.kf_rts_tv(model.F, model.Q, model.H, model.R, model.m0, model.P0, yy, u=model.u, d=model.d,
                            loglik=loglik)


def gpu_tv(pks, model, y, precision, separate=False):
    dm = pks.to_device(model, time_varying=True)
    dt = torch.float64 if precision == "fp64" else torch.float32
    yd = torch.as_tensor(np.ascontiguousarray(y)).to("cuda", dt)
    if separate:
        m, P = pks.filter(dm, yd, precision)
        ms, Ps = pks.smooth(dm, m, P, precision)
    else:
        m, P, ms, Ps = pks.filter_smooth(dm, yd, precision)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in zip(("m", "P", "ms", "Ps"), (m, P, ms, Ps))}


def check_tv(pks, model, y, precision, what, floor=None):
    floor = floor or ("rms" if precision == "mixed" else "none")
    ref = ref_tv(model, y, precision)
    out = gpu_tv(pks, model, y, precision)
    errs = {k: wl.max_rel_err(out[k], ref[k], floor) for k in ("m", "P", "ms", "Ps")}
    print(what, precision, {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= TOL[precision], (what, k, e)
    return out


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (3, 2), (4, 2), (4, 4), (2, 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tv_random_small(pks, nx, ny, precision):
    rng = np.random.default_rng(700 + 10 * nx + ny)
    model = wl.random_tv_model(nx, ny, 2001, rng)
    y, _ = wl.simulate_tv(model, rng)
    check_tv(pks, model, y, precision, "tv %dx%d" % (nx, ny))


@pytest.mark.parametrize("nx,ny,T", [(5, 2, 500), (8, 3, 400), (16, 8, 300), (33, 17, 64)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tv_random_large(pks, nx, ny, T, precision):
    rng = np.random.default_rng(800 + nx + 7 * ny)
    model = wl.random_tv_model(nx, ny, T, rng)
    y, _ = wl.simulate_tv(model, rng)
    check_tv(pks, model, y, precision, "tv large %dx%d" % (nx, ny))


@pytest.mark.parametrize("T", [1, 2, 3, 64, 65, 4099])
def test_tv_irregular_cv_lengths(pks, T):
    w = wl.workload(6, T=T)
    check_tv(pks, w.model, w.y, "fp64", "irregular cv T=%d" % T)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tv_irregular_cv_T2pow20(pks, precision):
    """The irregularly sampled constant-velocity workload at full size."""
    w = wl.workload(6)
    check_tv(pks, w.model, w.y, precision, "irregular cv T=2^20", floor="none")


@pytest.mark.parametrize("nx,ny", [(4, 2), (6, 3), (20, 3)])
def test_tv_with_equal_rows_equals_time_invariant(pks, nx, ny):
    """A time-varying model whose rows are all one model.  For nx <= 4 and
    nx > 16 the time-invariant call runs the same constants, kernels and
    arithmetic, so the results are bitwise the same; for 5 <= nx <= 16 one
    sequence of a time-invariant model runs the register-resident kernels
    (the time-varying one the packed-sequence kernels): the same mathematics
    in another order, compared at the parity tolerance."""
    rng = np.random.default_rng(31 + nx)
    mo = wl.random_small_model(nx, ny, rng) if nx <= 4 else wl.random_stable_model(nx, ny, rng,
                                                                                     with_offsets=True)
    T = 3000 if nx <= 4 else 300
    y, _ = wl.simulate(mo, T, rng)
    rep = lambda a: None if a is None else np.broadcast_to(a, (T,) + a.shape).copy()
    tv = wl.Model(rep(mo.F), rep(mo.Q), rep(mo.H), rep(mo.R), mo.m0, mo.P0, rep(mo.u), rep(mo.d))
    same_kernels = nx <= 4 or nx > 16
    for precision in ("fp64", "mixed"):
        dt = torch.float64 if precision == "fp64" else torch.float32
        yd = torch.as_tensor(y).to("cuda", dt)
        a = pks.filter_smooth(pks.to_device(mo), yd, precision)
        b = pks.filter_smooth(pks.to_device(tv, time_varying=True), yd, precision)
        torch.cuda.synchronize()
        for x, z in zip(a, b):
            if same_kernels:
                assert torch.equal(x, z), precision
            else:
                err = wl.max_rel_err(x.double().cpu().numpy(), z.double().cpu().numpy(),
                                     "rms" if precision == "mixed" else "none")
                assert err <= TOL[precision], (precision, err)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tv_separate_calls(pks, precision):
    rng = np.random.default_rng(5)
    model = wl.random_tv_model(4, 2, 3000, rng)
    y, _ = wl.simulate_tv(model, rng)
    ref = ref_tv(model, y, precision)
    out = gpu_tv(pks, model, y, precision, separate=True)
    floor = "rms" if precision == "mixed" else "none"
    for k in ("m", "P", "ms", "Ps"):
        assert wl.max_rel_err(out[k], ref[k], floor) <= TOL[precision], k


@pytest.mark.parametrize("nx,ny", [(4, 2), (6, 3), (17, 16), (33, 32)])
def test_tv_loglik(pks, nx, ny):
    """The per-step factors and partial sums of a time-varying model (FP64),
    each step's prediction from its own F_{k-1}, Q_{k-1}, u_{k-1}, H_k, R_k, d_k."""
    rng = np.random.default_rng(90 + nx)
    model = wl.random_tv_model(nx, ny, 2500, rng)
    y, _ = wl.simulate_tv(model, rng)
    ref = ref_tv(model, y, "fp64", loglik=True)
    rc, rt = oracle.loglik_prefix(ref["ll"])
    dm = pks.to_device(model, time_varying=True)
    yd = torch.as_tensor(y).cuda()
    m, P = pks.filter(dm, yd, "fp64")
    ll, tot = pks.loglik(dm, yd, m, P, "fp64")
    cum, tot2 = pks.loglik(dm, yd, m, P, "fp64", cumulative=True)
    torch.cuda.synchronize()
    ll, cum, tot = ll.cpu().numpy(), cum.cpu().numpy(), tot.cpu().numpy()
    assert np.max(np.abs(ll - ref["ll"]) / np.maximum(1.0, np.abs(ref["ll"]))) <= 1e-9
    assert np.max(np.abs(cum - rc) / np.maximum(1.0, np.abs(rc))) <= 1e-9
    assert abs(tot[0] - rt[0]) <= 1e-9 * max(1.0, abs(rt[0])) and tot2.item() == tot[0]


@pytest.mark.parametrize("nx", [3, 6])
def test_tv_numeric_flag(pks, nx):
    """A step whose innovation covariance is not positive definite: the flag
    names sequence 0 and the filtered outputs are NaN from that step on."""
    rng = np.random.default_rng(44 + nx)
    T, bad = 600, 333
    model = wl.random_tv_model(nx, 2, T, rng)
    y, _ = wl.simulate_tv(model, rng)
    model.R[bad] = -10.0 * np.eye(2)
    dm = pks.to_device(model, time_varying=True)
    ws = pks.workspace(nx, 2, T, 1, "fp64", time_varying=True)
    m, P = pks.filter(dm, torch.as_tensor(y).cuda(), "fp64", ws=ws)
    ok, first = pks.read_numeric_status(ws)
    assert not ok and first == 0
    assert not torch.isnan(m[:bad]).any() and torch.isnan(m[bad:]).all()


def _packed_tv(nx, ny, lengths, rng, per_sequence_prior):
    """Packed time-varying sequences: each sequence's rows from its own random
    model, rows concatenated like y; one prior per sequence or a shared one."""
    parts = [wl.random_tv_model(nx, ny, max(L, 1), rng) for L in lengths]
    ys = [wl.simulate_tv(mo, rng)[0][:L] for mo, L in zip(parts, lengths)]
    cat = lambda f: np.concatenate([getattr(mo, f)[:L] for mo, L in zip(parts, lengths)])
    if per_sequence_prior:
        m0 = np.stack([mo.m0 for mo in parts])
        P0 = np.stack([mo.P0 for mo in parts])
    else:
        m0, P0 = parts[0].m0, parts[0].P0
    model = wl.Model(cat("F"), cat("Q"), cat("H"), cat("R"), m0, P0, cat("u"), cat("d"))
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return model, np.concatenate(ys), offsets


def _ref_packed(model, y, offsets, per_sequence_prior, precision):
    yy = y if precision == "fp64" else y.astype(np.float32).astype(np.float64)
    total, nx = y.shape[0], model.nx
    out = {"m": np.empty((total, nx)), "P": np.empty((total, nx, nx)), "ms": np.empty((total, nx)),
           "Ps": np.empty((total, nx, nx)), "ll": np.empty(total)}
    for b in range(offsets.shape[0] - 1):
        s_ = slice(int(offsets[b]), int(offsets[b + 1]))
        if s_.stop == s_.start:
            continue
        m0 = model.m0[b] if per_sequence_prior else model.m0
        P0 = model.P0[b] if per_sequence_prior else model.P0
        r = oracle.kf_rts_tv(model.F[s_], model.Q[s_], model.H[s_], model.R[s_], m0, P0, yy[s_],
                             u=model.u[s_], d=model.d[s_], loglik=True)
        for k in out:
            out[k][s_] = r[k]
    return out


@pytest.mark.parametrize("nx,ny", [(3, 2), (6, 2)])
@pytest.mark.parametrize("per_sequence_prior", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tv_batched(pks, nx, ny, per_sequence_prior, precision):
    """Packed time-varying sequences (lengths 0, 1, 2 and several tiles): every
    sequence starts from its prior; filter, smoother and log-likelihood against
    the oracle run on each sequence's own rows."""
    rng = np.random.default_rng(60 + nx + (7 if per_sequence_prior else 0))
    lengths = [300, 0, 1, 2, 700, 64, 65] if nx <= 4 else [120, 0, 1, 2, 90]
    model, y, offsets = _packed_tv(nx, ny, lengths, rng, per_sequence_prior)
    ref = _ref_packed(model, y, offsets, per_sequence_prior, precision)
    dm = pks.to_device(model, per_sequence=per_sequence_prior, time_varying=True)
    dt = torch.float64 if precision == "fp64" else torch.float32
    yd = torch.as_tensor(y).to("cuda", dt)
    od = torch.as_tensor(offsets).cuda()
    m, P = pks.filter_batched(dm, od, yd, precision)
    ms, Ps = pks.smooth_batched(dm, od, m, P, precision)
    cum, tot = pks.loglik_batched(dm, od, yd, m, P, precision, cumulative=True)
    torch.cuda.synchronize()
    floor = "rms" if precision == "mixed" else "none"
    for k, g in (("m", m), ("P", P), ("ms", ms), ("Ps", Ps)):
        e = wl.max_rel_err(g.double().cpu().numpy(), ref[k], floor)
        print("tv batched", nx, per_sequence_prior, precision, k, "%.2e" % e, flush=True)
        assert e <= TOL[precision], k
    if precision == "fp64":
        rc, rt = oracle.loglik_prefix(ref["ll"], offsets)
        cum, tot = cum.cpu().numpy(), tot.cpu().numpy()
        assert np.max(np.abs(cum - rc) / np.maximum(1.0, np.abs(rc))) <= 1e-9
        assert np.max(np.abs(tot - rt) / np.maximum(1.0, np.abs(rt))) <= 1e-9


def test_tv_batched_numeric_flag(pks):
    """A failing step in sequence 2 of packed time-varying sequences: the flag
    names sequence 2, its outputs are NaN from that step on, the others finite."""
    rng = np.random.default_rng(8)
    lengths = [200, 150, 300, 100]
    model, y, offsets = _packed_tv(3, 2, lengths, rng, True)
    bad = int(offsets[2]) + 40
    model.R[bad] = -10.0 * np.eye(2)
    dm = pks.to_device(model, per_sequence=True, time_varying=True)
    ws = pks.workspace(3, 2, int(offsets[-1]), 4, "fp64", time_varying=True)
    od = torch.as_tensor(offsets).cuda()
    m, P = pks.filter_batched(dm, od, torch.as_tensor(y).cuda(), "fp64", ws=ws)
    ok, first = pks.read_numeric_status(ws)
    assert not ok and first == 2
    assert torch.isnan(m[bad:offsets[3]]).all() and not torch.isnan(m[offsets[2]:bad]).any()
    assert not torch.isnan(m[:offsets[2]]).any() and not torch.isnan(m[offsets[3]:]).any()


def test_tv_equal_rows_batched_equals_time_invariant_batched(pks):
    """Packed sequences whose rows all repeat one model, with one prior per
    sequence: bitwise the batched time-invariant result (same kernels and
    constants)."""
    w = wl.workload(4, B=9, T=900)
    mo = w.model.select(0)
    per_seq = wl.Model(*[np.stack([getattr(mo, f)] * w.B) for f in ("F", "Q", "H", "R")],
                       w.model.m0, w.model.P0)
    rep = lambda a: np.broadcast_to(a, (w.total,) + a.shape).copy()
    tv = wl.Model(rep(mo.F), rep(mo.Q), rep(mo.H), rep(mo.R), w.model.m0, w.model.P0)
    od = torch.as_tensor(w.offsets).cuda()
    yd = torch.as_tensor(w.y).cuda()
    a = pks.filter_batched(pks.to_device(per_seq, per_sequence=True), od, yd, "fp64")
    b = pks.filter_batched(pks.to_device(tv, per_sequence=True, time_varying=True), od, yd, "fp64")
    sa = pks.smooth_batched(pks.to_device(per_seq, per_sequence=True), od, *a, "fp64")
    sb = pks.smooth_batched(pks.to_device(tv, per_sequence=True, time_varying=True), od, *b, "fp64")
    torch.cuda.synchronize()
    for x, z in zip(a + sa, b + sb):
        assert torch.equal(x, z)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("batched", [False, True])
def test_tv_plan(pks, precision, batched):
    """A time-varying model captured into a plan (per-step precompute and both
    passes in one graph): against the oracle, every replay (with eager calls
    on the same stream in between) bitwise equal to the first, and equal to
    the eager call where that runs the same kernels (the batched eager path
    has no fused filter + smoother call, so in the mixed mode, where the plan
    fuses the filter down-sweep with the smoother reduce, its smoothed moments
    differ from the separate eager calls in rounding only)."""
    rng = np.random.default_rng(71 + (3 if batched else 0))
    dt = torch.float64 if precision == "fp64" else torch.float32
    floor = "rms" if precision == "mixed" else "none"
    if batched:
        model, y, offsets = _packed_tv(3, 2, [300, 0, 1, 2, 700, 65], rng, True)
        ref = _ref_packed(model, y, offsets, True, precision)
        dm = pks.to_device(model, per_sequence=True, time_varying=True)
        od = torch.as_tensor(offsets).cuda()
    else:
        model = wl.random_tv_model(4, 2, 3000, rng)
        y, _ = wl.simulate_tv(model, rng)
        ref = ref_tv(model, y, precision)
        dm = pks.to_device(model, time_varying=True)
        od = None
    yd = torch.as_tensor(np.ascontiguousarray(y)).to("cuda", dt)
    if batched:
        em, eP = pks.filter_batched(dm, od, yd, precision)
        ems, ePs = pks.smooth_batched(dm, od, em, eP, precision)
    else:
        em, eP, ems, ePs = pks.filter_smooth(dm, yd, precision)
    plan = pks.Plan(dm, yd, od, precision)
    first = None
    same_kernels = not (batched and precision == "mixed")
    for rep in range(3):
        out = [t.clone() for t in plan.launch()]
        torch.cuda.synchronize()
        first = first or out
        for k, g, e, f in zip(("m", "P", "ms", "Ps"), out, (em, eP, ems, ePs), first):
            assert torch.equal(g, f), (rep, k)
            if k in ("m", "P") or same_kernels:
                assert torch.equal(g, e), (rep, k)
            err = wl.max_rel_err(g.double().cpu().numpy(), ref[k], floor)
            assert err <= TOL[precision], (rep, k, err)
        if batched:                                   # eager work between replays
            pks.filter_batched(dm, od, yd, precision)
        else:
            pks.filter(dm, yd, precision)
    plan.close()