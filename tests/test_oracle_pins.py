"""Pins for the oracle: checks against what the paper and the mathematics fix.

None of these retypes the oracle's formulas.  Each compares the sequential
recursion (``oracle.kf_rts``) or the element/operator restatement
(``oracle.elements``) with an independent computation: a dense joint-Gaussian
solve, a closed form, hand-derived values, a library DARE solver, numerical
quadrature of the defining integrals, or a structural invariant.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import elements as el
from paper_1905_13002_amd import workloads as wl
from tests.dense_posterior import joint_loglik, posterior, posterior_tv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nerr(X, Xref):
    return wl.max_rel_err(X, Xref)


def run(model, y, **kw):
    return oracle.kf_rts(model.F, model.Q, model.H, model.R, model.m0, model.P0, y,
                         u=model.u, d=model.d, **kw)


# ---------------------------------------------------------------------------
# the sequential oracle vs a dense joint-Gaussian solve
# ---------------------------------------------------------------------------

DENSE_CASES = [
    (1, 1, 1, False), (1, 1, 9, False), (2, 1, 12, False), (3, 2, 20, False),
    (4, 2, 24, False), (4, 3, 16, True), (5, 2, 10, True), (3, 3, 2, False),
]


@pytest.mark.parametrize("nx,ny,T,singQ", DENSE_CASES)
def test_oracle_matches_dense_joint_posterior(nx, ny, T, singQ):
    rng = np.random.default_rng(1000 + 17 * nx + 3 * ny + T)
    model = wl.random_small_model(nx, ny, rng, singular_Q=singQ)
    y, _ = wl.simulate(model, T, rng)
    out = run(model, y)
    m, P, ms, Ps = posterior(model.F, model.Q, model.H, model.R, model.m0, model.P0, y,
                             model.u, model.d)
    assert nerr(out["m"], m) < 1e-10
    assert nerr(out["P"], P) < 1e-10
    assert nerr(out["ms"], ms) < 1e-10
    assert nerr(out["Ps"], Ps) < 1e-10


def test_oracle_cv_model_matches_dense_joint_posterior():
    w = wl.workload(1, T=40)
    out = run(w.model, w.y)
    m, P, ms, Ps = posterior(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0,
                             w.model.P0, w.y)
    for a, b in ((out["m"], m), (out["P"], P), (out["ms"], ms), (out["Ps"], Ps)):
        assert nerr(a, b) < 1e-10


# ---------------------------------------------------------------------------
# closed forms and hand values
# ---------------------------------------------------------------------------

def test_static_model_closed_form():
    """F = I, u = 0, Q = 0: information adds up, x never moves (smoothed = last filtered)."""
    rng = np.random.default_rng(7)
    nx, ny, T = 3, 2, 50
    H = rng.standard_normal((ny, nx))
    R = np.array([[0.5, 0.1], [0.1, 0.3]])
    m0 = rng.standard_normal(nx)
    P0 = np.diag([2.0, 1.0, 0.5])
    model = wl.Model(np.eye(nx), np.zeros((nx, nx)), H, R, m0, P0, None, np.array([0.2, -0.1]))
    y, _ = wl.simulate(model, T, rng)
    out = run(model, y)
    Ri = np.linalg.inv(R)
    P0i = np.linalg.inv(P0)
    acc = np.zeros(nx)
    for k in range(T):
        acc += H.T @ Ri @ (y[k] - model.d)
        Pk = np.linalg.inv(P0i + (k + 1) * H.T @ Ri @ H)
        mk = Pk @ (P0i @ m0 + acc)
        assert np.linalg.norm(out["P"][k] - Pk) <= 1e-12 * np.linalg.norm(Pk)
        assert np.linalg.norm(out["m"][k] - mk) <= 1e-12 * max(1.0, np.linalg.norm(mk))
    for k in range(T):
        assert np.linalg.norm(out["ms"][k] - out["m"][-1]) <= 1e-12 * max(1.0, np.linalg.norm(out["m"][-1]))
        assert np.linalg.norm(out["Ps"][k] - out["P"][-1]) <= 1e-12 * np.linalg.norm(out["P"][-1])


def test_scalar_hand_derived_values():
    g = json.load(open(os.path.join(GOLDEN, "scalar_T2.json")))
    mo = g["model"]
    out = oracle.kf_rts(mo["F"], mo["Q"], mo["H"], mo["R"], mo["m0"], mo["P0"], g["y"])
    for key in ("m", "P", "ms", "Ps"):
        np.testing.assert_allclose(out[key], np.array(g[key]), rtol=1e-15, atol=0)  # a few ulps of rounding


def test_cv_model_constants_match_section5():
    g = json.load(open(os.path.join(GOLDEN, "cv_model_section5.json")))
    mo = wl.cv_model(q=g["q"], r=g["sigma"] ** 2, dt=g["dt"], m0=g["m0"])
    for key in ("F", "Q", "H", "R"):
        np.testing.assert_allclose(getattr(mo, key), np.array(g[key], dtype=float), rtol=1e-15, atol=0)
    np.testing.assert_array_equal(mo.m0, np.array(g["m0"]))


def test_steady_state_matches_dare():
    """Time-invariant, detectable/stabilisable model: P^-_k tends to the DARE solution (scipy)."""
    mo = wl.cv_model(1.0, 0.25)
    w = wl.workload(1, T=600)
    out = run(mo, w.y, predicted=True)
    X = scipy.linalg.solve_discrete_are(mo.F.T, mo.H.T, mo.Q, mo.R)
    assert np.linalg.norm(out["Pp"][-1] - X) <= 1e-10 * np.linalg.norm(X)
    # and the filtered covariance is the update of it
    S = mo.H @ X @ mo.H.T + mo.R
    Pf = X - X @ mo.H.T @ np.linalg.solve(S, mo.H @ X)
    assert np.linalg.norm(out["P"][-1] - Pf) <= 1e-10 * np.linalg.norm(Pf)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_T1_smoothed_equals_filtered_bitwise():
    rng = np.random.default_rng(3)
    mo = wl.random_small_model(3, 2, rng)
    y, _ = wl.simulate(mo, 1, rng)
    out = run(mo, y)
    assert np.array_equal(out["ms"], out["m"]) and np.array_equal(out["Ps"], out["P"])


def test_last_smoothed_equals_last_filtered_bitwise():
    w = wl.workload(1)
    out = run(w.model, w.y)
    assert np.array_equal(out["ms"][-1], out["m"][-1])
    assert np.array_equal(out["Ps"][-1], out["P"][-1])


def test_covariances_symmetric_and_psd():
    rng = np.random.default_rng(11)
    for nx, ny, singQ in ((4, 2, False), (5, 3, True), (2, 2, False)):
        mo = wl.random_small_model(nx, ny, rng, singular_Q=singQ)
        y, _ = wl.simulate(mo, 200, rng)
        out = run(mo, y)
        for key in ("P", "Ps"):
            X = out[key]
            assert np.array_equal(X, np.swapaxes(X, 1, 2))
            ev = np.linalg.eigvalsh(X)
            nrm = np.linalg.norm(X, axis=(1, 2))
            assert np.all(ev.min(axis=1) >= -1e-12 * nrm)


def test_covariances_independent_of_y_and_means_affine():
    rng = np.random.default_rng(5)
    mo = wl.random_small_model(4, 2, rng)
    T = 64
    y1, _ = wl.simulate(mo, T, rng)
    y2, _ = wl.simulate(mo, T, rng)
    o1, o2 = run(mo, y1), run(mo, y2)
    o12, o0 = run(mo, y1 + y2), run(mo, np.zeros_like(y1))
    for key in ("P", "Ps"):
        assert np.array_equal(o1[key], o2[key])
    for key in ("m", "ms"):
        resid = o12[key] - o1[key] - o2[key] + o0[key]
        scale = np.abs(o1[key]).max() + np.abs(o2[key]).max()
        assert np.abs(resid).max() <= 1e-12 * scale


def test_batched_matches_per_sequence():
    w = wl.workload(4, B=6, T=300)
    out = oracle.kf_rts_batched(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0,
                                w.model.P0, w.y, w.offsets, per_sequence=True, threads=3)
    for b in range(w.B):
        s = w.seq(b)
        one = run(w.model_of(b), w.y[s])
        for key in ("m", "P", "ms", "Ps"):
            assert np.array_equal(out[key][s], one[key])


# ---------------------------------------------------------------------------
# elements and operators (Lemmas 1-4) against the recursion and the integrals
# ---------------------------------------------------------------------------

def test_filter_elements_left_fold_equals_kalman_filter():
    """Theorem 1: the prefix a_1 ⊗ ... ⊗ a_k holds p(x_k | y_{1:k})."""
    rng = np.random.default_rng(21)
    for nx, ny in ((1, 1), (3, 2), (4, 2), (5, 3)):
        mo = wl.random_small_model(nx, ny, rng)
        y, _ = wl.simulate(mo, 60, rng)
        els = el.filter_elements(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, y, mo.u, mo.d)
        m, P = el.filter_prefix_fold(els)
        ref = run(mo, y)
        assert nerr(m, ref["m"]) < 1e-12 and nerr(P, ref["P"]) < 1e-12


def test_smoother_elements_suffix_fold_equals_rts():
    """Theorem 2: a_k ⊗ ... ⊗ a_n holds p(x_k | y_{1:n})."""
    rng = np.random.default_rng(22)
    for nx, ny in ((1, 1), (3, 2), (4, 2), (5, 3)):
        mo = wl.random_small_model(nx, ny, rng)
        y, _ = wl.simulate(mo, 60, rng)
        ref = run(mo, y)
        els = el.smoother_elements(mo.F, mo.Q, ref["m"], ref["P"], mo.u)
        ms, Ps = el.smoother_suffix_fold(els)
        assert nerr(ms, ref["ms"]) < 1e-12 and nerr(Ps, ref["Ps"]) < 1e-12


def _random_filter_element(nx, rng, zeroA=False):
    A = np.zeros((nx, nx)) if zeroA else rng.standard_normal((nx, nx)) * 0.7
    b = rng.standard_normal(nx)
    Bc = rng.standard_normal((nx, nx))
    C = Bc @ Bc.T / nx
    eta = rng.standard_normal(nx)
    Bj = rng.standard_normal((nx, max(1, nx - 1)))
    J = Bj @ Bj.T / nx
    return (A, b, C, eta, J)


def _random_smoother_element(nx, rng):
    E = rng.standard_normal((nx, nx)) * 0.6
    g = rng.standard_normal(nx)
    Bl = rng.standard_normal((nx, nx))
    return (E, g, Bl @ Bl.T / nx)


def _close(x, y, tol=1e-12):
    return all(np.linalg.norm(a - b) <= tol * max(1.0, np.linalg.norm(b)) for a, b in zip(x, y))


def test_filter_operator_associative_and_identity():
    rng = np.random.default_rng(31)
    for nx in (1, 2, 4, 6):
        for _ in range(5):
            a, b, c = (_random_filter_element(nx, rng) for _ in range(3))
            lhs = el.filter_combine(el.filter_combine(a, b), c)
            rhs = el.filter_combine(a, el.filter_combine(b, c))
            assert _close(lhs, rhs, 1e-11)
            e = el.filter_identity(nx)
            assert _close(el.filter_combine(e, a), a, 0) and _close(el.filter_combine(a, e), a, 0)


def test_smoother_operator_associative_and_identity():
    rng = np.random.default_rng(32)
    for nx in (1, 3, 4):
        a, b, c = (_random_smoother_element(nx, rng) for _ in range(3))
        lhs = el.smoother_combine(el.smoother_combine(a, b), c)
        rhs = el.smoother_combine(a, el.smoother_combine(b, c))
        assert _close(lhs, rhs, 1e-13)
        e = el.smoother_identity(nx)
        assert _close(el.smoother_combine(e, a), a, 0) and _close(el.smoother_combine(a, e), a, 0)


def test_any_bracketing_gives_the_filter():
    """A balanced-tree bracketing of the elements equals the sequential filter (Section V claim)."""
    w = wl.workload(1, T=50)
    mo = w.model
    els = el.filter_elements(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y)
    items = [tuple(x[k] for x in els) for k in range(50)]
    while len(items) > 1:
        nxt = [el.filter_combine(items[i], items[i + 1]) for i in range(0, len(items) - 1, 2)]
        if len(items) % 2:
            nxt.append(items[-1])
        items = nxt
    ref = run(mo, w.y)
    assert np.linalg.norm(items[0][1] - ref["m"][-1]) <= 1e-12 * np.linalg.norm(ref["m"][-1])
    assert np.linalg.norm(items[0][2] - ref["P"][-1]) <= 1e-12 * np.linalg.norm(ref["P"][-1])
    assert np.array_equal(items[0][0], np.zeros((4, 4)))


def test_concatenated_sequences_reset_without_flags():
    """Element A_1 = 0 at a sequence start erases the left operand's f-part;
    E_n = 0 at a sequence end erases the right operand (Lemmas 1-4)."""
    w = wl.workload(4, B=3, T=100)
    ys, fel, ref = [], [], []
    for b in range(w.B):
        mo = w.model_of(b)
        yb = w.y[w.seq(b)]
        e = el.filter_elements(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, yb)
        fel.append(e)
        ref.append(run(mo, yb))
    cat = tuple(np.concatenate([e[i] for e in fel]) for i in range(5))
    m, P = el.filter_prefix_fold(cat)
    for b in range(w.B):
        s = w.seq(b)
        assert nerr(m[s], ref[b]["m"]) < 1e-12 and nerr(P[s], ref[b]["P"]) < 1e-12
    sel = [el.smoother_elements(w.model_of(b).F, w.model_of(b).Q, ref[b]["m"], ref[b]["P"])
           for b in range(w.B)]
    cat = tuple(np.concatenate([e[i] for e in sel]) for i in range(3))
    ms, Ps = el.smoother_suffix_fold(cat)
    for b in range(w.B):
        s = w.seq(b)
        assert nerr(ms[s], ref[b]["ms"]) < 1e-12 and nerr(Ps[s], ref[b]["Ps"]) < 1e-12


def _npdf(x, m, v):
    return np.exp(-0.5 * (x - m) ** 2 / v) / np.sqrt(2 * np.pi * v)


def test_lemma2_by_quadrature_scalar():
    """Definition 1 integrals evaluated on a grid (nx = 1) give Lemma 2's parameters."""
    Ai, bi, Ci, etai, Ji = 0.8, 0.3, 0.5, 0.7, 0.4
    Aj, bj, Cj, etaj, Jj = -0.6, 1.1, 0.3, -0.2, 1.3
    A, b, C, eta, J = (np.asarray(v).item() for v in el.filter_combine(
        tuple(np.atleast_2d(v) if k in (0, 2, 4) else np.atleast_1d(v)
              for k, v in enumerate((Ai, bi, Ci, etai, Ji))),
        tuple(np.atleast_2d(v) if k in (0, 2, 4) else np.atleast_1d(v)
              for k, v in enumerate((Aj, bj, Cj, etaj, Jj)))))
    yv = np.linspace(-30, 30, 60001)
    gj = np.exp(-0.5 * Jj * yv ** 2 + etaj * yv)
    logg = []
    zs = np.linspace(-2, 2, 9)
    for z in zs:
        fi = _npdf(yv, Ai * z + bi, Ci)
        den = np.trapezoid(gj * fi, yv)
        for x in (-1.3, 0.0, 0.9, 2.2):
            num = np.trapezoid(gj * _npdf(x, Aj * yv + bj, Cj) * fi, yv)
            assert abs(num / den - _npdf(x, A * z + b, C)) <= 1e-11
        gi = np.exp(-0.5 * Ji * z ** 2 + etai * z)
        logg.append(np.log(gi * den) - (-0.5 * J * z ** 2 + eta * z))
    assert np.ptp(logg) <= 1e-11


def test_lemma4_by_quadrature_scalar():
    Ei, gi, Li = 0.7, -0.4, 0.6
    Ej, gj, Lj = -1.2, 0.5, 0.2
    E, g, L = (np.asarray(v).item() for v in el.smoother_combine(
        (np.atleast_2d(Ei), np.atleast_1d(gi), np.atleast_2d(Li)),
        (np.atleast_2d(Ej), np.atleast_1d(gj), np.atleast_2d(Lj))))
    yv = np.linspace(-30, 30, 60001)
    for z in (-1.5, 0.2, 1.7):
        for x in (-2.0, -0.3, 0.8):
            val = np.trapezoid(_npdf(x, Ei * yv + gi, Li) * _npdf(yv, Ej * z + gj, Lj), yv)
            assert abs(val - _npdf(x, E * z + g, L)) <= 1e-12


def test_appendixC_identities_2d():
    """Appendix C: product and marginal identities, checked by log-density differences / 2-D quadrature."""
    rng = np.random.default_rng(9)
    n = 2
    Bm = rng.standard_normal((n, n))
    C = Bm @ Bm.T + 0.5 * np.eye(n)
    Bj = rng.standard_normal((n, n))
    J = Bj @ Bj.T * 0.5
    eta = rng.standard_normal(n)
    m = rng.standard_normal(n)

    def logN(x, mu, S):
        dlt = x - mu
        return -0.5 * dlt @ np.linalg.solve(S, dlt) - 0.5 * np.log(np.linalg.det(2 * np.pi * S))

    Ci = np.linalg.inv(C)
    S_post = np.linalg.inv(J + Ci)
    mu_post = S_post @ (eta + Ci @ m)
    diffs = []
    for _ in range(10):
        x = rng.standard_normal(n) * 2
        lhs = (-0.5 * x @ J @ x + eta @ x) + logN(x, m, C)
        diffs.append(lhs - logN(x, mu_post, S_post))
    assert np.ptp(diffs) < 1e-12
    # marginal identity, by quadrature on a 2-D grid
    A = rng.standard_normal((n, n)) * 0.5
    b = rng.standard_normal(n) * 0.3
    g1 = np.linspace(-12, 12, 801)
    Y1, Y2 = np.meshgrid(g1, g1, indexing="ij")
    Yg = np.stack([Y1, Y2], -1)
    h = g1[1] - g1[0]
    Minv = np.linalg.inv(np.eye(n) + J @ C)
    eta_z = A.T @ Minv @ (eta - J @ b)
    J_z = A.T @ Minv @ J @ A
    Ci_det = np.linalg.det(2 * np.pi * C)
    vals = []
    for z in rng.standard_normal((6, n)):
        mu = A @ z + b
        dlt = Yg - mu
        quad = np.einsum("...i,ij,...j->...", dlt, Ci, dlt)
        integrand = np.exp(-0.5 * np.einsum("...i,ij,...j->...", Yg, J, Yg) + Yg @ eta - 0.5 * quad) / np.sqrt(Ci_det)
        I = integrand.sum() * h * h
        vals.append(np.log(I) - (-0.5 * z @ J_z @ z + eta_z @ z))
    assert np.ptp(vals) < 1e-9


def test_prefix_sum_worked_example():
    """Section II-B example; also checks the tree scan with the root reset (Fig. 1 reading)."""
    g = json.load(open(os.path.join(GOLDEN, "prefix_sum_example.json")))
    a = list(g["a"])
    n = len(a)
    x = a[:]
    b = a[:]
    d = 1
    while d < n:                       # up-sweep, 0-based: x[k-1] <- x[j-1] + x[k-1]
        for i in range(0, n, 2 * d):
            x[i + 2 * d - 1] = x[i + d - 1] + x[i + 2 * d - 1]
        d *= 2
    x[n - 1] = 0                       # root reset (missing in the printed figure)
    d = n // 2
    while d >= 1:
        for i in range(0, n, 2 * d):
            t = x[i + d - 1]
            x[i + d - 1] = x[i + 2 * d - 1]
            x[i + 2 * d - 1] = x[i + 2 * d - 1] + t
        d //= 2
    x = [x[i] + b[i] for i in range(n)]
    assert x == g["prefix_sums"]
    assert list(np.cumsum(a)) == g["prefix_sums"]


# ---------------------------------------------------------------------------
# marginal likelihood (Section III-C): the per-step factors p(y_k | y_1:k-1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,T,singQ", DENSE_CASES)
def test_oracle_loglik_matches_dense_joint_density(nx, ny, T, singQ):
    """The running sum of the oracle's log factors equals the dense Gaussian
    log-density of y_1..y_k for every k (chain rule of the joint density)."""
    rng = np.random.default_rng(2000 + 17 * nx + 3 * ny + T)
    model = wl.random_small_model(nx, ny, rng, singular_Q=singQ)
    y, _ = wl.simulate(model, T, rng)
    out = run(model, y, loglik=True)
    cum, tot = oracle.loglik_prefix(out["ll"])
    ref = joint_loglik(model.F, model.Q, model.H, model.R, model.m0, model.P0, y, model.u, model.d)
    assert np.max(np.abs(cum - ref) / np.maximum(1.0, np.abs(ref))) < 1e-10
    assert tot[0] == cum[-1]


def test_oracle_loglik_cv_model_matches_dense_joint_density():
    w = wl.workload(1, T=30)
    out = run(w.model, w.y, loglik=True)
    cum, _ = oracle.loglik_prefix(out["ll"])
    ref = joint_loglik(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0, w.model.P0, w.y)
    assert np.max(np.abs(cum - ref) / np.maximum(1.0, np.abs(ref))) < 1e-10


def test_oracle_loglik_scalar_first_step_closed_form():
    """T = 1, nx = ny = 1: y_1 ~ N(h (f m0 + u) + d, h^2 (f^2 p0 + q) + r)."""
    f, q, h, r, m0, p0, u, d, y1 = 0.9, 0.3, 1.7, 0.2, 0.4, 2.0, 0.25, -0.1, 1.3
    one = lambda v: np.array([[v]])
    out = oracle.kf_rts(one(f), one(q), one(h), one(r), np.array([m0]), one(p0), np.array([[y1]]),
                        u=np.array([u]), d=np.array([d]), loglik=True)
    mu = h * (f * m0 + u) + d
    var = h * h * (f * f * p0 + q) + r
    ref = -0.5 * (np.log(2 * np.pi * var) + (y1 - mu) ** 2 / var)
    assert abs(out["ll"][0] - ref) < 1e-14 * abs(ref)


def test_oracle_loglik_static_model_closed_form():
    """F = I, Q = 0, u = 0: y_k = H x + d + r_k with one x ~ N(m0, P0), so
    y_1..y_k ~ N(1 (x) (H m0 + d), (1 1^T) (x) (H P0 H^T) + I (x) R); the
    density of that block matrix is evaluated by the matrix determinant lemma
    and the Woodbury identity, without forming it."""
    rng = np.random.default_rng(7)
    nx, ny, T = 3, 2, 9
    model = wl.random_small_model(nx, ny, rng)
    F, Q = np.eye(nx), np.zeros((nx, nx))
    H, R, m0, P0 = model.H, model.R, model.m0, model.P0
    y = rng.standard_normal((T, ny))
    out = oracle.kf_rts(F, Q, H, R, m0, P0, y, loglik=True)
    cum, _ = oracle.loglik_prefix(out["ll"])
    Ri = np.linalg.inv(R)
    for k in range(1, T + 1):
        r = y[:k] - (H @ m0)                      # k x ny residuals
        # Sigma = I_k (x) R + U U^T with U = 1_k (x) (H L0), P0 = L0 L0^T
        L0 = np.linalg.cholesky(P0)
        HL = H @ L0
        M = np.eye(nx) + k * HL.T @ Ri @ HL       # I + U^T (I (x) R^-1) U
        logdet = k * np.linalg.slogdet(R)[1] + np.linalg.slogdet(M)[1]
        Rr = r @ Ri                               # rows (R^-1 r_i)^T
        v = HL.T @ Rr.sum(axis=0)                 # U^T (I (x) R^-1) r
        quad = np.sum(Rr * r) - v @ np.linalg.solve(M, v)
        ref = -0.5 * (k * ny * np.log(2 * np.pi) + logdet + quad)
        assert abs(cum[k - 1] - ref) < 1e-12 * max(1.0, abs(ref))


def test_oracle_loglik_batched_restarts_per_sequence():
    rng = np.random.default_rng(11)
    nx, ny, B = 3, 2, 5
    lens = [7, 0, 1, 12, 4]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    models = [wl.random_small_model(nx, ny, rng) for _ in range(B)]
    ys = [wl.simulate(mo, L, rng)[0] if L else np.zeros((0, ny)) for mo, L in zip(models, lens)]
    stack = lambda a: np.stack([getattr(mo, a) for mo in models])
    out = oracle.kf_rts_batched(stack("F"), stack("Q"), stack("H"), stack("R"), stack("m0"),
                                stack("P0"), np.concatenate(ys), offsets, per_sequence=True,
                                smooth=False, loglik=True, threads=2)
    cum, tot = oracle.loglik_prefix(out["ll"], offsets)
    for b in range(B):
        if lens[b] == 0:
            assert tot[b] == 0.0
            continue
        mo = models[b]
        ref = joint_loglik(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, ys[b])
        sl = slice(offsets[b], offsets[b + 1])
        assert np.max(np.abs(cum[sl] - ref) / np.maximum(1.0, np.abs(ref))) < 1e-10
        assert tot[b] == cum[offsets[b + 1] - 1]



def test_loglik_factors_from_oracle_moments_match_dense_joint_density():
    """The extended-precision factors, fed the oracle's own filtered moments,
    sum to the dense Gaussian log-density of y_1..y_k (chain rule), for models
    with u, d, singular Q and several sequences with their own models."""
    rng = np.random.default_rng(31)
    for nx, ny, T, singQ in ((1, 1, 9, False), (3, 2, 17, True), (4, 4, 12, False), (2, 3, 20, False)):
        model = wl.random_small_model(nx, ny, rng, singular_Q=singQ)
        model = wl.Model(model.F, model.Q, model.H, model.R, model.m0, model.P0,
                         rng.standard_normal(nx), rng.standard_normal(ny))
        y, _ = wl.simulate(model, T, rng)
        out = run(model, y)
        f = oracle.loglik_factors(model.F, model.Q, model.H, model.R, model.m0, model.P0, y, out["m"], out["P"],
                                  u=model.u, d=model.d)
        ref = joint_loglik(model.F, model.Q, model.H, model.R, model.m0, model.P0, y, model.u, model.d)
        assert np.max(np.abs(np.cumsum(f) - ref) / np.maximum(1.0, np.abs(ref))) < 1e-10
    # per-sequence models: each sequence restarts from its own prior
    lens = [5, 0, 1, 9]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    models = [wl.random_small_model(3, 2, rng) for _ in lens]
    ys = [wl.simulate(mo, L, rng)[0] if L else np.zeros((0, 2)) for mo, L in zip(models, lens)]
    stack = lambda a: np.stack([getattr(mo, a) for mo in models])
    y = np.concatenate(ys)
    out = oracle.kf_rts_batched(stack("F"), stack("Q"), stack("H"), stack("R"), stack("m0"), stack("P0"), y,
                                offsets, per_sequence=True, smooth=False, threads=2)
    f = oracle.loglik_factors(stack("F"), stack("Q"), stack("H"), stack("R"), stack("m0"), stack("P0"), y,
                              out["m"], out["P"], offsets=offsets, per_sequence=True)
    for b, mo in enumerate(models):
        if lens[b]:
            sl = slice(offsets[b], offsets[b + 1])
            ref = joint_loglik(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, ys[b])
            assert np.max(np.abs(np.cumsum(f[sl]) - ref) / np.maximum(1.0, np.abs(ref))) < 1e-10


def test_loglik_factors_scalar_closed_form_at_large_state():
    """nx = ny = 1 with a filtered mean of 1e7 and a residual of order one: the
    factor log N(y; h (f m + u) + d, h^2 (f^2 p + q) + r) evaluated in exact
    rational arithmetic (fractions of the float64 inputs), then rounded.  A
    float64 evaluation of the residual would lose about seven digits here."""
    from fractions import Fraction as Fr
    import math
    f, q, h, r, u, d = 1.0, 1e-3, 1.0 + 2.0 ** -30, 0.25, 0.125, -0.375
    m_prev = np.array([[12345678.123456789]])
    p_prev = np.array([[[0.0625]]])
    mu = h * (f * m_prev[0, 0] + u) + d
    y = np.array([[mu + 0.731]])
    one = lambda v: np.array([[v]])
    # the first step uses the prior: make the prior the given moments
    got = oracle.loglik_factors(one(f), one(q), one(h), one(r), m_prev[0], p_prev[0], y,
                                np.zeros((1, 1)), np.zeros((1, 1, 1)), u=np.array([u]), d=np.array([d]))[0]
    F_, H_, m_ = Fr(f), Fr(h), Fr(m_prev[0, 0])
    res = Fr(y[0, 0]) - (H_ * (F_ * m_ + Fr(u)) + Fr(d))
    var = H_ * H_ * (F_ * F_ * Fr(p_prev[0, 0, 0]) + Fr(q)) + Fr(r)
    ref = -0.5 * (math.log(2 * math.pi) + math.log(float(var)) + float(res * res / var))
    # bar: the extended format's rounding (2^-64) of terms of size |h f m|,
    # through the gradient v = res / var, plus a float64 rounding of the result
    ext = 16 * 2.0 ** -64 * abs(float(res / var)) * abs(h * f * m_prev[0, 0])
    assert abs(got - ref) <= ext + 4e-16 * abs(ref)
    # and a plain float64 residual really is off at this size (what the
    # extended evaluation is for): its error is well above that bar
    naive = y[0, 0] - (h * (f * m_prev[0, 0] + u) + d)
    assert abs(naive - float(res)) * abs(float(1 / var)) > 10 * ext


def test_loglik_factors_detect_a_planted_offset():
    """A shift of one filtered mean by 1e-9 of its size changes exactly the
    next factor, by the first-order amount (G^T v) . dm."""
    w = wl.workload(1, T=200)
    mo = w.model
    out = run(mo, w.y)
    f0 = oracle.loglik_factors(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y, out["m"], out["P"])
    m1 = out["m"].copy()
    dm = 1e-9 * np.abs(m1[120]) + 1e-12
    m1[120] += dm
    f1 = oracle.loglik_factors(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y, m1, out["P"])
    changed = np.nonzero(f1 != f0)[0]
    assert list(changed) == [121]
    G = mo.H @ mo.F
    S = G @ out["P"][120] @ G.T + mo.H @ mo.Q @ mo.H.T + mo.R
    r = w.y[121] - G @ out["m"][120]
    v = np.linalg.solve(S, r)
    assert abs((f1[121] - f0[121]) - v @ (G @ dm)) <= 1e-6 * abs(v @ (G @ dm))


# ---------------------------------------------------------------------------
# time-varying models (Section IV's general model, one row per step)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,T", [(1, 1, 7), (2, 1, 12), (3, 2, 15), (4, 2, 10), (5, 3, 8)])
def test_oracle_tv_matches_dense_joint_posterior(nx, ny, T):
    """Per-step F, Q, u, H, R, d: the recursion against the dense joint
    Gaussian built from the products F_{k-1} ... F_i, including the
    log-likelihood of every prefix."""
    rng = np.random.default_rng(3000 + 31 * nx + ny + T)
    model = wl.random_tv_model(nx, ny, T, rng)
    y, _ = wl.simulate_tv(model, rng)
    out = oracle.kf_rts_tv(model.F, model.Q, model.H, model.R, model.m0, model.P0, y, u=model.u, d=model.d,
                           loglik=True)
    m, P, ms, Ps, ll = posterior_tv(model.F, model.Q, model.H, model.R, model.m0, model.P0, y, model.u, model.d)
    for key, ref in (("m", m), ("P", P), ("ms", ms), ("Ps", Ps)):
        assert nerr(out[key], ref) < 1e-10, key
    cum, _ = oracle.loglik_prefix(out["ll"])
    assert np.max(np.abs(cum - ll) / np.maximum(1.0, np.abs(ll))) < 1e-10


def test_oracle_tv_irregular_cv_matches_dense():
    w = wl.workload(6, T=25)
    mo = w.model
    out = oracle.kf_rts_tv(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y, loglik=True)
    m, P, ms, Ps, ll = posterior_tv(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y)
    for key, ref in (("m", m), ("P", P), ("ms", ms), ("Ps", Ps)):
        assert nerr(out[key], ref) < 1e-10, key


def test_oracle_tv_with_equal_rows_is_the_time_invariant_recursion():
    """Every row the same model: bitwise the time-invariant result."""
    rng = np.random.default_rng(12)
    mo = wl.random_small_model(3, 2, rng)
    T = 50
    y, _ = wl.simulate(mo, T, rng)
    rep = lambda a: np.broadcast_to(a, (T,) + a.shape).copy()
    tv = oracle.kf_rts_tv(rep(mo.F), rep(mo.Q), rep(mo.H), rep(mo.R), mo.m0, mo.P0, y, u=rep(mo.u),
                          d=rep(mo.d), loglik=True)
    ti = run(mo, y, loglik=True)
    for key in ("m", "P", "ms", "Ps", "ll"):
        assert np.array_equal(tv[key], ti[key]), key


def test_irregular_cv_model_constants():
    """Workload 6's per-step model is the constant-velocity model of its own
    interval (the Section V matrices with dt_k in place of dt)."""
    w = wl.workload(6, T=5)
    dts = w.model.F[:, 0, 2].copy()
    for k in range(5):
        ref = wl.cv_model(1.0, 0.25, dt=dts[k])
        assert np.allclose(w.model.F[k], ref.F, rtol=0, atol=0)
        assert np.allclose(w.model.Q[k], ref.Q, rtol=1e-15, atol=0)
    assert np.all((dts >= 0.05) & (dts <= 0.15))


# ---------------------------------------------------------------------------
# discrete-state hidden Markov model (the framework with the counting measure)
# ---------------------------------------------------------------------------
from oracle import hmm_elements as hel  # noqa: E402


def _random_hmm(K, T, rng, sparse=False):
    Pi = rng.random((K, K)) + 0.05
    if sparse:
        Pi *= rng.random((K, K)) < 0.5
        Pi[np.arange(K), np.arange(K)] += 0.1        # every row keeps a way out
    Pi /= Pi.sum(axis=1, keepdims=True)
    p0 = rng.random(K) + 0.1
    p0 /= p0.sum()
    L = rng.normal(0.0, 1.5, size=(T, K))
    return Pi, p0, L


def _hmm_brute_force(Pi, p0, L):
    """Sum over every state path x_0..x_T of p0[x_0] prod Pi[x_{k-1}][x_k]
    exp(L[k-1][x_k]): filtered and smoothed marginals and log p(y_1:k)."""
    import itertools
    K = Pi.shape[0]
    T = L.shape[0]
    alpha = np.zeros((T, K))
    gamma = np.zeros((T, K))
    logp = np.zeros(T)
    for k in range(1, T + 1):                        # data y_1..y_k
        acc = np.zeros(K)
        tot = 0.0
        for path in itertools.product(range(K), repeat=k + 1):
            w = p0[path[0]]
            for t in range(1, k + 1):
                w *= Pi[path[t - 1], path[t]] * np.exp(L[t - 1, path[t]])
            acc[path[k]] += w
            tot += w
            if k == T:
                for t in range(1, T + 1):
                    gamma[t - 1, path[t]] += w
        alpha[k - 1] = acc / tot
        logp[k - 1] = np.log(tot)
        if k == T:
            gamma /= tot
    return alpha, gamma, logp


@pytest.mark.parametrize("K,T,sparse", [(2, 1, False), (2, 4, False), (3, 5, False), (3, 4, True), (4, 3, False)])
def test_hmm_oracle_matches_brute_force(K, T, sparse):
    rng = np.random.default_rng(70 + 10 * K + T)
    Pi, p0, L = _random_hmm(K, T, rng, sparse)
    out = oracle.hmm_fb(Pi, p0, L)
    a, g, lp = _hmm_brute_force(Pi, p0, L)
    assert np.max(np.abs(out["alpha"] - a)) < 1e-13
    assert np.max(np.abs(out["gamma"] - g)) < 1e-13
    assert np.max(np.abs(np.cumsum(out["ll"]) - lp)) < 1e-12 * max(1.0, np.max(np.abs(lp)))


def test_hmm_oracle_two_state_by_hand():
    """Two states, two steps, numbers worked by hand:
    pred_1 = p0 Pi = (0.55, 0.45); u_1 = pred_1 * (0.3, 0.6) = (0.165, 0.27),
    p(y_1) = 0.435; pred_2 = alpha_1 Pi; gamma_1 from the backward equation."""
    Pi = np.array([[0.9, 0.1], [0.2, 0.8]])
    p0 = np.array([0.5, 0.5])
    lik = np.array([[0.3, 0.6], [0.5, 0.1]])
    out = oracle.hmm_fb(Pi, p0, np.log(lik))
    a1 = np.array([0.165, 0.27]) / 0.435
    assert np.allclose(out["alpha"][0], a1, rtol=0, atol=1e-15)
    assert abs(out["ll"][0] - np.log(0.435)) < 1e-15
    pred2 = np.array([a1[0] * 0.9 + a1[1] * 0.2, a1[0] * 0.1 + a1[1] * 0.8])
    u2 = pred2 * lik[1]
    a2 = u2 / u2.sum()
    assert np.allclose(out["alpha"][1], a2, rtol=0, atol=1e-15)
    assert abs(out["ll"][1] - np.log(u2.sum())) < 1e-15
    g1 = a1 * np.array([0.9 * a2[0] / pred2[0] + 0.1 * a2[1] / pred2[1],
                        0.2 * a2[0] / pred2[0] + 0.8 * a2[1] / pred2[1]])
    assert np.allclose(out["gamma"][0], g1, rtol=0, atol=1e-15)
    assert np.array_equal(out["gamma"][1], out["alpha"][1])


def test_hmm_oracle_deterministic_cycle():
    """A cyclic permutation Pi[i][(i+1) % K] = 1 with x_0 = 0 known: x_k = k mod K
    whatever the measurements, so filtered = smoothed = that indicator and
    log p(y_1:T) = sum_k L[k-1][k mod K].  A transposed Pi would run the cycle
    backwards."""
    K, T = 5, 23
    Pi = np.roll(np.eye(K), 1, axis=1)
    p0 = np.eye(K)[0]
    L = np.random.default_rng(3).normal(size=(T, K))
    out = oracle.hmm_fb(Pi, p0, L)
    ind = np.eye(K)[np.arange(1, T + 1) % K]
    assert np.array_equal(out["alpha"], ind) and np.array_equal(out["gamma"], ind)
    assert abs(out["ll"].sum() - L[np.arange(T), np.arange(1, T + 1) % K].sum()) < 1e-12


def test_hmm_oracle_invariants():
    """Marginals sum to one, gamma_T = alpha_T bitwise, and a constant added to
    one step's log-likelihoods moves only that step's factor, by the constant."""
    rng = np.random.default_rng(12)
    Pi, p0, L = _random_hmm(6, 300, rng, sparse=True)
    out = oracle.hmm_fb(Pi, p0, L)
    assert np.max(np.abs(out["alpha"].sum(axis=1) - 1)) < 1e-14
    assert np.max(np.abs(out["gamma"].sum(axis=1) - 1)) < 1e-13
    assert np.array_equal(out["gamma"][-1], out["alpha"][-1])
    L2 = L.copy()
    L2[100] += 7.25
    out2 = oracle.hmm_fb(Pi, p0, L2)
    d = out2["ll"] - out["ll"]
    assert abs(d[100] - 7.25) < 1e-13 and np.max(np.abs(np.delete(d, 100))) < 1e-13
    assert np.max(np.abs(out2["alpha"] - out["alpha"])) < 1e-14
    assert np.max(np.abs(out2["gamma"] - out["gamma"])) < 1e-14


@pytest.mark.parametrize("sparse", [False, True])
def test_hmm_elements_fold_equals_forward_backward(sparse):
    """Theorems 1-2 with sums: the left fold of the filtering elements under
    Definition 1 gives the filtered marginals and log p(y_1:k); the right fold
    of the smoothing elements under Definition 2 the smoothed marginals."""
    rng = np.random.default_rng(5 if sparse else 6)
    Pi, p0, L = _random_hmm(5, 40, rng, sparse)
    out = oracle.hmm_fb(Pi, p0, L)
    f, g = hel.filter_elements(Pi, p0, L)
    alpha, logp = hel.filter_prefix_fold(f, g)
    assert np.max(np.abs(alpha - out["alpha"])) < 1e-13
    assert np.max(np.abs(logp - np.cumsum(out["ll"]))) < 1e-11
    a = hel.smoother_elements(Pi, out["alpha"])
    gamma = hel.smoother_suffix_fold(a)
    assert np.max(np.abs(gamma - out["gamma"])) < 1e-13


def test_hmm_operators_associative_with_identity_and_any_bracketing():
    rng = np.random.default_rng(8)
    Pi, p0, L = _random_hmm(4, 9, rng)
    f, g = hel.filter_elements(Pi, p0, L)
    e = hel.filter_identity(4)
    for i in range(1, 7):
        x, y, z = (f[i], g[i]), (f[i + 1], g[i + 1]), (f[i + 2], g[i + 2])
        l = hel.filter_combine(*hel.filter_combine(*x, *y), *z)
        r = hel.filter_combine(*x, *hel.filter_combine(*y, *z))
        assert np.max(np.abs(l[0] - r[0])) < 1e-14 and np.max(np.abs(l[1] / r[1] - 1)) < 1e-14
        for a_, b_ in (hel.filter_combine(*x, *e), hel.filter_combine(*e, *x)):
            assert np.max(np.abs(a_ - x[0])) < 1e-15 and np.max(np.abs(b_ / x[1] - 1)) < 1e-15
    # a balanced tree gives the sequential result
    pairs = [(f[k], g[k]) for k in range(8)]
    while len(pairs) > 1:
        pairs = [hel.filter_combine(*pairs[2 * i], *pairs[2 * i + 1]) for i in range(len(pairs) // 2)]
    out = oracle.hmm_fb(Pi, p0, L[:8])
    assert np.max(np.abs(pairs[0][0][0] - out["alpha"][7])) < 1e-14
    assert abs(np.log(pairs[0][1][0]) - out["ll"].sum()) < 1e-12
    a = hel.smoother_elements(Pi, oracle.hmm_fb(Pi, p0, L)["alpha"])
    for i in range(6):
        l = hel.smoother_combine(hel.smoother_combine(a[i], a[i + 1]), a[i + 2])
        r = hel.smoother_combine(a[i], hel.smoother_combine(a[i + 1], a[i + 2]))
        assert np.max(np.abs(l - r)) < 1e-15
