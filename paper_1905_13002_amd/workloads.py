"""Seeded synthetic inputs: state-space models and simulated measurements.

This module holds no filtering or smoothing arithmetic.  It builds model
matrices and simulates the linear/Gaussian model
    x_0 ~ N(m0, P0),  x_k = F x_{k-1} + u + q_{k-1},  y_k = H x_k + d + r_k
with numpy's PCG64 generator seeded by
``SeedSequence([190513002, workload_id, sequence_index])``.  Both the GPU
path's tests/benchmark and the CPU oracle receive the arrays it returns.

Workloads (ids 1..5):
  1  2-D constant-velocity tracking (the paper's Section V model, with
     q = 1, sigma^2 = 0.25, dt = 0.1, m0 = 0, P0 = I), T = 1024
  2  the same model, T = 2**20
  3  random stable model nx = 16, ny = 8, T = 2**16
  4  4096 constant-velocity sequences of uneven length (256..16384) with
     per-sequence q in [0.1, 10] and r in [0.01, 1]
  5  64 sequences of a shared nx = 64, ny = 32 random stable model, T = 8192
  6  time-varying model: 2-D constant-velocity tracking sampled at irregular
     times (dt_k ~ U(0.05, 0.15), so F_{k-1} and Q_{k-1} change every step),
     q = 1, sigma^2 = 0.25, T = 2**20

Discrete-state hidden Markov model inputs (:func:`hmm_workload`): a sticky
transition matrix, a uniform prior and Gaussian emissions y_k ~ N(mu_{x_k}, 1)
with mu_j = j / 2; the inputs of the method are the emission log-likelihoods
L[k-1][j] = log N(y_k; mu_j, 1).  Workload 7: K = 64 states, T = 2**16.

A time-varying model is a Model whose F, Q, H, R (and u, d) carry a leading
[T] axis: row k-1 holds the transition into step k (F_{k-1}, Q_{k-1}, u_{k-1})
and the measurement model of step k (H_k, R_k, d_k).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_ROOT = 190513002


def rng_for(workload: int, seq: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, int(workload), int(seq)]))


@dataclass
class Model:
    """Time-invariant linear/Gaussian model (float64, row-major numpy arrays).

    For B stacked per-sequence models every array carries a leading [B] axis.
    """
    F: np.ndarray
    Q: np.ndarray
    H: np.ndarray
    R: np.ndarray
    m0: np.ndarray
    P0: np.ndarray
    u: Optional[np.ndarray] = None
    d: Optional[np.ndarray] = None

    @property
    def nx(self) -> int:
        return self.F.shape[-1]

    @property
    def ny(self) -> int:
        return self.H.shape[-2]

    def select(self, b: int) -> "Model":
        """Model b of a stacked set."""
        pick = lambda a: None if a is None else a[b]
        return Model(self.F[b], self.Q[b], self.H[b], self.R[b], self.m0[b], self.P0[b],
                     pick(self.u), pick(self.d))


@dataclass
class Workload:
    name: str
    model: Model
    y: np.ndarray                       # [total, ny] float64
    offsets: np.ndarray                 # [B+1] int64
    per_sequence: bool = False
    x: Optional[np.ndarray] = None      # simulated states (kept only when asked)
    meta: dict = field(default_factory=dict)
    time_varying: bool = False          # model rows per step (single sequence)

    @property
    def B(self) -> int:
        return len(self.offsets) - 1

    @property
    def total(self) -> int:
        return int(self.offsets[-1])

    def model_of(self, b: int) -> Model:
        return self.model.select(b) if self.per_sequence else self.model

    def seq(self, b: int) -> slice:
        return slice(int(self.offsets[b]), int(self.offsets[b + 1]))


# ---------------------------------------------------------------------------
# model builders
# ---------------------------------------------------------------------------

def cv_model(q: float = 1.0, r: float = 0.25, dt: float = 0.1,
             m0=(0.0, 0.0, 0.0, 0.0), P0=None) -> Model:
    """2-D constant-velocity tracking model, state (u, v, du, dv), measuring (u, v).

    F, Q (white-acceleration noise with spectral density q) and H as printed in
    the paper's Section V; R = r * I with r the measurement variance.
    """
    I2 = np.eye(2)
    Z2 = np.zeros((2, 2))
    F = np.block([[I2, dt * I2], [Z2, I2]])
    Q = q * np.block([[dt ** 3 / 3 * I2, dt ** 2 / 2 * I2], [dt ** 2 / 2 * I2, dt * I2]])
    H = np.hstack([I2, Z2])
    R = r * I2
    m0 = np.asarray(m0, dtype=np.float64)
    P0 = np.eye(4) if P0 is None else np.asarray(P0, dtype=np.float64)
    return Model(F, Q, H, R, m0, P0)


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix (QR of a Gaussian matrix, signs fixed)."""
    Z = rng.standard_normal((n, n))
    Qm, Rm = np.linalg.qr(Z)
    return Qm * np.sign(np.diag(Rm))[None, :]


def spd_with_condition(n: int, rng: np.random.Generator, cond: float = 1e2,
                       top: float = 1.0) -> np.ndarray:
    """V diag(logspace(log10 top, log10(top/cond), n)) V^T with V Haar."""
    V = haar_orthogonal(n, rng)
    ev = np.logspace(np.log10(top), np.log10(top / cond), n) if n > 1 else np.array([top])
    X = (V * ev[None, :]) @ V.T
    return 0.5 * (X + X.T)


def random_stable_model(nx: int, ny: int, rng: np.random.Generator, radius: float = 0.99,
                        q_scale: float = 1.0, r_scale: float = 1.0, cond: float = 1e2,
                        with_offsets: bool = False) -> Model:
    F = radius * haar_orthogonal(nx, rng)
    H = rng.standard_normal((ny, nx)) / np.sqrt(nx)
    Q = spd_with_condition(nx, rng, cond, q_scale)
    R = spd_with_condition(ny, rng, cond, r_scale)
    m0 = np.zeros(nx)
    P0 = np.eye(nx)
    u = d = None
    if with_offsets:
        u = 0.1 * rng.standard_normal(nx)
        d = 0.1 * rng.standard_normal(ny)
        m0 = rng.standard_normal(nx)
        A0 = rng.standard_normal((nx, nx))
        P0 = A0 @ A0.T / nx + 0.5 * np.eye(nx)
    return Model(F, Q, H, R, m0, P0, u, d)


def random_small_model(nx: int, ny: int, rng: np.random.Generator,
                       singular_Q: bool = False, with_offsets: bool = True) -> Model:
    """A generic small model with non-trivial u, d, m0, P0 (for parity cases)."""
    F = rng.standard_normal((nx, nx)) / np.sqrt(nx)
    F = 0.97 * F / max(1.0, np.max(np.abs(np.linalg.eigvals(F))))
    H = rng.standard_normal((ny, nx))
    Bq = rng.standard_normal((nx, nx))
    Q = Bq @ Bq.T / nx + 0.05 * np.eye(nx)
    if singular_Q and nx > 1:
        Bq = rng.standard_normal((nx, 1))
        Q = Bq @ Bq.T
    Br = rng.standard_normal((ny, ny))
    R = Br @ Br.T / ny + 0.2 * np.eye(ny)
    m0 = rng.standard_normal(nx) if with_offsets else np.zeros(nx)
    B0 = rng.standard_normal((nx, nx))
    P0 = B0 @ B0.T / nx + 0.3 * np.eye(nx)
    u = 0.3 * rng.standard_normal(nx) if with_offsets else None
    d = 0.3 * rng.standard_normal(ny) if with_offsets else None
    return Model(F, Q, H, R, m0, P0, u, d)


def cv_model_tv(dts: np.ndarray, q: float = 1.0, r: float = 0.25, m0=None, P0=None) -> Model:
    """Constant-velocity model sampled at irregular times: step k moves by
    dts[k-1] (F_{k-1}, Q_{k-1} of the white-acceleration model for that
    interval), H and R = r I unchanged.  Arrays carry a leading [T] axis."""
    dts = np.asarray(dts, dtype=np.float64)
    T = dts.shape[0]
    I2 = np.eye(2)
    F = np.zeros((T, 4, 4))
    F[:, :2, :2] = I2
    F[:, 2:, 2:] = I2
    F[:, :2, 2:] = dts[:, None, None] * I2
    Q = np.zeros((T, 4, 4))
    Q[:, :2, :2] = (q * dts ** 3 / 3)[:, None, None] * I2
    Q[:, :2, 2:] = (q * dts ** 2 / 2)[:, None, None] * I2
    Q[:, 2:, :2] = (q * dts ** 2 / 2)[:, None, None] * I2
    Q[:, 2:, 2:] = (q * dts)[:, None, None] * I2
    H = np.broadcast_to(np.hstack([I2, np.zeros((2, 2))]), (T, 2, 4)).copy()
    R = np.broadcast_to(r * I2, (T, 2, 2)).copy()
    m0 = np.zeros(4) if m0 is None else np.asarray(m0, dtype=np.float64)
    P0 = np.eye(4) if P0 is None else np.asarray(P0, dtype=np.float64)
    return Model(F, Q, H, R, m0, P0)


def random_tv_model(nx: int, ny: int, T: int, rng: np.random.Generator, radius: float = 0.97,
                    with_offsets: bool = True) -> Model:
    """A generic time-varying model: per step a random F_{k-1} (spectral radius
    <= radius), SPD Q_{k-1}, R_k, a random H_k and (optionally) u_{k-1}, d_k."""
    F = rng.standard_normal((T, nx, nx)) / np.sqrt(nx)
    rad = np.max(np.abs(np.linalg.eigvals(F)), axis=1)
    F = radius * F / np.maximum(1.0, rad)[:, None, None]
    Bq = rng.standard_normal((T, nx, nx))
    Q = Bq @ np.swapaxes(Bq, 1, 2) / nx + 0.05 * np.eye(nx)
    H = rng.standard_normal((T, ny, nx)) / np.sqrt(nx)
    Br = rng.standard_normal((T, ny, ny))
    R = Br @ np.swapaxes(Br, 1, 2) / ny + 0.2 * np.eye(ny)
    m0 = rng.standard_normal(nx) if with_offsets else np.zeros(nx)
    B0 = rng.standard_normal((nx, nx))
    P0 = B0 @ B0.T / nx + 0.3 * np.eye(nx)
    u = 0.3 * rng.standard_normal((T, nx)) if with_offsets else None
    d = 0.3 * rng.standard_normal((T, ny)) if with_offsets else None
    return Model(F, Q, H, R, m0, P0, u, d)


# ---------------------------------------------------------------------------
# simulation
# ---------------------------------------------------------------------------

def _chol_psd(X: np.ndarray) -> np.ndarray:
    """A factor L with L L^T = X for symmetric PSD X (eigen-decomposition, robust to rank loss)."""
    w, V = np.linalg.eigh(0.5 * (X + X.T))
    return V * np.sqrt(np.clip(w, 0.0, None))[None, :]


def simulate(model: Model, T: int, rng: np.random.Generator, keep_states: bool = False):
    """Simulate one sequence of length T: returns (y [T,ny], x [T,nx] or None)."""
    nx, ny = model.nx, model.ny
    LQ, LR, L0 = _chol_psd(model.Q), _chol_psd(model.R), _chol_psd(model.P0)
    u = np.zeros(nx) if model.u is None else model.u
    d = np.zeros(ny) if model.d is None else model.d
    x = model.m0 + L0 @ rng.standard_normal(nx)
    qn = rng.standard_normal((T, nx)) @ LQ.T
    rn = rng.standard_normal((T, ny)) @ LR.T
    xs = np.empty((T, nx))
    F = model.F
    for k in range(T):
        x = F @ x + u + qn[k]
        xs[k] = x
    y = xs @ model.H.T + d + rn
    return y, (xs if keep_states else None)


def simulate_tv(model: Model, rng: np.random.Generator, keep_states: bool = False):
    """Simulate a time-varying model over its T rows: returns (y [T,ny], x or None)."""
    T, nx, ny = model.F.shape[0], model.nx, model.ny
    x = model.m0 + _chol_psd(model.P0) @ rng.standard_normal(nx)
    w, V = np.linalg.eigh(0.5 * (model.Q + np.swapaxes(model.Q, 1, 2)))
    LQ = V * np.sqrt(np.clip(w, 0.0, None))[:, None, :]
    w, V = np.linalg.eigh(0.5 * (model.R + np.swapaxes(model.R, 1, 2)))
    LR = V * np.sqrt(np.clip(w, 0.0, None))[:, None, :]
    qn = np.einsum("kij,kj->ki", LQ, rng.standard_normal((T, nx)))
    rn = np.einsum("kij,kj->ki", LR, rng.standard_normal((T, ny)))
    u = np.zeros((T, nx)) if model.u is None else model.u
    d = np.zeros((T, ny)) if model.d is None else model.d
    xs = np.empty((T, nx))
    for k in range(T):
        x = model.F[k] @ x + u[k] + qn[k]
        xs[k] = x
    y = np.einsum("kij,kj->ki", model.H, xs) + d + rn
    return y, (xs if keep_states else None)


def simulate_cv_tv(dts: np.ndarray, q: float, r: float, rng: np.random.Generator, keep_states: bool = False):
    """Constant-velocity simulation at irregular intervals dts, vectorised: per
    axis the interval's noise (q dt^3/3, q dt^2/2; q dt^2/2, q dt) is drawn
    through its closed-form Cholesky factor."""
    dts = np.asarray(dts, dtype=np.float64)
    T = dts.shape[0]
    x0 = rng.standard_normal(4)                              # m0 = 0, P0 = I
    z = rng.standard_normal((T, 2, 2))                       # [k, axis, (pos, vel)]
    l11 = np.sqrt(q * dts ** 3 / 3)
    l21 = np.sqrt(3 * q * dts) / 2
    l22 = np.sqrt(q * dts / 4)
    qp = l11[:, None] * z[:, :, 0]
    qv = l21[:, None] * z[:, :, 0] + l22[:, None] * z[:, :, 1]
    v = x0[2:] + np.cumsum(qv, axis=0)
    v_prev = np.vstack([x0[2:][None, :], v[:-1]])
    p = x0[:2] + np.cumsum(dts[:, None] * v_prev + qp, axis=0)
    y = p + np.sqrt(r) * rng.standard_normal((T, 2))
    return y, (np.hstack([p, v]) if keep_states else None)


def simulate_cv(q: float, r: float, T: int, rng: np.random.Generator, dt: float = 0.1,
                m0=None, P0=None, keep_states: bool = False):
    """Constant-velocity simulation, vectorised (velocity is a random walk, position its sum)."""
    model = cv_model(q, r, dt)
    m0 = np.zeros(4) if m0 is None else np.asarray(m0, dtype=np.float64)
    P0 = np.eye(4) if P0 is None else np.asarray(P0, dtype=np.float64)
    x0 = m0 + _chol_psd(P0) @ rng.standard_normal(4)
    qn = rng.standard_normal((T, 4)) @ _chol_psd(model.Q).T
    rn = np.sqrt(r) * rng.standard_normal((T, 2))
    # v_k = v_{k-1} + qv_{k-1};  p_k = p_{k-1} + dt v_{k-1} + qp_{k-1}
    v = x0[2:] + np.cumsum(qn[:, 2:], axis=0)
    v_prev = np.vstack([x0[2:][None, :], v[:-1]])
    p = x0[:2] + np.cumsum(dt * v_prev + qn[:, :2], axis=0)
    y = p + rn
    xs = np.hstack([p, v]) if keep_states else None
    return y, xs


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

WORKLOAD_NAMES = {
    1: "cv_T1024",
    2: "cv_T1048576",
    3: "random_nx16_ny8_T65536",
    4: "cv_batched_B4096_uneven",
    5: "random_nx64_ny32_B64_T8192",
    6: "cv_irregular_T1048576",
    7: "hmm_K64_T65536",
}


def _single(name, model, y, x=None, **meta):
    T = y.shape[0]
    return Workload(name, model, np.ascontiguousarray(y), np.array([0, T], dtype=np.int64),
                    False, x, meta)


def workload(wid: int, keep_states: bool = False, T: Optional[int] = None,
             B: Optional[int] = None) -> Workload:
    """Build workload ``wid``; ``T``/``B`` override the length/count for reduced tests."""
    if wid in (1, 2):
        T = T if T is not None else (1024 if wid == 1 else 1 << 20)
        rng = rng_for(wid, 0)
        model = cv_model(1.0, 0.25)
        y, x = simulate_cv(1.0, 0.25, T, rng, keep_states=keep_states)
        return _single(WORKLOAD_NAMES[wid], model, y, x, q=1.0, r=0.25, dt=0.1)
    if wid == 3:
        T = T if T is not None else 1 << 16
        rng = rng_for(3, 0)
        model = random_stable_model(16, 8, rng, radius=0.99)
        y, x = simulate(model, T, rng_for(3, 1), keep_states)
        return _single(WORKLOAD_NAMES[3], model, y, x)
    if wid == 4:
        B = B if B is not None else 4096
        rng = rng_for(4, 0)
        lengths = rng.integers(256, 16384, size=B, endpoint=True)
        if T is not None:                       # reduced variant: scale lengths down
            lengths = np.maximum(1, (lengths * T) // 16384)
        qs = rng.uniform(0.1, 10.0, size=B)
        rs = rng.uniform(0.01, 1.0, size=B)
        offsets = np.zeros(B + 1, dtype=np.int64)
        offsets[1:] = np.cumsum(lengths)
        ys = np.empty((int(offsets[-1]), 2))
        xs = np.empty((int(offsets[-1]), 4)) if keep_states else None
        models = [cv_model(qs[b], rs[b]) for b in range(B)]
        for b in range(B):
            yb, xb = simulate_cv(qs[b], rs[b], int(lengths[b]), rng_for(4, b + 1), keep_states=keep_states)
            ys[offsets[b]:offsets[b + 1]] = yb
            if keep_states:
                xs[offsets[b]:offsets[b + 1]] = xb
        stack = lambda attr: np.stack([getattr(mo, attr) for mo in models])
        model = Model(stack("F"), stack("Q"), stack("H"), stack("R"), stack("m0"), stack("P0"))
        return Workload(WORKLOAD_NAMES[4], model, ys, offsets, True, xs,
                        dict(q=qs, r=rs, lengths=lengths))
    if wid == 5:
        B = B if B is not None else 64
        T = T if T is not None else 8192
        rng = rng_for(5, 0)
        nx, ny = 64, 32
        F = 0.995 * haar_orthogonal(nx, rng)
        H = rng.standard_normal((ny, nx)) / np.sqrt(nx)
        model = Model(F, 0.01 * np.eye(nx), H, 0.1 * np.eye(ny), np.zeros(nx), np.eye(nx))
        offsets = np.arange(B + 1, dtype=np.int64) * T
        ys = np.empty((B * T, ny))
        xs = np.empty((B * T, nx)) if keep_states else None
        # simulate the B sequences together (independent draws per sequence)
        X = np.stack([rng_for(5, b + 1).standard_normal(nx) for b in range(B)])   # x0 = 0 + I^(1/2) z
        gens = [rng_for(5, 1000 + b) for b in range(B)]
        qn = np.stack([g.standard_normal((T, nx)) for g in gens]) * np.sqrt(0.01)
        rn = np.stack([g.standard_normal((T, ny)) for g in gens]) * np.sqrt(0.1)
        Xs = np.empty((B, T, nx))
        for k in range(T):
            X = X @ F.T + qn[:, k]
            Xs[:, k] = X
        Y = Xs @ H.T + rn
        ys[:] = Y.reshape(B * T, ny)
        if keep_states:
            xs[:] = Xs.reshape(B * T, nx)
        return Workload(WORKLOAD_NAMES[5], model, ys, offsets, False, xs)
    if wid == 6:
        T = T if T is not None else 1 << 20
        rng = rng_for(6, 0)
        dts = rng.uniform(0.05, 0.15, size=T)
        model = cv_model_tv(dts, 1.0, 0.25)
        y, x = simulate_cv_tv(dts, 1.0, 0.25, rng_for(6, 1), keep_states)
        w = _single(WORKLOAD_NAMES[6], model, y, x, q=1.0, r=0.25)
        w.time_varying = True
        return w
    raise ValueError("unknown workload %r" % wid)


def single_sequence(model: Model, T: int, seed: int, keep_states: bool = False) -> Workload:
    """An ad-hoc single sequence of the given model (tests)."""
    y, x = simulate(model, T, rng_for(100, seed), keep_states)
    return _single("custom", model, y, x)


# ---------------------------------------------------------------------------
# error metric (per-step normwise relative error, maximised over steps)
# ---------------------------------------------------------------------------

def max_rel_err(X: np.ndarray, Xref: np.ndarray, floor: str = "none") -> float:
    """max_k ||X_k - Xref_k||_F / max(||Xref_k||_F, f) over the leading axis.

    floor = "none": f = 1e-300 (plain per-step normwise relative error);
    floor = "rms":  f = root-mean-square of ||Xref_k||_F over k (for results
    that pass through zero, e.g. the mean of a scalar state).
    """
    X = np.asarray(X, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    n = X.shape[0]
    if n == 0:
        return 0.0
    D = (X - Xref).reshape(n, -1)
    num = np.sqrt(np.einsum("ij,ij->i", D, D))
    R = Xref.reshape(n, -1)
    nrm = np.sqrt(np.einsum("ij,ij->i", R, R))
    f = 1e-300 if floor == "none" else max(1e-300, float(np.sqrt(np.mean(nrm ** 2))))
    den = np.maximum(nrm, f)
    with np.errstate(invalid="ignore"):
        r = num / den
    if np.any(np.isnan(r)):
        return float("nan")
    return float(np.max(r))


# ---------------------------------------------------------------------------
# discrete-state hidden Markov model
# ---------------------------------------------------------------------------
@dataclass
class HmmWorkload:
    name: str
    Pi: np.ndarray          # [K, K] row-stochastic
    p0: np.ndarray          # [K]
    L: np.ndarray           # [T, K] emission log-likelihoods
    x: Optional[np.ndarray] = None   # [T] simulated states

    @property
    def K(self) -> int:
        return self.Pi.shape[0]

    @property
    def T(self) -> int:
        return self.L.shape[0]


def hmm_model(K: int, rng: np.random.Generator, stay: float = 0.9, sparse: bool = False):
    """Sticky transitions: Pi = stay I + (1 - stay) D with D's rows drawn from
    a flat Dirichlet (with ``sparse``, about half of D's entries are zero);
    uniform prior."""
    D = rng.dirichlet(np.ones(K), size=K)
    if sparse:
        D *= rng.random((K, K)) < 0.5
        D[np.arange(K), (np.arange(K) + 1) % K] += 1e-3
        D /= D.sum(axis=1, keepdims=True)
    Pi = stay * np.eye(K) + (1.0 - stay) * D
    Pi /= Pi.sum(axis=1, keepdims=True)
    return Pi, np.full(K, 1.0 / K)


def hmm_simulate(Pi: np.ndarray, p0: np.ndarray, T: int, rng: np.random.Generator, sigma: float = 1.0):
    """States x_1..x_T of the chain and the Gaussian emission log-likelihoods
    of y_k ~ N(x_k / 2, sigma^2) under every state."""
    K = Pi.shape[0]
    cum = np.cumsum(Pi, axis=1)
    x = np.empty(T, dtype=np.int64)
    s = rng.choice(K, p=p0)
    u = rng.random(T)
    for k in range(T):
        s = min(int(np.searchsorted(cum[s], u[k], side="right")), K - 1)
        x[k] = s
    mu = 0.5 * np.arange(K)
    y = mu[x] + sigma * rng.standard_normal(T)
    L = -0.5 * ((y[:, None] - mu[None, :]) / sigma) ** 2 - np.log(sigma * np.sqrt(2.0 * np.pi))
    return np.ascontiguousarray(L), x


def hmm_workload(K: int = 64, T: int = 1 << 16, seed: int = 7, sparse: bool = False) -> HmmWorkload:
    rng = rng_for(seed, K)
    Pi, p0 = hmm_model(K, rng, sparse=sparse)
    L, x = hmm_simulate(Pi, p0, T, rng)
    return HmmWorkload("hmm_K%d_T%d" % (K, T), Pi, p0, L, x)
