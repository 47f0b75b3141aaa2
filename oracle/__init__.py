"""The oracle: a plain, sequential FP64 CPU Kalman filter + RTS smoother.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1905_13002_amd``) and imports nothing from it.

* :func:`kf_rts` / :func:`kf_rts_batched` wrap ``kfrts.c`` (plain C, FP64,
  built with ``gcc -O3 -ffp-contract=off``): the textbook recursions that the
  paper's parallel method reproduces exactly (Theorems 1 and 2).
* :func:`kf_rts_tv` runs the same recursion on a time-varying model (one
  row of F, u, Q, H, d, R per step; Section IV's general model).
* ``loglik=True`` adds the per-step factors log p(y_k | y_1:k-1) of the
  marginal likelihood (Section III-C); :func:`loglik_prefix` turns them into
  log p(y_1:k) and the per-sequence totals log p(y_1:n).
* :func:`loglik_factors` evaluates the same factors from GIVEN filtered
  moments, in extended precision (numpy ``longdouble``, 64-bit significand):
  the definition of each factor written out, so that it can serve as the
  reference for a likelihood computed from someone else's moments.
* :func:`hmm_fb` wraps ``hmm.c``: the sequential forward-backward recursion
  of a discrete-state hidden Markov model (the filtering and smoothing
  equations of Section II-A with sums in place of integrals).
  :mod:`oracle.hmm_elements` restates the paper's general elements and
  operators (Theorems 1-2, Definitions 1-2) for a finite state space.
* :mod:`oracle.elements` restates the paper's linear/Gaussian elements and
  associative operators (Lemmas 1-4) in numpy FP64, for operator-level checks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kfrts.c")
_SRCS = [_SRC, os.path.join(_HERE, "hmm.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``kfrts.c`` into ``liboracle.so`` next to it (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC",
               "-shared", "-pthread"] + _SRCS + ["-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_kf_rts.restype = ctypes.c_int
        lib.oracle_kf_rts.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long] + [dp] * 16
        lib.oracle_kf_rts_tv.restype = ctypes.c_int
        lib.oracle_kf_rts_tv.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long] + [dp] * 16
        lib.oracle_hmm.restype = ctypes.c_int
        lib.oracle_hmm.argtypes = [ctypes.c_int, ctypes.c_long] + [dp] * 6
        lib.oracle_kf_rts_batched.restype = ctypes.c_int
        lib.oracle_kf_rts_batched.argtypes = (
            [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_long), ctypes.c_int]
            + [dp] * 14 + [ctypes.c_int])
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def kf_rts(F, Q, H, R, m0, P0, y, u=None, d=None, smooth=True, predicted=False, loglik=False):
    """Run the sequential Kalman filter and (optionally) the RTS smoother.

    ``y`` is ``[T, ny]``; returns a dict with ``m [T,nx]``, ``P [T,nx,nx]`` and,
    when ``smooth``, ``ms``, ``Ps``; with ``predicted`` also ``mp``, ``Pp``
    (the one-step predictions m^-_k, P^-_k); with ``loglik`` also ``ll [T]``,
    the log predictive density log p(y_k | y_1:k-1) of every step.
    """
    lib = _load()
    F, Q, H, R, m0, P0, y = map(_f64, (F, Q, H, R, m0, P0, y))
    u, d = _f64(u), _f64(d)
    nx, ny = F.shape[0], H.shape[0]
    y = y.reshape(-1, ny)
    T = y.shape[0]
    m = np.empty((T, nx))
    P = np.empty((T, nx, nx))
    ms = np.empty((T, nx)) if smooth else None
    Ps = np.empty((T, nx, nx)) if smooth else None
    mp = np.empty((T, nx)) if predicted else None
    Pp = np.empty((T, nx, nx)) if predicted else None
    ll = np.empty(T) if loglik else None
    st = lib.oracle_kf_rts(nx, ny, T, _p(F), _p(u), _p(Q), _p(H), _p(d), _p(R), _p(m0), _p(P0),
                           _p(y), _p(m), _p(P), _p(ms), _p(Ps), _p(mp), _p(Pp), _p(ll))
    if st:
        raise OracleError("oracle: Cholesky failed (code %d)" % st)
    out = {"m": m, "P": P}
    if smooth:
        out.update(ms=ms, Ps=Ps)
    if predicted:
        out.update(mp=mp, Pp=Pp)
    if loglik:
        out["ll"] = ll
    return out


def kf_rts_tv(F, Q, H, R, m0, P0, y, u=None, d=None, smooth=True, predicted=False, loglik=False):
    """Time-varying model: F [T,nx,nx], Q [T,nx,nx], H [T,ny,nx], R [T,ny,ny],
    u [T,nx], d [T,ny] hold one row per step (row k-1: the transition into
    step k and the measurement model of step k).  Same outputs as kf_rts."""
    lib = _load()
    F, Q, H, R, m0, P0, y = map(_f64, (F, Q, H, R, m0, P0, y))
    u, d = _f64(u), _f64(d)
    nx, ny = F.shape[-1], H.shape[-2]
    y = y.reshape(-1, ny)
    T = y.shape[0]
    for a, shape in ((F, (T, nx, nx)), (Q, (T, nx, nx)), (H, (T, ny, nx)), (R, (T, ny, ny))):
        if a.shape != shape:
            raise ValueError("time-varying model arrays must be %s, got %s" % (shape, a.shape))
    m = np.empty((T, nx))
    P = np.empty((T, nx, nx))
    ms = np.empty((T, nx)) if smooth else None
    Ps = np.empty((T, nx, nx)) if smooth else None
    mp = np.empty((T, nx)) if predicted else None
    Pp = np.empty((T, nx, nx)) if predicted else None
    ll = np.empty(T) if loglik else None
    st = lib.oracle_kf_rts_tv(nx, ny, T, _p(F), _p(u), _p(Q), _p(H), _p(d), _p(R), _p(m0), _p(P0),
                              _p(y), _p(m), _p(P), _p(ms), _p(Ps), _p(mp), _p(Pp), _p(ll))
    if st:
        raise OracleError("oracle: Cholesky failed (code %d)" % st)
    out = {"m": m, "P": P}
    if smooth:
        out.update(ms=ms, Ps=Ps)
    if predicted:
        out.update(mp=mp, Pp=Pp)
    if loglik:
        out["ll"] = ll
    return out


def kf_rts_batched(F, Q, H, R, m0, P0, y, offsets, u=None, d=None, per_sequence=False,
                   threads=None, smooth=True, loglik=False):
    """Independent sequences packed back to back; see ``oracle_kf_rts_batched``."""
    lib = _load()
    F, Q, H, R, m0, P0, y = map(_f64, (F, Q, H, R, m0, P0, y))
    u, d = _f64(u), _f64(d)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    nx = F.shape[-1]
    ny = H.shape[-2]
    B = offsets.shape[0] - 1
    total = int(offsets[-1])
    y = y.reshape(total, ny)
    m = np.empty((total, nx))
    P = np.empty((total, nx, nx))
    ms = np.empty((total, nx)) if smooth else None
    Ps = np.empty((total, nx, nx)) if smooth else None
    ll = np.empty(total) if loglik else None
    if threads is None:
        threads = os.cpu_count() or 1
    st = lib.oracle_kf_rts_batched(
        nx, ny, B, offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), 1 if per_sequence else 0,
        _p(F), _p(u), _p(Q), _p(H), _p(d), _p(R), _p(m0), _p(P0), _p(y), _p(m), _p(P),
        _p(ms), _p(Ps), _p(ll), int(threads))
    if st:
        raise OracleError("oracle: Cholesky failed in sequence %d" % (st - 1))
    out = {"m": m, "P": P}
    if smooth:
        out.update(ms=ms, Ps=Ps)
    if loglik:
        out["ll"] = ll
    return out


def hmm_fb(Pi, p0, L, smooth=True):
    """Discrete-state hidden Markov model, sequential forward-backward
    (``hmm.c``): x_0 ~ p0, p(x_k = j | x_{k-1} = i) = Pi[i][j] and
    p(y_k | x_k = j) = exp(L[k-1][j]).  Returns a dict with the filtered
    marginals ``alpha [T,K]`` = p(x_k | y_1:k), the per-step factors
    ``ll [T]`` = log p(y_k | y_1:k-1) and, when ``smooth``, the smoothed
    marginals ``gamma [T,K]`` = p(x_k | y_1:T)."""
    lib = _load()
    Pi, p0, L = map(_f64, (Pi, p0, L))
    K = Pi.shape[0]
    L = L.reshape(-1, K)
    T = L.shape[0]
    alpha = np.empty((T, K))
    gamma = np.empty((T, K)) if smooth else None
    ll = np.empty(T)
    st = lib.oracle_hmm(K, T, _p(Pi), _p(p0), _p(L), _p(alpha), _p(gamma), _p(ll))
    if st < 0:
        raise MemoryError("oracle_hmm")
    if st:
        raise OracleError("oracle: the measurements of step %d have probability 0 under the model" % st)
    out = {"alpha": alpha, "ll": ll}
    if smooth:
        out["gamma"] = gamma
    return out


def loglik_prefix(ll, offsets=None):
    """From per-step factors log p(y_k | y_1:k-1) to the prefixes log p(y_1:k)
    of every sequence (a running sum that restarts at each sequence start, in
    step order) and the per-sequence totals log p(y_1:n) (0 for an empty
    sequence).  Section III-C: the marginal likelihood is the product of the
    factors, so its logarithm is their sum."""
    ll = np.asarray(ll, dtype=np.float64)
    if offsets is None:
        offsets = np.array([0, ll.shape[0]], dtype=np.int64)
    offsets = np.asarray(offsets, dtype=np.int64)
    cum = np.empty_like(ll)
    tot = np.zeros(offsets.shape[0] - 1)
    for b in range(offsets.shape[0] - 1):
        acc = 0.0
        for k in range(int(offsets[b]), int(offsets[b + 1])):
            acc += ll[k]
            cum[k] = acc
        tot[b] = acc
    return cum, tot


_LOG_2PI_LD = np.log(np.longdouble(2) * np.longdouble("3.14159265358979323846264338327950288"))


def _chol_logdet_quad(S, r):
    """Cholesky factor of every S[k] (unrolled over columns, vectorised over
    k), returning log det S[k] and r[k]^T S[k]^-1 r[k]; NaN where a pivot is
    not positive."""
    n = S.shape[-1]
    L = np.zeros_like(S)
    z = np.zeros_like(r)
    logdet = np.zeros(S.shape[0], dtype=S.dtype)
    ok = np.ones(S.shape[0], dtype=bool)
    for j in range(n):
        d = S[:, j, j] - np.sum(L[:, j, :j] * L[:, j, :j], axis=1)
        ok &= d > 0
        ljj = np.sqrt(np.where(d > 0, d, np.longdouble(1)))
        L[:, j, j] = ljj
        for i in range(j + 1, n):
            L[:, i, j] = (S[:, i, j] - np.sum(L[:, i, :j] * L[:, j, :j], axis=1)) / ljj
        z[:, j] = (r[:, j] - np.sum(L[:, j, :j] * z[:, :j], axis=1)) / ljj
        logdet += 2 * np.log(ljj)
    quad = np.sum(z * z, axis=1)
    nan = np.longdouble("nan")
    return np.where(ok, logdet, nan), np.where(ok, quad, nan)


def loglik_factors(F, Q, H, R, m0, P0, y, m, P, offsets=None, u=None, d=None, per_sequence=False):
    """log p(y_k | y_1:k-1) of every step, from GIVEN filtered moments m, P.

    Section III-C: each factor is the Gaussian density of y_k under the
    one-step prediction of the filtered moments of step k-1 (of the prior
    x_0 ~ N(m0, P0) at a sequence's first step):
        m^-_k = F m_{k-1} + u,   P^-_k = F P_{k-1} F^T + Q,
        log N(y_k; H m^-_k + d, H P^-_k H^T + R).
    Evaluated in extended precision (numpy longdouble) from the float64 values
    of the inputs, so the result is the factor of exactly those inputs, to
    about 1e-18 relative of its terms: where the residual y_k - H m^-_k - d is a
    small difference of large numbers (positions of 1e7) a float64 evaluation
    loses about seven digits of it.  Returns float64 [total].
    Sequences as in kf_rts_batched (offsets [B+1], per-sequence models when
    ``per_sequence``)."""
    ld = np.longdouble
    y = np.asarray(y)
    total = y.shape[0]
    if offsets is None:
        offsets = np.array([0, total], dtype=np.int64)
    offsets = np.asarray(offsets, dtype=np.int64)
    out = np.empty(total)
    for b in range(offsets.shape[0] - 1):
        s, e = int(offsets[b]), int(offsets[b + 1])
        if e <= s:
            continue
        pick = (lambda a: a[b]) if per_sequence else (lambda a: a)
        Fb, Qb, Hb, Rb = (np.asarray(pick(a), dtype=np.float64).astype(ld) for a in (F, Q, H, R))
        m0b, P0b = (np.asarray(pick(a), dtype=np.float64).astype(ld) for a in (m0, P0))
        nx, ny = Fb.shape[0], Hb.shape[0]
        ub = np.zeros(nx, dtype=ld) if u is None else np.asarray(pick(u), dtype=np.float64).astype(ld)
        db = np.zeros(ny, dtype=ld) if d is None else np.asarray(pick(d), dtype=np.float64).astype(ld)
        mprev = np.concatenate([m0b[None], np.asarray(m[s:e - 1], dtype=np.float64).astype(ld)])
        Pprev = np.concatenate([P0b[None], np.asarray(P[s:e - 1], dtype=np.float64).astype(ld)])
        mp = mprev @ Fb.T + ub
        Pp = Fb @ Pprev @ Fb.T + Qb
        S = Hb @ Pp @ Hb.T + Rb
        r = np.asarray(y[s:e], dtype=np.float64).astype(ld) - mp @ Hb.T - db
        logdet, quad = _chol_logdet_quad(S, r)
        out[s:e] = (-(ny * _LOG_2PI_LD + logdet + quad) / 2).astype(np.float64)
    return out


if __name__ == "__main__":  # pragma: no cover
    print(build(force=True), file=sys.stderr)
