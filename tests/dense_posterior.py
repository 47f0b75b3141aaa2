"""Dense joint-Gaussian (batch least-squares) posterior of a linear/Gaussian model.

An independent check of the sequential oracle: all states x_1..x_T are an
affine map of (x_0, q_0, ..., q_{T-1}), so X and Y = H X + d + r are jointly
Gaussian and the smoothed moments are the conditional moments E[X | Y],
Cov[X | Y] computed with one dense solve.  The filtered moment at step k is
the same computation restricted to y_1..y_k, read at its last block.
Works with singular Q.  No recursion, no Kalman gain, no element or operator.
The same joint moments give the marginal likelihood: y_1..y_k are jointly
Gaussian, so log p(y_1:k) is one dense Gaussian log-density.
"""
from __future__ import annotations

import numpy as np


def _stack_maps(F, T):
    nx = F.shape[0]
    # X = Phi x0 + G w,  w = (q_0, ..., q_{T-1})
    Phi = np.zeros((T * nx, nx))
    G = np.zeros((T * nx, T * nx))
    Fp = [np.eye(nx)]
    for _ in range(T):
        Fp.append(F @ Fp[-1])
    for k in range(T):                 # block k holds x_{k+1}
        Phi[k * nx:(k + 1) * nx] = Fp[k + 1]
        for i in range(k + 1):         # q_i enters x_{i+1} and later
            G[k * nx:(k + 1) * nx, i * nx:(i + 1) * nx] = Fp[k - i]
    return Phi, G


def joint_moments(F, Q, H, R, m0, P0, T, u=None, d=None):
    nx, ny = F.shape[0], H.shape[0]
    u = np.zeros(nx) if u is None else np.asarray(u, float)
    d = np.zeros(ny) if d is None else np.asarray(d, float)
    Phi, G = _stack_maps(F, T)
    muX = Phi @ m0 + G @ np.tile(u, T)
    SigW = np.kron(np.eye(T), Q)
    SigX = Phi @ P0 @ Phi.T + G @ SigW @ G.T
    Hb = np.kron(np.eye(T), H)
    muY = Hb @ muX + np.tile(d, T)
    SigY = Hb @ SigX @ Hb.T + np.kron(np.eye(T), R)
    SigXY = SigX @ Hb.T
    return muX, SigX, muY, SigY, SigXY


def posterior(F, Q, H, R, m0, P0, y, u=None, d=None):
    """Returns (ms [T,nx], Ps [T,nx,nx]) = smoothed and (m, P) = filtered moments."""
    y = np.asarray(y, float)
    nx, ny = F.shape[0], H.shape[0]
    T = y.shape[0]
    muX, SigX, muY, SigY, SigXY = joint_moments(F, Q, H, R, m0, P0, T, u, d)
    Yv = y.reshape(-1)
    mean = muX + SigXY @ np.linalg.solve(SigY, Yv - muY)
    cov = SigX - SigXY @ np.linalg.solve(SigY, SigXY.T)
    ms = mean.reshape(T, nx)
    Ps = np.stack([cov[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] for k in range(T)])
    m = np.empty((T, nx))
    P = np.empty((T, nx, nx))
    for k in range(T):
        n = (k + 1) * ny
        sl = slice(k * nx, (k + 1) * nx)
        SY = SigY[:n, :n]
        SXY = SigXY[sl, :n]
        m[k] = muX[sl] + SXY @ np.linalg.solve(SY, Yv[:n] - muY[:n])
        P[k] = SigX[sl, sl] - SXY @ np.linalg.solve(SY, SXY.T)
    return m, P, ms, Ps


def joint_loglik(F, Q, H, R, m0, P0, y, u=None, d=None):
    """log p(y_1:k) for k = 1..T, each the dense Gaussian log-density of the
    stacked measurements y_1..y_k (slogdet and one solve of its covariance)."""
    y = np.asarray(y, float)
    ny = H.shape[0]
    T = y.shape[0]
    _, _, muY, SigY, _ = joint_moments(F, Q, H, R, m0, P0, T, u, d)
    Yv = y.reshape(-1)
    out = np.empty(T)
    for k in range(T):
        n = (k + 1) * ny
        r = Yv[:n] - muY[:n]
        sign, logdet = np.linalg.slogdet(SigY[:n, :n])
        assert sign > 0
        out[k] = -0.5 * (n * np.log(2.0 * np.pi) + logdet + r @ np.linalg.solve(SigY[:n, :n], r))
    return out


def joint_moments_tv(F, Q, H, R, m0, P0, u=None, d=None):
    """Joint moments of X = (x_1..x_T), Y = (y_1..y_T) for per-step matrices:
    F[k-1], Q[k-1], u[k-1] carry x_{k-1} to x_k, H[k-1], R[k-1], d[k-1]
    measure x_k.  x_k = Phi_k x_0 + sum_{i<k} Psi_{k,i} (u_i + q_i) with
    Phi_k = F[k-1] ... F[0] and Psi_{k,i} = F[k-1] ... F[i+1]."""
    T, nx = F.shape[0], F.shape[-1]
    ny = H.shape[-2]
    u = np.zeros((T, nx)) if u is None else np.asarray(u, float)
    d = np.zeros((T, ny)) if d is None else np.asarray(d, float)
    Phi = np.zeros((T * nx, nx))
    G = np.zeros((T * nx, T * nx))
    for k in range(T):                      # block k holds x_{k+1}
        Phi[k * nx:(k + 1) * nx] = F[k] @ (Phi[(k - 1) * nx:k * nx] if k else np.eye(nx))
        for i in range(k + 1):              # q_i, u_i enter x_{i+1} and later
            G[k * nx:(k + 1) * nx, i * nx:(i + 1) * nx] = (
                np.eye(nx) if i == k else F[k] @ G[(k - 1) * nx:k * nx, i * nx:(i + 1) * nx])
    muX = Phi @ m0 + G @ u.reshape(-1)
    SigW = np.zeros((T * nx, T * nx))
    Hb = np.zeros((T * ny, T * nx))
    Rb = np.zeros((T * ny, T * ny))
    for k in range(T):
        SigW[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = Q[k]
        Hb[k * ny:(k + 1) * ny, k * nx:(k + 1) * nx] = H[k]
        Rb[k * ny:(k + 1) * ny, k * ny:(k + 1) * ny] = R[k]
    SigX = Phi @ P0 @ Phi.T + G @ SigW @ G.T
    muY = Hb @ muX + d.reshape(-1)
    SigY = Hb @ SigX @ Hb.T + Rb
    SigXY = SigX @ Hb.T
    return muX, SigX, muY, SigY, SigXY


def posterior_tv(F, Q, H, R, m0, P0, y, u=None, d=None):
    """posterior() for per-step matrices; also returns log p(y_1:k) for every k."""
    y = np.asarray(y, float)
    T, ny = y.shape
    nx = F.shape[-1]
    muX, SigX, muY, SigY, SigXY = joint_moments_tv(F, Q, H, R, m0, P0, u, d)
    Yv = y.reshape(-1)
    mean = muX + SigXY @ np.linalg.solve(SigY, Yv - muY)
    cov = SigX - SigXY @ np.linalg.solve(SigY, SigXY.T)
    ms = mean.reshape(T, nx)
    Ps = np.stack([cov[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] for k in range(T)])
    m = np.empty((T, nx))
    P = np.empty((T, nx, nx))
    ll = np.empty(T)
    for k in range(T):
        n = (k + 1) * ny
        sl = slice(k * nx, (k + 1) * nx)
        SY = SigY[:n, :n]
        SXY = SigXY[sl, :n]
        r = Yv[:n] - muY[:n]
        m[k] = muX[sl] + SXY @ np.linalg.solve(SY, r)
        P[k] = SigX[sl, sl] - SXY @ np.linalg.solve(SY, SXY.T)
        ll[k] = -0.5 * (n * np.log(2 * np.pi) + np.linalg.slogdet(SY)[1] + r @ np.linalg.solve(SY, r))
    return m, P, ms, Ps, ll
