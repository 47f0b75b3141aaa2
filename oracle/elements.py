"""The paper's linear/Gaussian scan elements and associative operators, in numpy FP64.

TEST INFRASTRUCTURE ONLY (see the ``oracle`` package docstring).  Written from
Section IV of Sarkka & Garcia-Fernandez, "Temporal Parallelization of Bayesian
Smoothers", in the paper's notation, with ``numpy.linalg.solve`` as the only
library step.  Nothing here is blocked, fused or reordered.

Filtering element  a_k = (A_k, b_k, C_k, eta_k, J_k)       (Lemma 1)
  f_k(x_k | x_{k-1}) = N(x_k; A_k x_{k-1} + b_k, C_k)
  g_k(x_{k-1})      ∝ N_I(x_{k-1}; eta_k, J_k)
Filtering operator (A_i..J_i) ⊗ (A_j..J_j)                 (Lemma 2)
Smoothing element  a_k = (E_k, g_k, L_k)                   (Lemma 3)
  a_k(x_k | x_{k+1}) = N(x_k; E_k x_{k+1} + g_k, L_k)
Smoothing operator (E_i, g_i, L_i) ⊗ (E_j, g_j, L_j)       (Lemma 4)

Readings where the paper is silent:
* eta_1 = 0, J_1 = 0: the first element's likelihood p(y_1) does not depend on
  x_0 (Theorem 1 sets g_1 = p(y_1)), so its information parameters are zero.
* Identity elements: (I, 0, 0, 0, 0) for filtering, (I, 0, 0) for smoothing.
* The smoothing scan is a suffix scan a_k ⊗ (a_{k+1} ⊗ ... ⊗ a_n) in the
  original operand order (Theorem 2).
"""
from __future__ import annotations

import numpy as np


def _sym(X):
    return 0.5 * (X + np.swapaxes(X, -1, -2))


# ---------------------------------------------------------------------------
# Lemma 1: filtering elements
# ---------------------------------------------------------------------------

def filter_elements(F, Q, H, R, m0, P0, y, u=None, d=None):
    """All T filtering elements for a time-invariant model (Lemma 1).

    Returns arrays A [T,nx,nx], b [T,nx], C [T,nx,nx], eta [T,nx], J [T,nx,nx].
    """
    F, Q, H, R, m0, P0 = (np.asarray(a, dtype=np.float64) for a in (F, Q, H, R, m0, P0))
    y = np.asarray(y, dtype=np.float64)
    nx, ny = F.shape[0], H.shape[0]
    y = y.reshape(-1, ny)
    T = y.shape[0]
    u = np.zeros(nx) if u is None else np.asarray(u, dtype=np.float64)
    d = np.zeros(ny) if d is None else np.asarray(d, dtype=np.float64)
    I = np.eye(nx)

    A = np.empty((T, nx, nx))
    b = np.empty((T, nx))
    C = np.empty((T, nx, nx))
    eta = np.empty((T, nx))
    J = np.empty((T, nx, nx))

    # k > 1 : the transition density p(x_k | x_{k-1}) updated with y_k
    S = H @ Q @ H.T + R
    K = np.linalg.solve(S.T, (Q @ H.T).T).T          # K = Q H^T S^{-1}
    A_k = (I - K @ H) @ F
    C_k = (I - K @ H) @ Q
    HF = H @ F
    Sinv_HF = np.linalg.solve(S, HF)                   # S^{-1} H F
    J_k = F.T @ H.T @ Sinv_HF                          # F^T H^T S^{-1} H F
    for k in range(1, T):
        res = y[k] - H @ u - d
        A[k] = A_k
        b[k] = u + K @ res
        C[k] = C_k
        eta[k] = F.T @ H.T @ np.linalg.solve(S, res)   # F^T H^T S^{-1} (y - H u - d)
        J[k] = J_k

    # k = 1 : one Kalman prediction + update from x_0 ~ N(m0, P0)
    if T > 0:
        mm = F @ m0 + u
        Pm = F @ P0 @ F.T + Q
        S1 = H @ Pm @ H.T + R
        K1 = np.linalg.solve(S1.T, (Pm @ H.T).T).T
        A[0] = 0.0
        b[0] = mm + K1 @ (y[0] - H @ mm - d)
        C[0] = Pm - K1 @ S1 @ K1.T
        eta[0] = 0.0
        J[0] = 0.0
    return A, b, C, eta, J


def filter_identity(nx):
    return (np.eye(nx), np.zeros(nx), np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx)))


# ---------------------------------------------------------------------------
# Lemma 2: filtering operator
# ---------------------------------------------------------------------------

def filter_combine(ei, ej):
    """(A_i,b_i,C_i,eta_i,J_i) ⊗ (A_j,b_j,C_j,eta_j,J_j), Lemma 2, term by term."""
    Ai, bi, Ci, etai, Ji = ei
    Aj, bj, Cj, etaj, Jj = ej
    nx = Ai.shape[0]
    I = np.eye(nx)
    M = I + Ci @ Jj                  # I + C_i J_j
    Mt = I + Jj @ Ci                 # I + J_j C_i
    Aij = Aj @ np.linalg.solve(M, Ai)
    bij = Aj @ np.linalg.solve(M, bi + Ci @ etaj) + bj
    Cij = Aj @ np.linalg.solve(M, Ci) @ Aj.T + Cj
    etaij = Ai.T @ np.linalg.solve(Mt, etaj - Jj @ bi) + etai
    Jij = Ai.T @ np.linalg.solve(Mt, Jj) @ Ai + Ji
    return (Aij, bij, Cij, etaij, Jij)


def filter_prefix_fold(elems):
    """Sequential all-prefix-sums a_1, a_1⊗a_2, ... (Definition of all-prefix-sums).

    Returns the filtered means b_{1:k} and covariances C_{1:k} (Theorem 1: the
    prefix's f-part is p(x_k | y_{1:k})).
    """
    A, b, C, eta, J = elems
    T = A.shape[0]
    acc = (A[0], b[0], C[0], eta[0], J[0])
    m = np.empty_like(b)
    P = np.empty_like(C)
    m[0], P[0] = acc[1], acc[2]
    for k in range(1, T):
        acc = filter_combine(acc, (A[k], b[k], C[k], eta[k], J[k]))
        m[k], P[k] = acc[1], acc[2]
    return m, P


# ---------------------------------------------------------------------------
# Lemma 3: smoothing elements
# ---------------------------------------------------------------------------

def smoother_elements(F, Q, m, P, u=None):
    """All T smoothing elements from filtered means m [T,nx] and covariances P [T,nx,nx]."""
    F, Q = np.asarray(F, dtype=np.float64), np.asarray(Q, dtype=np.float64)
    m, P = np.asarray(m, dtype=np.float64), np.asarray(P, dtype=np.float64)
    T, nx = m.shape
    u = np.zeros(nx) if u is None else np.asarray(u, dtype=np.float64)
    E = np.empty((T, nx, nx))
    g = np.empty((T, nx))
    L = np.empty((T, nx, nx))
    for k in range(T - 1):
        Pk = P[k]
        Pp = F @ Pk @ F.T + Q
        Ek = np.linalg.solve(Pp.T, (Pk @ F.T).T).T       # P_k F^T (F P_k F^T + Q)^{-1}
        E[k] = Ek
        g[k] = m[k] - Ek @ (F @ m[k] + u)
        L[k] = Pk - Ek @ F @ Pk
    if T > 0:
        E[T - 1] = 0.0
        g[T - 1] = m[T - 1]
        L[T - 1] = P[T - 1]
    return E, g, L


def smoother_identity(nx):
    return (np.eye(nx), np.zeros(nx), np.zeros((nx, nx)))


# ---------------------------------------------------------------------------
# Lemma 4: smoothing operator
# ---------------------------------------------------------------------------

def smoother_combine(ei, ej):
    """(E_i,g_i,L_i) ⊗ (E_j,g_j,L_j), Lemma 4."""
    Ei, gi, Li = ei
    Ej, gj, Lj = ej
    return (Ei @ Ej, Ei @ gj + gi, Ei @ Lj @ Ei.T + Li)


def smoother_suffix_fold(elems):
    """Sequential suffix products a_k ⊗ ... ⊗ a_n for all k (Theorem 2).

    Returns smoothed means g and covariances L of each suffix.
    """
    E, g, L = elems
    T = E.shape[0]
    acc = (E[T - 1], g[T - 1], L[T - 1])
    ms = np.empty_like(g)
    Ps = np.empty_like(L)
    ms[T - 1], Ps[T - 1] = acc[1], acc[2]
    for k in range(T - 2, -1, -1):
        acc = smoother_combine((E[k], g[k], L[k]), acc)
        ms[k], Ps[k] = acc[1], acc[2]
    return ms, Ps
