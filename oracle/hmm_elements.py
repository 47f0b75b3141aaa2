"""The paper's general filtering and smoothing elements and operators for a
finite state space, in numpy FP64.

TEST INFRASTRUCTURE ONLY (see the ``oracle`` package docstring).  Written from
Section III of Sarkka & Garcia-Fernandez, "Temporal Parallelization of
Bayesian Smoothers" (Definitions 1-2, Theorems 1-2), with integrals replaced by
sums over the states (the counting measure; the paper's concluding section
says the framework holds there).  A density of x given z is a K x K matrix
whose row z holds the distribution of x; a likelihood of z is a K-vector.
Nothing here is blocked, fused or reordered.

Model: x_0 ~ p0, p(x_k = j | x_{k-1} = i) = Pi[i][j], p(y_k | x_k = j) =
exp(L[k-1][j]).

Filtering element (Theorem 1)  a_k = (f_k, g_k):
  f_k[z][x] = p(x_k = x | y_k, x_{k-1} = z),   g_k[z] = p(y_k | x_{k-1} = z);
  for k = 1 both are taken from the prior: f_1[z] = p(x_1 | y_1), g_1[z] = p(y_1)
  for every z.
Filtering operator (Definition 1):
  f_ij[z][x] = sum_y g_j[y] f_j[y][x] f_i[z][y] / sum_y g_j[y] f_i[z][y],
  g_ij[z]    = g_i[z] sum_y g_j[y] f_i[z][y].
Smoothing element (Theorem 2)  a_k[z][x] = p(x_k = x | y_1:k, x_{k+1} = z),
  a_T[z][x] = p(x_T = x | y_1:T) for every z.
Smoothing operator (Definition 2): (a_i (x) a_j)(x | z) = sum_y a_i(x | y) a_j(y | z),
  i.e. the matrix a_j @ a_i in the row-z-is-the-condition layout.

Readings where the paper is silent (a conditional density of a state that has
probability zero):
* a filtering row z whose normaliser sum_y g_j[y] f_i[z][y] is 0: g_ij[z] = 0
  and f_ij[z] = f_i[z] @ f_j (any distribution; nothing downstream weighs it);
* a smoothing row z that the filter cannot reach (sum_x alpha_k[x] Pi[x][z]
  = 0): the row is alpha_k.
"""
from __future__ import annotations

import numpy as np


def filter_elements(Pi, p0, L):
    """All T filtering elements (Theorem 1): f [T,K,K], g [T,K]."""
    Pi = np.asarray(Pi, dtype=np.float64)
    lik = np.exp(np.asarray(L, dtype=np.float64))
    joint = Pi[None, :, :] * lik[:, None, :]          # p(x_k = x, y_k | x_{k-1} = z)
    first = (np.asarray(p0, dtype=np.float64) @ Pi) * lik[0]   # p(x_1 = x, y_1)
    joint[0] = first[None, :]
    g = joint.sum(axis=2)
    f = joint / np.where(g > 0, g, 1.0)[:, :, None]
    return f, g


def filter_combine(fi, gi, fj, gj):
    """Definition 1 with sums over the states."""
    w = fi * gj[None, :]                 # w[z][y] = f_i[z][y] g_j[y]
    den = w.sum(axis=1)
    num = w @ fj
    fij = np.where(den[:, None] > 0, num / np.where(den > 0, den, 1.0)[:, None], fi @ fj)
    return fij, gi * den


def filter_identity(K):
    """f = I, g = 1: (f, g) (x) e = e (x) (f, g) = (f, g)."""
    return np.eye(K), np.ones(K)


def smoother_elements(Pi, alpha):
    """All T smoothing elements (Theorem 2) from the filtered marginals."""
    Pi = np.asarray(Pi, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    T, K = alpha.shape
    a = np.empty((T, K, K))
    for k in range(T - 1):
        w = alpha[k][:, None] * Pi          # w[x][z] = alpha_k[x] Pi[x][z]
        den = w.sum(axis=0)                 # p(x_{k+1} = z | y_1:k)
        rows = (w / np.where(den > 0, den, 1.0)[None, :]).T
        a[k] = np.where(den[:, None] > 0, rows, alpha[k][None, :])
    a[T - 1] = alpha[T - 1][None, :]
    return a


def smoother_combine(ai, aj):
    """Definition 2 with sums: (a_i (x) a_j)[z][x] = sum_y a_j[z][y] a_i[y][x]."""
    return aj @ ai


def filter_prefix_fold(f, g):
    """a_1 (x) ... (x) a_k for every k, left to right: the filtered marginals
    (row 0 of f; every row is the same) and log p(y_1:k)."""
    T, K = g.shape
    alpha = np.empty((T, K))
    logp = np.empty(T)
    acc_f, acc_g = f[0], g[0]
    alpha[0], logp[0] = acc_f[0], np.log(acc_g[0])
    for k in range(1, T):
        acc_f, acc_g = filter_combine(acc_f, acc_g, f[k], g[k])
        alpha[k], logp[k] = acc_f[0], np.log(acc_g[0])
    return alpha, logp


def smoother_suffix_fold(a):
    """a_k (x) ... (x) a_T for every k, right to left: the smoothed marginals."""
    T, K, _ = a.shape
    gamma = np.empty((T, K))
    acc = a[T - 1]
    gamma[T - 1] = acc[0]
    for k in range(T - 2, -1, -1):
        acc = smoother_combine(a[k], acc)
        gamma[k] = acc[0]
    return gamma
