"""Dense matrices of the paper's factorization, for tiny n (test infrastructure).

Everything is built literally from the definitions so that tests can check
the identities the paper states, and can pin the C oracle against them:

* ``fourier(n)``      (F_n)_{jk} = w_n^{jk}, w_n = exp(-2 pi i / n)
                      (Sec. "1D problem").
* ``butterfly(r, k)`` B_{r,k} = (F_r (x) I_{k/r}) diag(I, W, ..., W^{r-1}),
                      W = Omega_{r,k/r} = diag(w_k^j) (eq. 25).
* ``a_rho(rho)``      A_rho = B_{r_t,n} (I (x) B_{r_{t-1},k_{t-1}}) ...
                      (I (x) B_{r_1,r_1}) (Sec. "Mixed-radix framework";
                      for uniform r, the product of Sec. "General radix
                      Cooley-Tukey framework").
* ``mod_sort(r, m)``  the modulo-r sort R_{r,m} (eq. r-ary-sorting).
* ``p_rho(rho)``      P_rho as the product of perfect shuffles
                      Pi_{r,m} = R_{r,m}^{-1} (Sec. "Mixed-radix framework").
* ``p_uniform(r, t)`` P_{r,n} = R_{r,t,n} ... R_{r,1,n},
                      R_{r,q,n} = I_{r^{q-1}} (x) R_{r,n/r^{q-1}}
                      (Sec. "General radix Cooley-Tukey framework").
* ``pos(rho, k)``     where entry k of F x sits in A_rho^T x: mixed-radix digit
                      reversal (a consequence of F = P_rho A_rho^T; checked
                      against the matrices above in the tests).
"""
from __future__ import annotations

import numpy as np


def w(n, e):
    return np.exp(-2j * np.pi * (np.asarray(e) % n) / n)


def fourier(n):
    j = np.arange(n)
    return w(n, np.outer(j, j))


def butterfly(r, k):
    m = k // r
    diag = np.concatenate([w(k, p * np.arange(m)) for p in range(r)])
    return np.kron(fourier(r), np.eye(m)) @ np.diag(diag)


def a_rho(rho):
    n = int(np.prod(rho))
    a = np.eye(n, dtype=complex)
    k = 1
    for r in rho:                      # rightmost factor (r_1) applied first
        k *= r
        a = np.kron(np.eye(n // k), butterfly(r, k)) @ a
    return a


def mod_sort(r, m):
    """R_{r,m}: rows pick x_0, x_r, x_2r, ..., x_1, x_{r+1}, ... (0-based)."""
    mat = np.zeros((m, m))
    order = [b * r + a for a in range(r) for b in range(m // r)]
    for i, src in enumerate(order):
        mat[i, src] = 1.0
    return mat


def p_rho(rho):
    n = int(np.prod(rho))
    p = np.eye(n)
    k = 1
    for r in rho:
        k *= r
        shuffle = mod_sort(r, k).T     # Pi = R^{-1} = R^T
        p = np.kron(np.eye(n // k), shuffle) @ p
    return p


def p_uniform(r, t):
    n = r ** t
    p = np.eye(n)
    for q in range(1, t + 1):          # R_{r,1,n} applied first
        rq = np.kron(np.eye(r ** (q - 1)), mod_sort(r, n // r ** (q - 1)))
        p = rq @ p
    return p


def pos(rho, k):
    """Position of frequency k in A_rho^T x.

    Write k = d_t + r_t (d_{t-1} + r_{t-1} (... + r_2 d_1)); then
    pos = d_1 + r_1 (d_2 + r_2 (... + r_{t-1} d_t)).
    """
    t = len(rho)
    d = [0] * t
    x = int(k)
    for i in range(t - 1, -1, -1):
        d[i] = x % rho[i]
        x //= rho[i]
    p = 0
    for i in range(t - 1, -1, -1):
        p = p * rho[i] + d[i]
    return p


def pos_table(rho):
    n = int(np.prod(rho))
    return np.array([pos(rho, k) for k in range(n)], dtype=np.int64)
