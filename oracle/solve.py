"""Solving the discrete second-kind system (oracle step O5).

Algorithm 1 solves eq. bie with GMRES.  The discrete system is solved exactly
(up to rounding) by dense LU, which is what GMRES converges to; the MGS-GMRES
below is kept for iteration counts only (unrestarted, zero or given initial
guess, relative residual ||f - A x||_2 / ||f||_2).
"""
from __future__ import annotations

import numpy as np


def lu_solve(A, f):
    return np.linalg.solve(A, f)


def gmres(apply, f, tol=1e-10, maxiter=200, x0=None):
    """Unrestarted GMRES with modified Gram-Schmidt.  Returns (x, iterations, residual history)."""
    N = f.shape[0]
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - apply(x) if x0 is not None else f.copy()
    fn = np.linalg.norm(f)
    beta = np.linalg.norm(r)
    hist = [beta / fn]
    if beta / fn <= tol:
        return x, 0, hist
    V = np.zeros((maxiter + 1, N))
    H = np.zeros((maxiter + 1, maxiter))
    V[0] = r / beta
    g = np.zeros(maxiter + 1)
    g[0] = beta
    cs = np.zeros(maxiter)
    sn = np.zeros(maxiter)
    k = 0
    for k in range(maxiter):
        w = apply(V[k])
        for j in range(k + 1):
            H[j, k] = V[j] @ w
            w = w - H[j, k] * V[j]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        for j in range(k):
            t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
            H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
            H[j, k] = t
        den = np.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / fn)
        if hist[-1] <= tol:
            k += 1
            break
    else:
        k = maxiter
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = x + V[:k].T @ y
    return x, k, hist
