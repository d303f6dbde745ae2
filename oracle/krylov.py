"""Flexible GMRES for one slab system (Remark solver-matrix-free-sg).

Test infrastructure (oracle): see the package docstring.

Right-preconditioned flexible GMRES (the preconditioner may change between iterations, so the
preconditioned directions Z are stored).  Readings where the paper is silent: restart length 30,
x0 = 0 unless given, classical Gram-Schmidt applied twice (CGS2), Givens rotations for the small
least-squares problem, and the stopping test on the true relative residual ||b - AA x|| / ||b||.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply, prec, b, x0=None, rtol=1e-8, restart=30, max_iter=1000):
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    stats = dict(iterations=0, restarts=0, vcycles=0, applies=0, converged=0)
    if bnorm == 0.0:
        stats.update(converged=1, rel_residual_true=0.0)
        return np.zeros(n), stats
    while True:
        r = b - apply(x)
        stats["applies"] += 1
        beta = np.linalg.norm(r)
        rel = beta / bnorm
        stats["rel_residual_true"] = rel
        if rel <= rtol:
            stats["converged"] = 1
            break
        if stats["iterations"] >= max_iter:
            break
        stats["restarts"] += 1
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = prec(V[j])
            stats["vcycles"] += 1
            w = apply(Z[j])
            stats["applies"] += 1
            h = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            stats["iterations"] += 1
            k = j + 1
            if hn == 0.0 or abs(g[j + 1]) / bnorm <= rtol or stats["iterations"] >= max_iter:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in reversed(range(k)):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
    return x, stats
