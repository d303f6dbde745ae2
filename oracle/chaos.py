"""Hermite polynomial chaos: index set and Galerkin triple-product tensors.

Test infrastructure (oracle): see the package docstring.

* Total-degree index set Lambda_p = {alpha in N0^M : |alpha|_1 <= p} with N_xi = C(M+p, p)
  (Section 2.6).  Ordering (the paper is silent): graded by |alpha|, then lexicographically
  descending inside a degree, e.g. M=2: (0,0),(1,0),(0,1),(2,0),(1,1),(0,2).
* [G_mu]_{alpha beta} = E[Psi_mu Psi_alpha Psi_beta] (eq. triple_stoch) factorises over the M
  variables (Remark "Factorization of stochastic couplings").  The one-dimensional factor for the
  orthonormal Hermite polynomials psi_n = He_n / sqrt(n!) (eq. Hermit_def) is the classical
  linearisation formula: with a+b+c = 2s even and s >= max(a,b,c),
      E[psi_a psi_b psi_c] = sqrt(a! b! c!) / ((s-a)! (s-b)! (s-c)!),   else 0.
"""
from __future__ import annotations

import math

import numpy as np


def total_degree_set(M: int, p: int) -> list[tuple[int, ...]]:
    """Lambda_p in graded, lexicographically descending order."""
    out: list[tuple[int, ...]] = []

    def rec(prefix: list[int], remaining: int, k: int) -> None:
        if k == M - 1:
            out.append(tuple(prefix + [remaining]))
            return
        for a in range(remaining, -1, -1):
            rec(prefix + [a], remaining - a, k + 1)

    for deg in range(p + 1):
        rec([], deg, 0)
    return out


def hermite_triple_1d(a: int, b: int, c: int) -> float:
    """E[psi_a(X) psi_b(X) psi_c(X)] for X ~ N(0, 1)."""
    tot = a + b + c
    if tot % 2:
        return 0.0
    s = tot // 2
    if s < a or s < b or s < c:
        return 0.0
    num = math.factorial(a) * math.factorial(b) * math.factorial(c)
    den = math.factorial(s - a) * math.factorial(s - b) * math.factorial(s - c)
    return math.sqrt(num) / den


def galerkin_tensor(mu: tuple[int, ...], index_set: list[tuple[int, ...]]) -> np.ndarray:
    """Dense [G_mu]_{alpha beta} over the given index set (product of 1D triple products)."""
    n = len(index_set)
    G = np.zeros((n, n))
    for ia, alpha in enumerate(index_set):
        for ib, beta in enumerate(index_set):
            v = 1.0
            for m in range(len(mu)):
                v *= hermite_triple_1d(mu[m], alpha[m], beta[m])
                if v == 0.0:
                    break
            G[ia, ib] = v
    return G


def hermite_probabilists(n: int, y: np.ndarray) -> np.ndarray:
    """He_n(y) from the three-term recurrence He_{k+1} = y He_k - k He_{k-1}."""
    y = np.asarray(y, dtype=np.float64)
    h0 = np.ones_like(y)
    if n == 0:
        return h0
    h1 = y.copy()
    for k in range(1, n):
        h0, h1 = h1, y * h1 - k * h0
    return h1


def psi_multi(alpha: tuple[int, ...], xi: np.ndarray) -> np.ndarray:
    """Psi_alpha(xi) = prod_m He_{alpha_m}(xi_m) / sqrt(alpha_m!); xi has shape [..., M]."""
    out = np.ones(xi.shape[:-1])
    for m, a in enumerate(alpha):
        out = out * hermite_probabilists(a, xi[..., m]) / math.sqrt(math.factorial(a))
    return out
