"""dG(r) time discretisation on one slab with the right Gauss-Radau nodal basis.

Test infrastructure (oracle): see the package docstring.

Section 2.5 fixes the basis: Lagrange polynomials {v_i} of degree r on the r+1 right Gauss-Radau
points of the slab (the last point is the right end of the slab).  On I_n = (t_{n-1}, t_n] with
length tau the matrices are (eqs. At, Bt, Ct):
    [A_t]_{ij} = int_{I_n} v_j' v_i dt + v_j(t_{n-1}^+) v_i(t_{n-1}^+)      (tau-free)
    [B_t]_{ij} = int_{I_n} v_j v_i dt                                      (scales with tau)
    [C_t]_{ij} = v_j^{(n-1)}(t_{n-1}^-) v_i^{(n)}(t_{n-1}^+)               (transfer, tau-free)
The integrals are done exactly (Gauss-Legendre with enough points) in the reference slab (0, 1)
and then scaled.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def right_radau_nodes(r: int) -> np.ndarray:
    """The r+1 right Gauss-Radau points on [0, 1]: roots of P_{r+1}(s) - P_r(s) on [-1, 1], mapped."""
    c = np.zeros(r + 2)
    c[r + 1] = 1.0
    c[r] -= 1.0
    s = np.sort(np.real(L.legroots(c)))
    s[-1] = 1.0  # the right end point is exactly a root
    return 0.5 * (s + 1.0)


def lagrange_value(nodes: np.ndarray, i: int, s: np.ndarray) -> np.ndarray:
    """l_i(s) = prod_{j != i} (s - s_j) / (s_i - s_j)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.ones_like(s)
    for j, nj in enumerate(nodes):
        if j != i:
            out = out * (s - nj) / (nodes[i] - nj)
    return out


def lagrange_deriv(nodes: np.ndarray, i: int, s: np.ndarray) -> np.ndarray:
    """l_i'(s) = sum_{k != i} 1/(s_i - s_k) prod_{j != i, k} (s - s_j)/(s_i - s_j)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    for k, nk in enumerate(nodes):
        if k == i:
            continue
        term = np.full_like(s, 1.0 / (nodes[i] - nk))
        for j, nj in enumerate(nodes):
            if j != i and j != k:
                term = term * (s - nj) / (nodes[i] - nj)
        out = out + term
    return out


def time_matrices(r: int, tau: float):
    """Return (A_t, B_t, C_t) for dG(r) on a slab of length tau.

    The integrands are polynomials of degree <= 2r, integrated exactly by the (r+2)-point
    Gauss-Legendre rule on the reference slab (0, 1).
    """
    nodes = right_radau_nodes(r)
    g, w = L.leggauss(r + 2)
    s = 0.5 * (g + 1.0)
    w = 0.5 * w
    n = r + 1
    val = [lagrange_value(nodes, i, s) for i in range(n)]
    der = [lagrange_deriv(nodes, i, s) for i in range(n)]
    at0 = [float(lagrange_value(nodes, i, np.array(0.0))) for i in range(n)]
    at1 = [float(lagrange_value(nodes, i, np.array(1.0))) for i in range(n)]
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    C = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            # d/dt v_j = (1/tau) d/ds v_j and dt = tau ds, so the derivative term is tau-free.
            A[i, j] = float(np.sum(w * der[j] * val[i])) + at0[j] * at0[i]
            B[i, j] = tau * float(np.sum(w * val[j] * val[i]))
            # previous slab's basis at its right end (s = 1) times this slab's basis at s = 0
            C[i, j] = at1[j] * at0[i]
    return A, B, C
