"""Batches of independent stochastic Galerkin problems, and the chaos moments of a solution.

Test infrastructure (oracle): see the package docstring.  Each member is an ordinary slab problem of
``slab`` (its own total-degree index set, its own scaled coefficient), solved on its own.

Chaos moments (Section 3.1, eqs. qoi-mean-chaos and qoi-variance-chaos): with an orthonormal basis
and Psi_0 = 1, the mean of u = sum_alpha u_alpha Psi_alpha is u_0 and its variance is
sum_{alpha != 0} u_alpha^2.
"""
from __future__ import annotations

import numpy as np

from . import adjoint, fem
from .slab import SlabProblem


def member_problem(mw, j: int, level: int = 0) -> SlabProblem:
    """Slab problem of member j: degree mw.degrees[j], coefficient modes scaled by mw.scales."""
    import sg_inputs
    w = mw.base
    n = w.n_cells_1d >> level
    mesh = fem.Mesh(w.dim, n, w.fe_degree, w.lo, w.hi)
    mus, vals = sg_inputs.coefficient_modes(w, mesh.qp_coords())
    sc = mw.scales(mus)[j]
    vals = [sc[k] * np.asarray(v) for k, v in enumerate(vals)]
    return SlabProblem(w.dim, n, w.fe_degree, w.time_degree, w.tau, w.n_vars, int(mw.degrees[j]),
                       mus, np.stack(vals), w.lo, w.hi)


def member_sequence(mw, j: int) -> list[np.ndarray]:
    """Slab vectors U^(1..N) of member j (u_0 = prod sin(pi x_k) in the mean mode, no forcing)."""
    import sg_inputs
    P = member_problem(mw, j)
    return adjoint.forward(P, sg_inputs.initial_value(P.mesh.node_coords()), mw.n_slabs)


def chaos_moments(u: np.ndarray, n_xi: int) -> tuple[np.ndarray, np.ndarray]:
    """(mean, variance) of a slab vector [n_xi * rest]: mode 0, and the sum of squares of the others."""
    U = np.asarray(u, dtype=np.float64).reshape(n_xi, -1)
    var = np.zeros(U.shape[1])
    for a in range(1, n_xi):
        var += U[a] ** 2
    return U[0].copy(), var
