"""Monte-Carlo pathwise problems and the sample estimators (Section 5).

Test infrastructure (oracle): see the package docstring.  Plain FP64, assembled sparse matrices,
direct solves; one sample at a time.

Pathwise problem (Problem mc-pathwise-deterministic): for a draw xi^(s) the heat equation is
deterministic with the coefficient a(x, xi^(s)) = sum_mu a_mu(x) Psi_mu(xi^(s)) (eq. coeff_expansion
evaluated at the sample).  Its dG(r)-in-time, Q_k-in-space slab system (eq. mc-slab-system),

    (A_t (x) M_x + B_t (x) K_{a(., xi^(s))}) U_n = (C_t (x) M_x) U_{n-1},

is the slab operator of ``slab`` with a single chaos mode (p_xi = 0, N_xi = 1) and that single
coefficient field, so it is built here as such a problem.

Estimators (Section 5.2, eqs. mc-mean-estimator and mc-variance-estimator-unbiased), per entry:
    mean = (1/N) sum_s u^(s),   var = 1/(N - 1) sum_s (u^(s) - mean)^2;
the biased variant divides by N instead.
"""
from __future__ import annotations

import numpy as np

from . import adjoint, chaos, fem
from .slab import SlabProblem


def sampled_coefficient(w, xi: np.ndarray, points: np.ndarray) -> np.ndarray:
    """a(x, xi) at the given points for one sample xi [M]: sum over the coefficient modes."""
    import sg_inputs
    mus, vals = sg_inputs.coefficient_modes(w, points)
    xi = np.asarray(xi, dtype=np.float64).reshape(1, -1)
    return sum(float(chaos.psi_multi(tuple(mu), xi)[0]) * v for mu, v in zip(mus, vals))


def pathwise_problem(w, xi: np.ndarray, level: int = 0) -> SlabProblem:
    """The deterministic slab problem of sample xi (one mode, coefficient a(x, xi))."""
    n = w.n_cells_1d >> level
    mesh = fem.Mesh(w.dim, n, w.fe_degree, w.lo, w.hi)
    a = sampled_coefficient(w, xi, mesh.qp_coords())
    if not np.all(a > 0.0):
        raise ValueError("the sampled coefficient is not positive")
    return SlabProblem(w.dim, n, w.fe_degree, w.time_degree, w.tau, w.n_vars, 0,
                       [tuple([0] * w.n_vars)], a[None], w.lo, w.hi)


def pathwise_sequence(sw, xi: np.ndarray, n_slabs: int | None = None) -> list[np.ndarray]:
    """Slab vectors U^(1..N) of one sample (initial value u_0 = prod sin(pi x_k), no forcing)."""
    import sg_inputs
    P = pathwise_problem(sw.base, xi)
    u0 = sg_inputs.initial_value(P.mesh.node_coords())
    return adjoint.forward(P, u0, sw.n_slabs if n_slabs is None else n_slabs)


def sample_mean(U: np.ndarray) -> np.ndarray:
    """(1/N) sum_s U[s] (samples along axis 0)."""
    U = np.asarray(U, dtype=np.float64)
    total = np.zeros(U.shape[1:])
    for s in range(U.shape[0]):
        total += U[s]
    return total / U.shape[0]


def sample_variance(U: np.ndarray, unbiased: bool = True) -> np.ndarray:
    """1/(N - 1) sum_s (U[s] - mean)^2, or 1/N with unbiased=False."""
    U = np.asarray(U, dtype=np.float64)
    N = U.shape[0]
    m = sample_mean(U)
    total = np.zeros(U.shape[1:])
    for s in range(N):
        total += (U[s] - m) ** 2
    return total / ((N - 1) if unbiased else N)


def batch_final_slabs(sw, samples: np.ndarray | None = None) -> np.ndarray:
    """Last slab vector of every sample, [N, N_t * N_x]."""
    xs = sw.samples() if samples is None else samples
    return np.stack([pathwise_sequence(sw, xi)[-1] for xi in xs])
