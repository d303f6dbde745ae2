"""Monte-Carlo estimators of the finite-chaos benchmark and their error split (Section 5).

Test infrastructure (oracle): see the package docstring.  One sample at a time, assembled matrices,
one sparse LU per sample reused over the slabs.

Pathwise problem at xi (Problem mc-pathwise-deterministic with the benchmark's data): coefficient
a(x, xi) (one field), exact solution u(x, t, xi) = phi(x, t) G_q(xi), forcing
f = G_q(xi) [d_t phi - div(a(., xi) grad phi)], so its slab load (eq. load_vector, divergence
integrated by parts) is
    F_i = G_q(xi) ( T1_i m + T2_i sum_mu Psi_mu(xi) k_mu )
with m, k_mu, T1, T2 as in ``finitechaos``.  Slab sequence (eq. mc-slab-system): AA U^(1) = F^(1),
AA U^(n) = F^(n) + JJ U^(n-1).

Estimators at every space-time quadrature point (eqs. mc-mean-estimator, mc-variance-estimator-unbiased,
mc-exact-sampled-mean-estimator, mc-exact-sampled-var-estimator) and the errors in L2_t(L2_x)
(eqs. mc-error-mean-L2,mc-error-var-L2, mc-disc-mean-error, mc-pure-sampling-mean-error,
mc-disc-var-error, mc-pure-sampling-var-error):
    tot  = || M_hat[u_h] - M[u] ||,   disc = || M_hat[u_h] - M_hat[u] ||,   mc = || M_hat[u] - M[u] ||
and the same for the variance, with M[u] = phi and V[u] = C2 phi^2.  Space rule: (k+3)-point Gauss per
direction; time rule: (r+3)-point Gauss per slab.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as L

from . import adjoint, chaos, timebasis
from . import finitechaos as fc
from . import montecarlo as mc
from .slab import from_workload


def g_q_many(xs: np.ndarray) -> np.ndarray:
    """G_q(xi) = sum_{|alpha| <= q} c_alpha Psi_alpha(xi) for every row of xs [N, 4]."""
    import sg_inputs
    la, lc = sg_inputs.finite_chaos_exact_modes()
    xs = np.atleast_2d(np.asarray(xs, dtype=np.float64))
    return sum(c * chaos.psi_multi(tuple(int(v) for v in a), xs) for a, c in zip(la, lc))


def g_q(xi: np.ndarray) -> float:
    return float(g_q_many(np.asarray(xi)[None])[0])


def _chaos_problem(ew):
    """An SG problem of the benchmark (degree 0) that carries the 11 coefficient modes for the loads."""
    return from_workload(ew.base)


def pathwise_march(ew, xi: np.ndarray, loads=None) -> list[np.ndarray]:
    P = mc.pathwise_problem(ew.base, xi)
    Q = _chaos_problem(ew)
    m, k = fc.spatial_loads(Q) if loads is None else loads
    psi_mu = np.array([chaos.psi_multi(mu, np.asarray(xi)[None])[0] for mu in Q.coef_mu])
    g = g_q(xi)
    kx = psi_mu @ k
    lu = spla.splu(P.assemble_full().tocsc())
    JJ = adjoint.transfer_matrix(P)
    U, prev = [], np.zeros(P.n)
    for n in range(1, ew.n_slabs + 1):
        T1, T2 = fc.time_loads(P, n, ew.base.tau)
        F = np.concatenate([g * (T1[i] * m + T2[i] * kx) for i in range(P.n_t)])
        u = lu.solve(F + JJ @ prev)
        U.append(u)
        prev = u
    return U


def error_split(ew, xs: np.ndarray | None = None) -> dict:
    """The six Monte-Carlo errors (tot / disc / mc, mean and variance) over the samples xs."""
    import sg_inputs
    xs = ew.samples() if xs is None else xs
    N = len(xs)
    Q = _chaos_problem(ew)
    loads = fc.spatial_loads(Q)
    sols = [pathwise_march(ew, xi, loads) for xi in xs]
    gs = g_q_many(xs)
    la, lc = sg_inputs.finite_chaos_exact_modes()
    C2 = float(np.sum(lc[np.any(la != 0, axis=1)] ** 2))
    mesh = Q.mesh
    nq1 = mesh.k + 3
    phi_t, _, w, ref = fc._tables(mesh, nq1)
    x = fc._points(mesh, ref)
    s, _ = sg_inputs.finite_chaos_phi(x)
    wq = w * mesh.h ** mesh.dim
    dofs = mesh.all_cell_dofs()
    r = Q.n_t - 1
    nodes = timebasis.right_radau_nodes(r)
    gl, wg = L.leggauss(r + 3)
    st = 0.5 * (gl + 1.0)
    wg = 0.5 * wg
    vt = np.array([timebasis.lagrange_value(nodes, i, st) for i in range(r + 1)])
    tau = ew.base.tau
    acc = dict.fromkeys(["tot_mean", "disc_mean", "mc_mean", "tot_var", "disc_var", "mc_var"], 0.0)
    for n in range(ew.n_slabs):
        vals = []
        for U in sols:
            Ub = U[n].reshape(Q.n_t, Q.n_x)[:, dofs]                       # [i, cells, a]
            vals.append(np.einsum("ica,qa->icq", Ub, phi_t))
        vals = np.array(vals)                                              # [s, i, cells, q]
        for tq in range(len(st)):
            t = n * tau + tau * st[tq]
            wt = tau * wg[tq]
            us = np.einsum("i,sicq->scq", vt[:, tq], vals)                 # discrete samples
            ue = np.array([g * t ** 4 * s for g in gs])                    # exact samples
            Mh, Me = mc.sample_mean(us), mc.sample_mean(ue)
            Vh, Ve = mc.sample_variance(us), mc.sample_variance(ue)
            ph = t ** 4 * s
            for key, d in [("tot_mean", Mh - ph), ("disc_mean", Mh - Me), ("mc_mean", Me - ph),
                           ("tot_var", Vh - C2 * ph * ph), ("disc_var", Vh - Ve), ("mc_var", Ve - C2 * ph * ph)]:
                acc[key] += wt * np.einsum("q,cq->", wq, d * d)
    return {k: math.sqrt(v) for k, v in acc.items()} | {"N": N}
