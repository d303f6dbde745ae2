"""The finite-chaos benchmark: projected forcing, slab-by-slab time marching and the error quantities.

Test infrastructure (oracle): see the package docstring.  Plain FP64, explicit element quadrature,
assembled matrices, one sparse LU per problem reused over the slabs.

Benchmark (Section 3.2): D = (-1, 1)^2, T = 1, M = 4, coefficient a = d_min + (sum_k xi_k g_k(x))^2
(eq. diffusion_benchmark, non-affine: 11 Hermite modes, given by sg_inputs), exact solution
u = phi(x, t) G_q(xi) with phi = t^4 s(x), s = sin(pi (x_1+1)/2) sin(pi (x_2+1)/2), and
G_q = sum_{alpha in Lambda_q} c_alpha Psi_alpha (eqs. finite-exact-separated .. finite-chaos-coefficients).

Forcing (eq. finite_rhs_factorized, projected on Psi_beta as in Section 3): with
d_{mu beta} = sum_{alpha in Lambda_q} c_alpha E[Psi_mu Psi_alpha Psi_beta],
    f_beta = c_beta d_t phi - div( sum_mu d_{mu beta} a_mu grad phi ),
and its slab load (eq. load_vector), after integrating the divergence by parts (v = 0 on the boundary),
    F_{beta, i, j} = c_beta T1_i (s, psi_j) + T2_i sum_mu d_{mu beta} (a_mu grad s, grad psi_j),
    T1_i = int_{I_n} 4 t^3 v_i dt,  T2_i = int_{I_n} t^4 v_i dt.
The space integrals use the (k+3)-point Gauss rule per direction, the time integrals the (r+3)-point
Gauss rule (exact).  Slab sequence: AA U^(1) = F^(1) (u(0) = 0), AA U^(n) = F^(n) + JJ U^(n-1).

Errors (Definition def:error-norms-and-quantities): per slab, space-time quadrature with the
(k+3)-point rule per space direction and the (r+3)-point rule in time of
    full:  sum_{alpha in Lambda_q} |c_alpha phi - u_{h,alpha}|^2  (u_{h,alpha} = 0 outside Lambda_p),
    mean:  |phi - u_{h,0}|^2,
    var:   |phi^2 C2 - sum_{alpha != 0} u_{h,alpha}^2|^2,   C2 = sum_{0 != alpha in Lambda_q} c_alpha^2,
and the same with gradients for the H1-seminorm quantities (grad of the variance: 2 sum u grad u).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as L

from . import adjoint, chaos, fem, timebasis
from .slab import SlabProblem, from_workload


def exact_coefficients(index_set, fw) -> np.ndarray:
    return np.array([fw.c_alpha(a) for a in index_set])


def forcing_chaos_weights(P: SlabProblem, fw) -> np.ndarray:
    """d[mu, beta] = sum_{alpha in Lambda_q} c_alpha E[Psi_mu Psi_alpha Psi_beta] for beta in Lambda_p."""
    import sg_inputs
    Lq = chaos.total_degree_set(4, sg_inputs.FINITE_Q)
    d = np.zeros((len(P.coef_mu), P.n_xi))
    for k, mu in enumerate(P.coef_mu):
        for b, beta in enumerate(P.index_set):
            tot = 0.0
            for alpha in Lq:
                v = fw.c_alpha(alpha)
                for m in range(4):
                    v *= chaos.hermite_triple_1d(mu[m], alpha[m], beta[m])
                    if v == 0.0:
                        break
                tot += v
            d[k, b] = tot
    return d


def _tables(mesh: fem.Mesh, nq1: int):
    """Shape values [nq, nl], reference gradients [nq, nl, d], weights [nq] and reference points of the
    nq1-point Gauss rule per direction (points lexicographic, x fastest)."""
    pts, wts = fem.gauss_rule(nq1)
    k = mesh.k
    v1 = np.array([[float(timebasis.lagrange_value(mesh.support, a, np.array(x))) for a in range(k + 1)] for x in pts])
    d1 = np.array([[float(timebasis.lagrange_deriv(mesh.support, a, np.array(x))) for a in range(k + 1)] for x in pts])
    qloc = [tuple(reversed(t)) for t in itertools.product(range(nq1), repeat=mesh.dim)]
    loc = mesh.local_multi()
    phi = np.empty((len(qloc), len(loc)))
    dphi = np.empty((len(qloc), len(loc), mesh.dim))
    w = np.empty(len(qloc))
    ref = np.empty((len(qloc), mesh.dim))
    for q, qm in enumerate(qloc):
        w[q] = np.prod([wts[qm[d]] for d in range(mesh.dim)])
        ref[q] = [pts[qm[d]] for d in range(mesh.dim)]
        for a, am in enumerate(loc):
            phi[q, a] = np.prod([v1[qm[d], am[d]] for d in range(mesh.dim)])
            for e in range(mesh.dim):
                dphi[q, a, e] = np.prod([(d1 if d == e else v1)[qm[d], am[d]] for d in range(mesh.dim)])
    return phi, dphi, w, ref


def _points(mesh: fem.Mesh, ref: np.ndarray) -> np.ndarray:
    """Physical points [n_cells, nq, d] of reference points ref [nq, d]."""
    cm = np.array([mesh.cell_multi(c) for c in range(mesh.n_cells)], dtype=np.float64)
    return mesh.lo + mesh.h * (cm[:, None, :] + ref[None, :, :])


def spatial_loads(P: SlabProblem, nq1: int | None = None):
    """(m, k) with m_j = (s, psi_j) and k[mu]_j = (a_mu grad s, grad psi_j), Dirichlet entries zeroed."""
    import sg_inputs
    mesh = P.mesh
    nq1 = mesh.k + 3 if nq1 is None else nq1
    phi, dphi, w, ref = _tables(mesh, nq1)
    x = _points(mesh, ref)
    s, gs = sg_inputs.finite_chaos_phi(x)
    mus, a = sg_inputs.finite_chaos_coefficient_modes(x)
    assert [tuple(m) for m in mus] == P.coef_mu
    vol = mesh.h ** mesh.dim
    dofs = mesh.all_cell_dofs()
    m = np.zeros(mesh.n_nodes)
    np.add.at(m, dofs, np.einsum("cq,q,qa->ca", s, w * vol, phi))
    k = np.zeros((len(mus), mesh.n_nodes))
    for i in range(len(mus)):
        flux = a[i][..., None] * gs                                    # [cells, q, d]
        np.add.at(k[i], dofs, np.einsum("cqe,q,qae->ca", flux, w * vol / mesh.h, dphi))
    m[P.bmask] = 0.0
    k[:, P.bmask] = 0.0
    return m, k


def time_loads(P: SlabProblem, n: int, tau: float) -> tuple[np.ndarray, np.ndarray]:
    """T1_i = int_{I_n} 4 t^3 v_i dt, T2_i = int_{I_n} t^4 v_i dt for slab n = 1, 2, ..."""
    r = P.n_t - 1
    nodes = timebasis.right_radau_nodes(r)
    g, wg = L.leggauss(r + 3)
    s = 0.5 * (g + 1.0)
    wg = 0.5 * wg
    t = (n - 1) * tau + tau * s
    T1 = np.array([tau * np.sum(wg * 4.0 * t ** 3 * timebasis.lagrange_value(nodes, i, s)) for i in range(r + 1)])
    T2 = np.array([tau * np.sum(wg * t ** 4 * timebasis.lagrange_value(nodes, i, s)) for i in range(r + 1)])
    return T1, T2


def load_vector(P: SlabProblem, fw, n: int, loads=None, dweights=None) -> np.ndarray:
    m, k = spatial_loads(P) if loads is None else loads
    d = forcing_chaos_weights(P, fw) if dweights is None else dweights
    c = exact_coefficients(P.index_set, fw)
    T1, T2 = time_loads(P, n, fw.base.tau)
    F = np.zeros((P.n_xi, P.n_t, P.n_x))
    for b in range(P.n_xi):
        kb = d[:, b] @ k
        for i in range(P.n_t):
            F[b, i] = c[b] * T1[i] * m + T2[i] * kb
    return F.reshape(-1)


def march(fw, P: SlabProblem | None = None) -> list[np.ndarray]:
    """Slab vectors U^(1..N) of the benchmark."""
    P = from_workload(fw.base) if P is None else P
    lu = spla.splu(P.assemble_full().tocsc())
    JJ = adjoint.transfer_matrix(P)
    loads, d = spatial_loads(P), forcing_chaos_weights(P, fw)
    U, prev = [], np.zeros(P.n)
    for n in range(1, fw.n_slabs + 1):
        u = lu.solve(load_vector(P, fw, n, loads, d) + JJ @ prev)
        U.append(u)
        prev = u
    return U


def errors(P: SlabProblem, fw, U: list[np.ndarray], nq1: int | None = None) -> dict:
    """E^{full, mean, var} in the L2_t(L2_x) norm and the L2_t(H1-semi) seminorm."""
    import sg_inputs
    mesh = P.mesh
    nq1 = mesh.k + 3 if nq1 is None else nq1
    phi, dphi, w, ref = _tables(mesh, nq1)
    x = _points(mesh, ref)
    s, gs = sg_inputs.finite_chaos_phi(x)                          # [cells, q], [cells, q, d]
    vol = mesh.h ** mesh.dim
    dofs = mesh.all_cell_dofs()
    c = exact_coefficients(P.index_set, fw)
    Lq = chaos.total_degree_set(4, sg_inputs.FINITE_Q)
    c_all = np.array([fw.c_alpha(a) for a in Lq])
    C2 = float(np.sum(c_all[1:] ** 2))
    in_p = set(P.index_set)
    tail = float(sum(fw.c_alpha(a) ** 2 for a in Lq if a not in in_p))
    r = P.n_t - 1
    nodes = timebasis.right_radau_nodes(r)
    g, wg = L.leggauss(r + 3)
    st = 0.5 * (g + 1.0)
    wg = 0.5 * wg
    vt = np.array([timebasis.lagrange_value(nodes, i, st) for i in range(r + 1)])   # [i, tq]
    tau = fw.base.tau
    acc = dict.fromkeys(["full_L2", "full_H1", "mean_L2", "mean_H1", "var_L2", "var_H1", "phi_L2", "phi_H1"], 0.0)
    wq = w * vol
    for n, u in enumerate(U, start=1):
        Ub = u.reshape(P.n_xi, P.n_t, P.n_x)[:, :, dofs]              # [alpha, i, cells, a]
        val = np.einsum("aicl,ql->aicq", Ub, phi)                      # values at space points
        grd = np.einsum("aicl,qle->aicqe", Ub, dphi) / mesh.h
        for tq in range(len(st)):
            t = (n - 1) * tau + tau * st[tq]
            wt = tau * wg[tq]
            uh = np.einsum("i,aicq->acq", vt[:, tq], val)
            gh = np.einsum("i,aicqe->acqe", vt[:, tq], grd)
            ph, gp = t ** 4 * s, t ** 4 * gs
            e = c[:, None, None] * ph[None] - uh
            ge = c[:, None, None, None] * gp[None] - gh
            acc["full_L2"] += wt * np.einsum("q,acq->", wq, e * e)
            acc["full_H1"] += wt * np.einsum("q,acqe->", wq, ge * ge)
            acc["mean_L2"] += wt * np.einsum("q,cq->", wq, e[0] * e[0])
            acc["mean_H1"] += wt * np.einsum("q,cqe->", wq, ge[0] * ge[0])
            V = C2 * ph * ph - np.sum(uh[1:] ** 2, axis=0)
            gV = 2.0 * C2 * ph[..., None] * gp - 2.0 * np.sum(uh[1:, ..., None] * gh[1:], axis=0)
            acc["var_L2"] += wt * np.einsum("q,cq->", wq, V * V)
            acc["var_H1"] += wt * np.einsum("q,cqe->", wq, gV * gV)
            acc["phi_L2"] += wt * np.einsum("q,cq->", wq, ph * ph)
            acc["phi_H1"] += wt * np.einsum("q,cqe->", wq, gp * gp)
    out = {
        "E_full_L2": math.sqrt(acc["full_L2"] + tail * acc["phi_L2"]),
        "E_full_H1": math.sqrt(acc["full_H1"] + tail * acc["phi_H1"]),
        "E_mean_L2": math.sqrt(acc["mean_L2"]),
        "E_mean_H1": math.sqrt(acc["mean_H1"]),
        "E_var_L2": math.sqrt(acc["var_L2"]),
        "E_var_H1": math.sqrt(acc["var_H1"]),
    }
    return out


def run(fw) -> dict:
    P = from_workload(fw.base)
    return errors(P, fw, march(fw, P))
