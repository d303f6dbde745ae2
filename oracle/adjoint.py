"""Parameter gradient of a mean/variance quantity of interest by the adjoint slab sweep.

Test infrastructure (oracle): see the package docstring.  Plain FP64 with explicitly assembled
sparse matrices (route 1 of ``slab``) and direct solves; tiny meshes only.

Slab sequence (Problem tensor-product-slab-system with F = 0):
    AA U^(1) = B_0,        AA U^(n) = JJ U^(n-1)  (n = 2..N),
    JJ = I_xi (x) C_t (x) M_x  (eq. local_rhs_tensor),   B_0 = JJ applied to the initial value placed
    as the end-of-slab trace (eq. initial_vector with v_i(t_0^+) = [C_t]_{i r}).
The initial value u_0 (mean mode only) is taken as its nodal interpolant: the "projected initial
datum" read as interpolation onto V_h.  Dirichlet rows of AA are identity rows, Dirichlet columns are
dropped; rows of JJ at Dirichlet DoFs are zero (homogeneous data).

Quantity of interest at the final time T = t_N:  Q(xi) = int_D u(x, T, xi)^2 dx.  With the end-of-slab
traces u_a = U_{a, r} (r = N_t - 1, the right Radau node t_n) and m_ab = u_a^T M_x u_b,
    Q = sum_{a,b} m_ab Psi_a Psi_b = sum_eps q_eps Psi_eps,   q_eps = sum_{a,b} m_ab E[Psi_a Psi_b Psi_eps],
so by Section 3.1 (mean = zeroth chaos mode, variance = sum of the squared other modes, applied to Q)
    E[Q] = q_0,   Var[Q] = sum_{eps != 0} q_eps^2,   J = E[Q] + Var[Q].

Adjoint (Lagrangian L = J - sum_n lam^(n)^T (AA U^(n) - JJ U^(n-1))):
    AA^T lam^(N) = dJ/dU^(N),   AA^T lam^(n) = JJ^T lam^(n+1),
    dJ/dp = - sum_n lam^(n)^T (dAA/dp) U^(n),
    dAA/dtheta_m = G_{e_m} (x) B_t (x) K_{phi_m},   dAA/da_{0,K} = I (x) B_t (x) K_{chi_K}
(interior rows and columns only), for a(x, xi) = a_0(x) + sum_m theta_m phi_m(x) xi_m.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import chaos, fem
from .slab import SlabProblem


def build(aw, theta, a0_cells) -> SlabProblem:
    """Finest-level slab problem of an sg_inputs.AdjointWorkload for parameters (theta, a0)."""
    import sg_inputs
    w = aw.base
    mus, levels = sg_inputs.adjoint_coef_levels(
        aw, theta, a0_cells, lambda lvl: fem.Mesh(w.dim, w.n_cells_1d >> lvl, w.fe_degree, w.lo, w.hi).qp_coords())
    return SlabProblem(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree,
                       mus, levels[0], w.lo, w.hi)


def _interior(P: SlabProblem) -> sp.csr_matrix:
    return sp.diags((~P.full_boundary_mask()).astype(np.float64)).tocsr()


def transfer_matrix(P: SlabProblem) -> sp.csr_matrix:
    """JJ = I_xi (x) C_t (x) M_x with zero Dirichlet rows and dropped Dirichlet columns."""
    J = sp.kron(sp.identity(P.n_xi), sp.kron(sp.csr_matrix(P.Ct), P.Mx)).tocsr()
    D = _interior(P)
    return (D @ J @ D).tocsr()


def initial_trace(P: SlabProblem, u0_nodes: np.ndarray) -> np.ndarray:
    """B_0: JJ applied to the slab vector carrying u_0 (mean mode) as its end-of-slab trace."""
    x = np.zeros(P.n)
    r = P.n_t - 1
    x[r * P.n_x:(r + 1) * P.n_x] = u0_nodes
    x[P.full_boundary_mask()] = 0.0
    return transfer_matrix(P) @ x


def forward(P: SlabProblem, u0_nodes: np.ndarray, n_slabs: int) -> list[np.ndarray]:
    A = P.assemble_full().tocsc()
    JJ = transfer_matrix(P)
    b = initial_trace(P, u0_nodes)
    U = []
    for n in range(n_slabs):
        u = spla.spsolve(A, b)
        U.append(u)
        b = JJ @ u
    return U


def triple_table(P: SlabProblem, M: int, p: int):
    """E[Psi_a Psi_b Psi_eps] for a, b in the slab index set and |eps| <= 2p (eq. triple_stoch)."""
    A = P.index_set
    E = chaos.total_degree_set(M, 2 * p)
    T = np.zeros((len(A), len(A), len(E)))
    for i, a in enumerate(A):
        for j, b in enumerate(A):
            for e, eps in enumerate(E):
                v = 1.0
                for m in range(M):
                    v *= chaos.hermite_triple_1d(a[m], b[m], eps[m])
                T[i, j, e] = v
    return T, E


def qoi(P: SlabProblem, u_slab: np.ndarray, M: int, p: int, w_mean=1.0, w_var=1.0):
    """(E[Q], Var[Q], dJ/du) for J = w_mean E[Q] + w_var Var[Q] at the end of the slab vector u."""
    r = P.n_t - 1
    U = u_slab.reshape(P.n_xi, P.n_t, P.n_x)[:, r, :]
    Mx = P.Mx
    bm = P.bmask
    MU = np.stack([np.where(bm, 0.0, Mx @ np.where(bm, 0.0, U[a])) for a in range(P.n_xi)])
    m = U @ MU.T                                  # m[a, b] = u_a . (M u_b)
    T, E = triple_table(P, M, p)
    q = np.einsum("ab,abe->e", m, T)
    EQ, VQ = q[0], float(np.sum(q[1:] ** 2))
    C = 2.0 * w_mean * np.eye(P.n_xi) + 4.0 * w_var * np.einsum("e,ade->ad", q[1:], T[:, :, 1:])
    g = np.zeros((P.n_xi, P.n_t, P.n_x))
    g[:, r, :] = C @ MU
    return EQ, VQ, g.reshape(-1)


def dAA_dtheta(P: SlabProblem, m: int, phi_qp: np.ndarray) -> sp.csr_matrix:
    """G_{e_m} (x) B_t (x) K_{phi_m}, interior rows and columns."""
    M = len(P.index_set[0])
    mu = tuple(1 if j == m - 1 else 0 for j in range(M))
    G = chaos.galerkin_tensor(mu, P.index_set)
    K = P.mesh.stiffness(phi_qp)
    D = _interior(P)
    return (D @ sp.kron(sp.csr_matrix(G), sp.kron(sp.csr_matrix(P.Bt), K)) @ D).tocsr()


def cell_forms(P: SlabProblem, lam: np.ndarray, u: np.ndarray, G=None, coef_qp=None) -> np.ndarray:
    """lam^T (G (x) B_t (x) K_{c|K}) u for every cell K: the stiffness matrix of the field c (values at
    the Gauss points, default 1) restricted to K; G defaults to the identity (the mean mode)."""
    bm = P.full_boundary_mask()
    lam = np.where(bm, 0.0, lam).reshape(P.n_xi, P.n_t, P.n_x)
    u = np.where(bm, 0.0, u).reshape(P.n_xi, P.n_t, P.n_x)
    if coef_qp is None:
        coef_qp = np.ones((P.mesh.n_cells, P.mesh.nq))
    Ke = P.mesh.element_matrices(coef_qp)
    G = np.eye(P.n_xi) if G is None else G
    dofs = P.mesh.all_cell_dofs()
    out = np.zeros(P.mesh.n_cells)
    for c in range(P.mesh.n_cells):
        d = dofs[c]
        for i in range(P.n_t):
            Gu = G @ u[:, i, d]                     # [alpha, a] = sum_beta G[alpha, beta] u_beta
            out[c] += P.Bt[i, i] * np.einsum("ab,xa,xb->", Ke[c], lam[:, i, d], Gu)
    return out


def gradient(aw, theta, a0_cells, u0_nodes=None):
    """J and its gradient with respect to theta (M values) and a_0 per cell (n_cells values)."""
    import sg_inputs
    w = aw.base
    P = build(aw, theta, a0_cells)
    if u0_nodes is None:
        u0_nodes = sg_inputs.initial_value(P.mesh.node_coords())
    U = forward(P, u0_nodes, aw.n_slabs)
    EQ, VQ, g = qoi(P, U[-1], w.n_vars, w.chaos_degree)
    A = P.assemble_full().tocsc()
    AT = A.T.tocsc()
    JJ = transfer_matrix(P)
    pts = P.mesh.qp_coords()
    dth = np.zeros(w.n_vars)
    da0 = np.zeros(P.mesh.n_cells)
    Dth = [dAA_dtheta(P, m, sg_inputs.sine_shape_at(m, pts)) for m in range(1, w.n_vars + 1)]
    rhs = g
    for n in reversed(range(aw.n_slabs)):
        lam = spla.spsolve(AT, rhs)
        for m in range(w.n_vars):
            dth[m] -= lam @ (Dth[m] @ U[n])
        da0 -= cell_forms(P, lam, U[n])
        rhs = JJ.T @ lam
    return EQ + VQ, (EQ, VQ), dth, da0


def objective(aw, theta, a0_cells, u0_nodes=None) -> float:
    """J alone (forward sweep only)."""
    import sg_inputs
    w = aw.base
    P = build(aw, theta, a0_cells)
    if u0_nodes is None:
        u0_nodes = sg_inputs.initial_value(P.mesh.node_coords())
    U = forward(P, u0_nodes, aw.n_slabs)
    EQ, VQ, _ = qoi(P, U[-1], w.n_vars, w.chaos_degree)
    return EQ + VQ
