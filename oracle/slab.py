"""The coupled stochastic-Galerkin space-time slab operator (Problem tensor-product-slab-system).

Test infrastructure (oracle): see the package docstring.

On one slab the left-hand side is (eq. local_rhs_tensor)
    AA = M_xi (x) A_t (x) M_x  +  sum_{mu in M_a} G_mu (x) B_t (x) K_mu,       M_xi = I,
acting on the slab vector U ordered mode-major: index = alpha * (N_t N_x) + i * N_x + node.  The
paper lists the triple index in several orders; the Kronecker form fixes (alpha, i, node), which is
the layout used here.  Dirichlet rows are replaced by identity rows and Dirichlet columns are dropped
from the other rows (the homogeneous condition eq. heat_bc with boundary nodes kept in the vector).

Two independent routes compute y = AA x:
  route 1: assemble AA explicitly with scipy.sparse.kron (tiny meshes only);
  route 2: Kronecker identity with X[node, (alpha, i)]:
           Y = (M_x X)(I (x) A_t)^T + sum_mu (K_mu X)(G_mu (x) B_t)^T.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import chaos, fem, timebasis


class SlabProblem:
    """All matrices of one slab problem on one mesh level."""

    def __init__(self, dim, n_cells_1d, fe_degree, time_degree, tau, n_vars, chaos_degree,
                 coef_mu, coef_qp, lo=0.0, hi=1.0):
        self.mesh = fem.Mesh(dim, n_cells_1d, fe_degree, lo, hi)
        self.At, self.Bt, self.Ct = timebasis.time_matrices(time_degree, tau)
        self.index_set = chaos.total_degree_set(n_vars, chaos_degree)
        self.coef_mu = [tuple(m) for m in coef_mu]
        self.G = [chaos.galerkin_tensor(mu, self.index_set) for mu in self.coef_mu]
        coef_qp = np.asarray(coef_qp, dtype=np.float64)
        assert coef_qp.shape == (len(self.coef_mu), self.mesh.n_cells, self.mesh.nq)
        self.coef_qp = coef_qp
        self.Mx = self.mesh.mass()
        self.K = [self.mesh.stiffness(coef_qp[k]) for k in range(len(self.coef_mu))]
        self.bmask = self.mesh.boundary_mask()
        self.n_xi = len(self.index_set)
        self.n_t = time_degree + 1
        self.n_x = self.mesh.n_nodes
        self.n = self.n_xi * self.n_t * self.n_x
        # position of mu = 0 in the coefficient list (the mean field a_0)
        self.mu0 = self.coef_mu.index(tuple([0] * n_vars))

    # --- helpers ------------------------------------------------------------------------------
    def full_boundary_mask(self) -> np.ndarray:
        return np.tile(self.bmask, self.n_xi * self.n_t)

    def _apply_dirichlet(self, A: sp.spmatrix, nblocks: int) -> sp.csr_matrix:
        bm = np.tile(self.bmask, nblocks)
        interior = sp.diags((~bm).astype(np.float64))
        boundary = sp.diags(bm.astype(np.float64))
        return (interior @ A @ interior + boundary).tocsr()

    # --- route 1 ------------------------------------------------------------------------------
    def assemble_full(self) -> sp.csr_matrix:
        I_xi = sp.identity(self.n_xi, format="csr")
        A = sp.kron(I_xi, sp.kron(sp.csr_matrix(self.At), self.Mx))
        for G, K in zip(self.G, self.K):
            A = A + sp.kron(sp.csr_matrix(G), sp.kron(sp.csr_matrix(self.Bt), K))
        return self._apply_dirichlet(A, self.n_xi * self.n_t)

    def apply_route1(self, x: np.ndarray) -> np.ndarray:
        return self.assemble_full() @ x

    # --- route 2 ------------------------------------------------------------------------------
    def apply_route2(self, x: np.ndarray) -> np.ndarray:
        bm = self.full_boundary_mask()
        xin = np.where(bm, 0.0, x)
        X = xin.reshape(self.n_xi * self.n_t, self.n_x).T           # X[node, (alpha, i)]
        TA = np.kron(np.eye(self.n_xi), self.At)
        Y = (self.Mx @ X) @ TA.T
        for G, K in zip(self.G, self.K):
            Y = Y + (K @ X) @ np.kron(G, self.Bt).T
        y = Y.T.reshape(-1).copy()
        y[bm] = x[bm]
        return y

    # --- stochastic diagonal block (mean-based, affine coefficient) ----------------------------
    def mean_block(self) -> sp.csr_matrix:
        """A_0 = A_t (x) M_x + B_t (x) K_{a_0} with Dirichlet identity rows (one mode, N_t N_x)."""
        A = sp.kron(sp.csr_matrix(self.At), self.Mx) + sp.kron(sp.csr_matrix(self.Bt), self.K[self.mu0])
        return self._apply_dirichlet(A, self.n_t)

    def diagonal_block(self, a: int) -> sp.csr_matrix:
        """A_alpha = A_t (x) M_x + sum_mu [G_mu]_{alpha alpha} B_t (x) K_mu (Remark solver-matrix-free-sg)."""
        A = sp.kron(sp.csr_matrix(self.At), self.Mx)
        for G, K in zip(self.G, self.K):
            if G[a, a] != 0.0:
                A = A + G[a, a] * sp.kron(sp.csr_matrix(self.Bt), K)
        return self._apply_dirichlet(A, self.n_t)

    def apply_block_diagonal(self, x: np.ndarray) -> np.ndarray:
        """(I_xi (x) A_0) x, one mode at a time."""
        A0 = self.mean_block()
        X = x.reshape(self.n_xi, self.n_t * self.n_x)
        return np.concatenate([A0 @ X[a] for a in range(self.n_xi)])


def from_workload(w, level: int = 0, coef_fn=None) -> SlabProblem:
    """Build the oracle problem of a workload (sg_inputs.Workload) on multigrid level ``level``."""
    import sg_inputs
    n = w.n_cells_1d >> level
    mesh = fem.Mesh(w.dim, n, w.fe_degree, w.lo, w.hi)
    fn = coef_fn or sg_inputs.coefficient_modes
    mus, vals = fn(w, mesh.qp_coords())
    return SlabProblem(w.dim, n, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree,
                       mus, vals, w.lo, w.hi)
