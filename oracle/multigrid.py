"""Stochastic block-Jacobi preconditioner: geometric multigrid V-cycle with a Vanka smoother.

Test infrastructure (oracle): see the package docstring.

Remark solver-matrix-free-sg: each stochastic diagonal block A_alpha is preconditioned by one V-cycle
of a space-time geometric multigrid whose smoother solves local dense patch problems.  For an affine
coefficient [G_{e_m}]_{alpha alpha} = 0, so every diagonal block equals the mean block
A_0 = A_t (x) M_x + B_t (x) K_{a_0}; one hierarchy serves all modes.

Readings where the paper is silent (each also listed in the design notes):
  * patch of cell K: the non-Dirichlet nodes of the closed cell times all N_t time DoFs of the slab;
  * patch matrix: the restriction of the assembled A_0 (not the element matrix), solved exactly
    by LU with partial pivoting;
  * the smoother is additive over all cells, each patch correction weighted by 1 / (number of cells
    containing the node), damped by omega; Dirichlet DoFs are set to the right-hand side;
  * coarse operators are rediscretised on every level from that level's coefficient values;
  * prolongation P = nodal interpolation of the coarse Q_k function at the fine nodes, zero on
    Dirichlet nodes, applied to each time component; restriction R = P^T;
  * coarsest level: dense LU of A_0 on its interior DoFs.
With per-mode diagonal blocks (a non-affine coefficient, where [G_mu]_{alpha alpha} != 0 for even mu),
mode alpha gets its own hierarchy built the same way from A_alpha = A_t (x) M_x +
sum_mu [G_mu]_{alpha alpha} B_t (x) K_mu on every level.
Vectors here hold one stochastic mode: layout [i][node], length N_t N_x.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem
from .slab import SlabProblem


class Level:
    def __init__(self, prob: SlabProblem, block: int | None = None):
        """The mean block A_0, or with block = alpha the diagonal block A_alpha."""
        self.prob = prob
        self.mesh = prob.mesh
        self.n_t = prob.n_t
        self.A0 = prob.mean_block() if block is None else prob.diagonal_block(block)
        self.bdof = np.tile(prob.bmask, self.n_t)          # Dirichlet DoFs of one mode
        self.ndof = self.A0.shape[0]
        mult = np.zeros(self.mesh.n_nodes)
        cells = self.mesh.all_cell_dofs()
        for c in range(self.mesh.n_cells):
            mult[cells[c]] += 1.0
        self.weight_node = 1.0 / mult
        self.patches = []
        A0d = self.A0.tolil()
        for c in range(self.mesh.n_cells):
            nodes = [g for g in cells[c] if not prob.bmask[g]]
            dofs = np.array([i * self.mesh.n_nodes + g for i in range(self.n_t) for g in nodes],
                            dtype=np.int64)
            if len(dofs) == 0:
                continue
            Ak = self.A0[dofs][:, dofs].toarray()
            lu = sla.lu_factor(Ak)
            w = np.tile(self.weight_node[nodes], self.n_t)
            self.patches.append((dofs, lu, w))

    def residual(self, b, x):
        return b - self.A0 @ x

    def vanka(self, b, x, sweeps, omega):
        """Additive weighted Vanka sweeps: x <- x + omega sum_K R_K^T W_K A_{0,K}^{-1} R_K (b - A_0 x)."""
        x = x.copy()
        for _ in range(sweeps):
            r = self.residual(b, x)
            corr = np.zeros_like(x)
            for dofs, lu, w in self.patches:
                corr[dofs] += w * sla.lu_solve(lu, r[dofs])
            x = x + omega * corr
            x[self.bdof] = b[self.bdof]
        return x

    def exact(self, b):
        inner = ~self.bdof
        A = self.A0[inner][:, inner].toarray()
        x = b.copy()
        x[inner] = sla.lu_solve(sla.lu_factor(A), b[inner])
        return x


def prolongation(fine: Level, coarse: Level) -> sp.csr_matrix:
    """P for one mode: kron(I_{N_t}, D_f I D_c) with D the interior masks."""
    I = fem.interpolation_matrix(fine.mesh, coarse.mesh)
    Df = sp.diags((~fine.prob.bmask).astype(np.float64))
    Dc = sp.diags((~coarse.prob.bmask).astype(np.float64))
    return sp.kron(sp.identity(fine.n_t), Df @ I @ Dc).tocsr()


class Hierarchy:
    """Levels 0 (finest) .. L-1 (coarsest)."""

    def __init__(self, problems: list[SlabProblem], pre=1, post=1, omega=1.0, block: int | None = None):
        self.levels = [Level(p, block) for p in problems]
        self.P = [prolongation(self.levels[l], self.levels[l + 1]) for l in range(len(problems) - 1)]
        self.pre, self.post, self.omega = pre, post, omega

    def vcycle_level(self, l, b):
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            return lev.exact(b)
        x = np.zeros_like(b)
        x = lev.vanka(b, x, self.pre, self.omega)
        r = lev.residual(b, x)
        bc = self.P[l].T @ r
        xc = self.vcycle_level(l + 1, bc)
        x = x + self.P[l] @ xc
        x = lev.vanka(b, x, self.post, self.omega)
        return x

    def vcycle_mode(self, r):
        return self.vcycle_level(0, r)

    def vcycle(self, r_all: np.ndarray, n_xi: int) -> np.ndarray:
        """Block-Jacobi over the modes: one V-cycle per stochastic mode (layout [alpha][i][node])."""
        R = r_all.reshape(n_xi, -1)
        return np.concatenate([self.vcycle_mode(R[a]) for a in range(n_xi)])

    def smooth(self, level: int, b_all, x_all, sweeps: int, n_xi: int):
        B = b_all.reshape(n_xi, -1)
        X = x_all.reshape(n_xi, -1)
        lev = self.levels[level]
        return np.concatenate([lev.vanka(B[a], X[a], sweeps, self.omega) for a in range(n_xi)])


def hierarchy_from_workload(w, coef_fn=None) -> Hierarchy:
    from .slab import from_workload
    probs = [from_workload(w, l, coef_fn) for l in range(w.n_levels)]
    return Hierarchy(probs, w.pre_smooth, w.post_smooth, w.vanka_omega)


class BlockHierarchies:
    """Block-Jacobi over the modes with each mode's own diagonal block on every level."""

    def __init__(self, problems: list[SlabProblem], pre=1, post=1, omega=1.0):
        self.h = [Hierarchy(problems, pre, post, omega, block=a) for a in range(problems[0].n_xi)]

    def vcycle(self, r_all: np.ndarray, n_xi: int) -> np.ndarray:
        R = r_all.reshape(n_xi, -1)
        return np.concatenate([self.h[a].vcycle_mode(R[a]) for a in range(n_xi)])


def block_hierarchies_from_workload(w, coef_fn=None) -> BlockHierarchies:
    from .slab import from_workload
    probs = [from_workload(w, l, coef_fn) for l in range(w.n_levels)]
    return BlockHierarchies(probs, w.pre_smooth, w.post_smooth, w.vanka_omega)
