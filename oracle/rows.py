"""Selected rows of the slab operator, evaluated from the definition one node at a time.

Test infrastructure (oracle): see the package docstring.

For full-size problems the oracle does not assemble the global matrices; a row (alpha, i, m) of
    AA = I (x) A_t (x) M_x + sum_mu G_mu (x) B_t (x) K_mu     (eq. local_rhs_tensor)
only involves the cells whose closure contains node m, so it is summed from those cells' element
matrices (the same plain quadrature as fem.Mesh.element_matrices).  Dirichlet rows are identity
rows and Dirichlet columns are dropped, as in slab.SlabProblem.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import chaos, fem, timebasis


class RowOracle:
    def __init__(self, dim, n_cells_1d, fe_degree, time_degree, tau, n_vars, chaos_degree, coef_mu,
                 coef_fn, lo=0.0, hi=1.0):
        """coef_fn(points[..., d]) -> values [n_mu, ...] of a_mu at physical points."""
        self.mesh = fem.Mesh(dim, n_cells_1d, fe_degree, lo, hi)
        self.At, self.Bt, _ = timebasis.time_matrices(time_degree, tau)
        self.index_set = chaos.total_degree_set(n_vars, chaos_degree)
        self.G = [chaos.galerkin_tensor(tuple(mu), self.index_set) for mu in coef_mu]
        self.coef_fn = coef_fn
        self.n_xi, self.n_t, self.n_x = len(self.index_set), time_degree + 1, self.mesh.n_nodes
        self.phi, self.dphi, self.w = self.mesh.ref_tables()
        self.loc = self.mesh.local_multi()

    def _node_multi(self, m):
        out = []
        for _ in range(self.mesh.dim):
            out.append(m % self.mesh.n1)
            m //= self.mesh.n1
        return out

    def _is_boundary(self, idx):
        return any(i == 0 or i == self.mesh.n1 - 1 for i in idx)

    def rows(self, x: np.ndarray, picks):
        """y[(alpha, i, m)] for every (alpha, i, m) in picks."""
        mesh = self.mesh
        X = x.reshape(self.n_xi, self.n_t, self.n_x)
        out = []
        cache = {}
        for (a, i, m) in picks:
            idx = self._node_multi(m)
            if self._is_boundary(idx):
                out.append(X[a, i, m])
                continue
            if m not in cache:
                cache[m] = self._node_row_blocks(idx)
            acc = 0.0
            for dofs, Mrow, Krows in cache[m]:
                xin = X[:, :, dofs]                               # [n_xi, n_t, nloc]
                mass = Mrow @ xin[a].T                            # [n_t]
                acc += self.At[i] @ mass
                for G, Krow in zip(self.G, Krows):
                    gk = Krow @ xin[:, i, :].T                    # [n_xi]
                    acc += self.Bt[i, i] * (G[a] @ gk)
                    # B_t is diagonal for the right-Radau basis; the off-diagonal part is added too
                    for j in range(self.n_t):
                        if j != i:
                            acc += self.Bt[i, j] * (G[a] @ (Krow @ xin[:, j, :].T))
            out.append(acc)
        return np.array(out)

    def _node_row_blocks(self, idx):
        mesh = self.mesh
        k = mesh.k
        blocks = []
        ranges = []
        for d in range(mesh.dim):
            c = []
            if idx[d] % k == 0:
                if idx[d] // k - 1 >= 0:
                    c.append(idx[d] // k - 1)
                if idx[d] // k <= mesh.n - 1:
                    c.append(idx[d] // k)
            else:
                c.append(idx[d] // k)
            ranges.append(c)
        for cm in itertools.product(*ranges):
            cell = 0
            for d in reversed(range(mesh.dim)):
                cell = cell * mesh.n + cm[d]
            dofs = mesh.cell_dofs(cell).copy()
            loc_a = [idx[d] - cm[d] * k for d in range(mesh.dim)]
            a = self.loc.index(tuple(loc_a))
            # Dirichlet columns dropped
            bm = np.array([self._is_boundary(self._node_multi(g)) for g in dofs])
            pts = np.empty((mesh.nq, mesh.dim))
            for q, qm in enumerate(self.loc):
                for d in range(mesh.dim):
                    pts[q, d] = mesh.lo + mesh.h * (cm[d] + mesh.qpt[qm[d]])
            coef = self.coef_fn(pts)                          # [n_mu, nq]
            vol = mesh.h ** mesh.dim
            Mrow = np.einsum("q,q,qb->b", self.w * vol, self.phi[:, a], self.phi)
            gg = np.einsum("qe,qbe->qb", self.dphi[:, a, :], self.dphi) / mesh.h ** 2
            Krows = [np.einsum("q,q,qb->b", coef[mu], self.w * vol, gg) for mu in range(len(self.G))]
            Mrow[bm] = 0.0
            for Kr in Krows:
                Kr[bm] = 0.0
            blocks.append((dofs, Mrow, Krows))
        return blocks
