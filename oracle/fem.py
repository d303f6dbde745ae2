"""Conforming Q_k finite elements on a uniform Cartesian mesh of (lo, hi)^d, d in {2, 3}.

Test infrastructure (oracle): see the package docstring.

Section 2.4: nodal Lagrange basis of Q_k on quadrilaterals / hexahedra, globally continuous, with the
homogeneous Dirichlet condition.  Readings where the paper is silent:
  * support points: Gauss-Lobatto-Legendre (GLL) points of the reference interval (0, 1);
  * quadrature: tensor Gauss-Legendre rule with k+1 points per direction;
  * the coefficient enters only through its values a_mu(x_q) at those quadrature points;
  * numbering: nodes lexicographic with x fastest (index i_x + N1 (i_y + N1 i_z), N1 = n k + 1),
    cells lexicographic with x fastest, local nodes and quadrature points lexicographic x fastest;
  * boundary nodes are part of the vector (the paper counts them: N_x = 148225 = 385^2).
Element matrices are plain quadrature sums over all (k+1)^d points, assembled into scipy CSR.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as L

from .timebasis import lagrange_value, lagrange_deriv


def gll_points(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto-Legendre points on [0, 1]: end points and the roots of P_k'."""
    if k == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(k + 1)
    c[k] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(c))))
    s = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (s + 1.0)


def gauss_rule(n: int):
    """n-point Gauss-Legendre rule on [0, 1]."""
    g, w = L.leggauss(n)
    return 0.5 * (g + 1.0), 0.5 * w


class Mesh:
    """Uniform Cartesian mesh with n cells per direction and Q_k elements."""

    def __init__(self, dim: int, n: int, k: int, lo: float = 0.0, hi: float = 1.0):
        self.dim, self.n, self.k, self.lo, self.hi = dim, n, k, lo, hi
        self.h = (hi - lo) / n
        self.n1 = n * k + 1
        self.n_nodes = self.n1 ** dim
        self.n_cells = n ** dim
        self.nq1 = k + 1
        self.nq = self.nq1 ** dim
        self.nloc = (k + 1) ** dim
        self.support = gll_points(k)
        self.qpt, self.qwt = gauss_rule(k + 1)

    # --- numbering -------------------------------------------------------------------------
    def cell_multi(self, c: int) -> tuple[int, ...]:
        out = []
        for _ in range(self.dim):
            out.append(c % self.n)
            c //= self.n
        return tuple(out)

    def node_index(self, idx) -> int:
        g = 0
        for dd in reversed(range(self.dim)):
            g = g * self.n1 + idx[dd]
        return g

    def local_multi(self):
        """Local node / quadrature multi-indices, lexicographic with x fastest."""
        return [tuple(reversed(t)) for t in itertools.product(range(self.k + 1), repeat=self.dim)]

    def cell_dofs(self, c: int) -> np.ndarray:
        cm = self.cell_multi(c)
        return np.array([self.node_index([cm[d] * self.k + a[d] for d in range(self.dim)])
                         for a in self.local_multi()])

    def all_cell_dofs(self) -> np.ndarray:
        return np.stack([self.cell_dofs(c) for c in range(self.n_cells)])

    def node_coords(self) -> np.ndarray:
        """Physical coordinates of every node, shape [n_nodes, d]."""
        pts1 = np.empty(self.n1)
        for c in range(self.n):
            for a in range(self.k + 1):
                pts1[c * self.k + a] = self.lo + self.h * (c + self.support[a])
        grids = np.meshgrid(*([pts1] * self.dim), indexing="ij")
        # node index i_x + n1 (i_y + ...): x fastest, so reverse the axis order before flattening
        return np.stack([g.transpose(*reversed(range(self.dim))).reshape(-1) for g in grids], axis=-1)

    def boundary_mask(self) -> np.ndarray:
        """True on nodes of the domain boundary (homogeneous Dirichlet, eq. heat_bc)."""
        idx = np.indices([self.n1] * self.dim).reshape(self.dim, -1)[::-1]  # idx[0] = i_x
        m = np.zeros(self.n_nodes, dtype=bool)
        # np.indices enumerates with the last axis fastest; map to our numbering explicitly
        flat = np.zeros(self.n_nodes, dtype=np.int64)
        for dd in reversed(range(self.dim)):
            flat = flat * self.n1 + idx[dd]
        for dd in range(self.dim):
            m[flat[(idx[dd] == 0) | (idx[dd] == self.n1 - 1)]] = True
        return m

    def qp_coords(self) -> np.ndarray:
        """Physical quadrature points, shape [n_cells, nq, d] (cells and points x fastest)."""
        out = np.empty((self.n_cells, self.nq, self.dim))
        loc = self.local_multi()
        for c in range(self.n_cells):
            cm = self.cell_multi(c)
            for q, a in enumerate(loc):
                for d in range(self.dim):
                    out[c, q, d] = self.lo + self.h * (cm[d] + self.qpt[a[d]])
        return out

    # --- reference-cell tables ----------------------------------------------------------------
    def ref_tables(self):
        """phi[q, a], dphi[q, a, dir] on the reference cell (0,1)^d, and tensor weights w[q]."""
        k = self.k
        v1 = np.array([[lagrange_value(self.support, a, np.array(x)) for a in range(k + 1)]
                       for x in self.qpt])
        d1 = np.array([[lagrange_deriv(self.support, a, np.array(x)) for a in range(k + 1)]
                       for x in self.qpt])
        loc = self.local_multi()
        nq = nl = len(loc)
        phi = np.empty((nq, nl))
        dphi = np.empty((nq, nl, self.dim))
        w = np.empty(nq)
        for q, qm in enumerate(loc):
            w[q] = np.prod([self.qwt[qm[d]] for d in range(self.dim)])
            for a, am in enumerate(loc):
                phi[q, a] = np.prod([v1[qm[d], am[d]] for d in range(self.dim)])
                for e in range(self.dim):
                    dphi[q, a, e] = np.prod([(d1 if d == e else v1)[qm[d], am[d]]
                                             for d in range(self.dim)])
        return phi, dphi, w

    # --- assembly ---------------------------------------------------------------------------
    def element_matrices(self, coef_cell_qp: np.ndarray | None):
        """Mass (coef None) or stiffness element matrices for every cell: [n_cells, nl, nl].

        M_K[a, b] = sum_q w_q |K| phi_a phi_b,  K_K[a, b] = sum_q w_q |K| a(x_q) grad phi_a . grad phi_b
        with |K| = h^d and reference gradients scaled by 1/h.
        """
        phi, dphi, w = self.ref_tables()
        vol = self.h ** self.dim
        if coef_cell_qp is None:
            Me = np.einsum("q,qa,qb->ab", w * vol, phi, phi)
            return np.broadcast_to(Me, (self.n_cells,) + Me.shape)
        gg = np.einsum("qae,qbe->qab", dphi, dphi) / (self.h ** 2)
        return np.einsum("cq,q,qab->cab", coef_cell_qp, w * vol, gg)

    def assemble(self, elem: np.ndarray) -> sp.csr_matrix:
        dofs = self.all_cell_dofs()
        nl = dofs.shape[1]
        rows = np.repeat(dofs, nl, axis=1).reshape(-1)
        cols = np.tile(dofs, (1, nl)).reshape(-1)
        A = sp.coo_matrix((np.asarray(elem).reshape(-1), (rows, cols)),
                          shape=(self.n_nodes, self.n_nodes))
        return A.tocsr()

    def mass(self) -> sp.csr_matrix:
        return self.assemble(self.element_matrices(None))

    def stiffness(self, coef_cell_qp: np.ndarray) -> sp.csr_matrix:
        return self.assemble(self.element_matrices(coef_cell_qp))


def interpolation_matrix(fine: Mesh, coarse: Mesh) -> sp.csr_matrix:
    """I[f, c] = phi_c^{coarse}(x_f): nodal interpolation of coarse Q_k functions at fine nodes.

    The two meshes cover the same domain and fine.n = 2 coarse.n.  Each fine node is evaluated in
    one coarse cell that contains it (the coarse function is continuous, so any choice agrees).
    """
    assert fine.n == 2 * coarse.n and fine.k == coarse.k and fine.dim == coarse.dim
    X = fine.node_coords()
    rows, cols, vals = [], [], []
    loc = coarse.local_multi()
    for f in range(fine.n_nodes):
        cm = []
        ref = []
        for d in range(fine.dim):
            t = (X[f, d] - coarse.lo) / coarse.h
            c = min(int(math.floor(t + 1e-12)), coarse.n - 1)
            cm.append(c)
            ref.append(t - c)
        c_index = 0
        for d in reversed(range(fine.dim)):
            c_index = c_index * coarse.n + cm[d]
        dofs = coarse.cell_dofs(c_index)
        for a, am in enumerate(loc):
            v = 1.0
            for d in range(fine.dim):
                v *= float(lagrange_value(coarse.support, am[d], np.array(ref[d])))
            if abs(v) > 1e-14:
                rows.append(f)
                cols.append(dofs[a])
                vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_nodes, coarse.n_nodes))
