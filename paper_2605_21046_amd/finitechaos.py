"""The finite-chaos benchmark on one GPU: forcing, slab-by-slab time marching and error quantities.

Host orchestration over the slab library (libsgheat.so); every vector-sized step runs in its
kernels.  Benchmark (Section 3.2): D = (-1, 1)^2, T = 1, M = 4, the non-affine coefficient
a = d_min + (xi_1 x_1^2 + xi_2 x_1 x_2 + xi_3 x_2^2 + xi_4)^2 (11 Hermite modes), the exact solution
u = t^4 s(x) G_q(xi), s = sin(pi (x_1+1)/2) sin(pi (x_2+1)/2), G_q = sum_{|alpha| <= 6} c_alpha Psi_alpha.

Forcing (eq. finite_rhs_factorized projected on Psi_beta, divergence integrated by parts):
    F^(n)_beta = c_beta T1^(n) (x) m + sum_mu D[mu, beta] T2^(n) (x) k_mu,
    m_j = (s, psi_j),  k_mu,j = (a_mu grad s, grad psi_j)          (sg_load_vectors, once)
    D[mu, beta] = sum_alpha c_alpha E[Psi_mu Psi_alpha Psi_beta]     (sg_chaos_projection, once)
    T1_i = int_{I_n} 4 t^3 v_i,  T2_i = int_{I_n} t^4 v_i            (sg_time_load_weights, per slab)
assembled per slab by sg_separable_vector on top of the transfer JJ U^(n-1) (sg_slab_transfer).
Errors (Definition def:error-norms-and-quantities): sg_separable_error per slab, summed; the modes of
Lambda_q outside the computed set add c_alpha^2 |phi|^2 to the full errors.
"""
from __future__ import annotations

import math

import numpy as np

from . import sgheat


class FiniteChaosRun:
    """One stochastic degree p_xi of the benchmark (an sg_inputs.FiniteChaosWorkload)."""

    def __init__(self, fw, precision=sgheat.SG_FP64, rtol: float = 1e-10, max_iter: int = 2000, diag_blocks: int = 0):
        import torch
        import sg_inputs
        self.fw = fw
        w = fw.base
        self.rtol, self.max_iter = rtol, max_iter
        self.P = sgheat.problem_from_workload(w, precision, diag_blocks=diag_blocks)
        self.spec = self.P.spec
        self.nq1 = w.fe_degree + 3
        self.ntq = w.time_degree + 3
        dev = torch.device("cuda:0")
        pts = sgheat.gauss_points(self.spec, 0, self.nq1)                 # [cells, nq, 2]
        s, gs = sg_inputs.finite_chaos_phi(pts)
        mus, a = sg_inputs.finite_chaos_coefficient_modes(pts)
        nf = 1 + len(mus)
        fval = np.zeros((nf,) + s.shape)
        fval[0] = s
        fgrad = np.zeros((nf,) + gs.shape)
        for k in range(len(mus)):
            fgrad[1 + k] = a[k][..., None] * gs
        self.V = self.P.load_vectors(self.nq1, torch.from_numpy(fval).to(dev), torch.from_numpy(fgrad).to(dev))
        self.s_qp = torch.from_numpy(np.ascontiguousarray(s)).to(dev)
        self.gs_qp = torch.from_numpy(np.ascontiguousarray(gs)).to(dev)
        alpha = self.P.index_set()
        self.c = np.array([fw.c_alpha(tuple(int(v) for v in al)) for al in alpha])
        la, lc = sg_inputs.finite_chaos_exact_modes()
        self.D = self.P.chaos_projection(la, lc)                          # [n_mu, N_xi]
        self.C2 = float(np.sum(lc[np.any(la != 0, axis=1)] ** 2))
        computed = {tuple(int(v) for v in al) for al in alpha}
        self.tail = float(sum(cc ** 2 for al, cc in zip(la, lc) if tuple(int(v) for v in al) not in computed))
        self.st, _ = self.P.time_rule(self.ntq)
        self.info = []

    def close(self):
        self.P.close()

    def slab_weights(self, n: int) -> np.ndarray:
        """W[t, beta, i] of F^(n): t = 0 the mass load, t = 1 + mu the stiffness loads."""
        t = (n - 1) * self.fw.base.tau + self.fw.base.tau * self.st
        T = self.P.time_load_weights(np.stack([4.0 * t ** 3, t ** 4]))     # [2, N_t]
        W = np.empty((1 + self.D.shape[0], self.P.shape[0], self.P.shape[1]))
        W[0] = self.c[:, None] * T[0][None, :]
        W[1:] = self.D[:, :, None] * T[1][None, None, :]
        return W

    def run(self, n_slabs: int | None = None):
        """March the slabs; returns (errors dict, last slab vector)."""
        import torch
        n_slabs = self.fw.n_slabs if n_slabs is None else n_slabs
        n = self.P.n(0)
        u = torch.zeros(n, dtype=torch.float64, device="cuda")
        rhs = torch.zeros_like(u)
        acc = np.zeros(8)
        self.info = []
        for k in range(1, n_slabs + 1):
            if k == 1:
                self.P.separable_vector(self.slab_weights(k), self.V, rhs, beta=0.0)
            else:
                self.P.slab_transfer(u, rhs)
                self.P.separable_vector(self.slab_weights(k), self.V, rhs, beta=1.0)
            _, info = self.P.solve(rhs, u, rtol=self.rtol, max_iter=self.max_iter)
            self.info.append(info)
            if not info["converged"]:
                raise sgheat.SgError(sgheat.SG_NOT_CONVERGED, f"slab {k} did not converge")
            t = (k - 1) * self.fw.base.tau + self.fw.base.tau * self.st
            acc += self.P.separable_error(u, self.nq1, self.s_qp, self.gs_qp, t ** 4, self.c, self.C2)
        errs = {"E_full_L2": math.sqrt(acc[0] + self.tail * acc[6]), "E_full_H1": math.sqrt(acc[1] + self.tail * acc[7]),
                "E_mean_L2": math.sqrt(acc[2]), "E_mean_H1": math.sqrt(acc[3]),
                "E_var_L2": math.sqrt(acc[4]), "E_var_H1": math.sqrt(acc[5])}
        return errs, u
