"""Monte-Carlo pathwise slab sequences of a batch of samples on one GPU (Section 5).

Host orchestration over the slab library (libsgheat.so); every numerical step runs in its kernels.
All samples of the batch live in one sample-batch handle (``samples`` given at creation): the slab
vector is [sample][time DoF][node], row block s is the deterministic slab system of the sampled
coefficient a(x, xi^(s)) (eq. mc-slab-system), so one operator apply, one Vanka sweep or one
V-cycle advances every sample at once and the coefficient fields a_mu are read once per cell for the
whole batch.  The slab solve is one FGMRES over the batch (the stopping test is on the residual of
the whole batch), preconditioned by the V-cycle of the mean operator A_0 on every sample.

Per slab n (Algorithm alg:mc-fem, time loop of every sample):
    b = (I (x) C_t (x) M_x) U^(n-1)    (the initial value u_0 for n = 1)
    U^(n) = AA_batch^{-1} b
and at the end the sample mean and unbiased sample variance of the last slab (eqs. mc-mean-estimator,
mc-variance-estimator-unbiased).
"""
from __future__ import annotations

import numpy as np

from . import sgheat


class SampleBatch:
    """The slab sequences of one sg_inputs.SampleWorkload (or of explicit samples)."""

    def __init__(self, sw, samples=None, rtol: float = 1e-10, max_iter: int = 500, precision=sgheat.SG_FP64,
                 diag_blocks: int = 0):
        import torch
        import sg_inputs
        self.sw = sw
        self.w = w = sw.base
        self.samples = np.ascontiguousarray(sw.samples() if samples is None else samples, dtype=np.float64)
        self.rtol, self.max_iter = rtol, max_iter
        self.spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, 0, w.n_levels,
                                w.lo, w.hi, w.pre_smooth, w.post_smooth, w.vanka_omega, w.fgmres_restart,
                                diag_blocks=diag_blocks)
        mus, coef = sg_inputs.coef_qp_levels(w, lambda lvl: sgheat.quadrature_points(self.spec, lvl))
        self.P = sgheat.Problem(self.spec, mus, coef, precision, samples=self.samples)
        self.n_s, self.n_t, self.n_x = self.P.shape
        self.dev = torch.device("cuda:0")
        nodes = sgheat.node_coordinates(self.spec, 0)
        u0 = sg_inputs.initial_value(nodes)
        n1 = w.n_cells_1d * w.fe_degree + 1
        idx = np.arange(self.n_x)
        for _ in range(w.dim):
            i = idx % n1
            u0[(i == 0) | (i == n1 - 1)] = 0.0
            idx = idx // n1
        self.u0 = torch.from_numpy(u0).to(self.dev)
        self.info = []

    def close(self):
        if self.P is not None:
            self.P.close()
            self.P = None

    def _zeros(self):
        import torch
        return torch.zeros(self.n_s * self.n_t * self.n_x, dtype=torch.float64, device=self.dev)

    def first_rhs(self, out=None):
        """B_0: the transfer of u_0 placed as the end-of-slab trace of every sample."""
        x0 = self._zeros()
        x0.view(self.n_s, self.n_t, self.n_x)[:, self.n_t - 1, :] = self.u0
        return self.P.slab_transfer(x0, out)

    def run(self, n_slabs: int | None = None):
        """March n_slabs slabs (default: the workload's); returns the last slab vector [n_s*N_t*N_x]."""
        n_slabs = self.sw.n_slabs if n_slabs is None else n_slabs
        b = self.first_rhs()
        u = self._zeros()
        self.info = []
        for _ in range(n_slabs):
            u.zero_()
            _, info = self.P.solve(b, u, rtol=self.rtol, max_iter=self.max_iter)
            self.info.append(info)
            if not info["converged"]:
                raise sgheat.SgError(sgheat.SG_NOT_CONVERGED, "a slab solve of the sample batch did not converge")
            b = self.P.slab_transfer(u, b)
        return u

    def statistics(self, u, with_variance: bool = True):
        """Sample mean and unbiased sample variance of a batch slab vector, each [N_t, N_x]."""
        import torch
        m = self.n_t * self.n_x
        var = torch.empty(m, dtype=torch.float64, device=u.device) if with_variance else None
        mean, var = self.P.sample_statistics(u, var=var)
        return mean.view(self.n_t, self.n_x), (var.view(self.n_t, self.n_x) if var is not None else None)
