"""Gradient of the mean/variance quantity of interest of a slab sequence by the adjoint sweep.

Host orchestration over the slab library (libsgheat.so); every numerical step runs in its kernels:
slab solves (FGMRES + GMG/Vanka), the slab transfer, the QoI and its gradient, the cell-wise
bilinear forms.  The sequence (Problem tensor-product-slab-system, no forcing):

    AA U^(1) = B_0,   AA U^(n) = JJ U^(n-1),   JJ = I (x) C_t (x) M_x           (eq. local_rhs_tensor)
    J = E[Q] + Var[Q],  Q(xi) = int_D u(x, T, xi)^2 dx                           (Section 3.1)
    AA^T lam^(N) = dJ/dU^(N),   AA^T lam^(n) = JJ^T lam^(n+1)
    dJ/dtheta_m = -sum_n lam^(n)^T (G_{e_m} (x) B_t (x) K_{phi_m}) U^(n)
    dJ/da_{0,K} = -sum_n lam^(n)^T (I (x) B_t (x) K_{chi_K}) U^(n)

for a(x, xi) = a_0(x) + sum_m theta_m phi_m(x) xi_m with a_0 constant on every cell.  AA^T is the
slab operator of a handle created with transpose = 1 (A_t transposed, every other factor symmetric).

Checkpointing: the forward sweep keeps only the end-of-slab traces (N_xi x N_x per slab); the
backward sweep recomputes each slab's solution from the previous trace before using it.
"""
from __future__ import annotations

import numpy as np

from . import sgheat


class Checkpoint:
    """State of one forward sweep: its parameters, slab-end traces, final slab vector and dJ/dU."""

    def __init__(self, theta, a0, traces, u_last, grad_u):
        self.theta, self.a0 = theta, a0
        self.traces, self.u_last, self.grad_u = traces, u_last, grad_u


class SlabSequence:
    """Forward and adjoint sweeps of one sg_inputs.AdjointWorkload on the GPU."""

    def __init__(self, aw, rtol: float = 1e-10, max_iter: int = 500, precision=sgheat.SG_FP64):
        import torch
        import sg_inputs
        self.aw = aw
        self.w = w = aw.base
        self.rtol, self.max_iter, self.precision = rtol, max_iter, precision
        self.spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree,
                                w.n_levels, w.lo, w.hi, w.pre_smooth, w.post_smooth, w.vanka_omega, w.fgmres_restart)
        self.qp = [sgheat.quadrature_points(self.spec, lvl) for lvl in range(w.n_levels)]
        self.nodes = sgheat.node_coordinates(self.spec, 0)
        self.n_x = self.nodes.shape[0]
        self.n_xi, self.n_t = w.n_chaos, w.n_time
        self.dev = torch.device("cuda:0")
        u0 = sg_inputs.initial_value(self.nodes)
        bnd = self._boundary_mask()
        u0[bnd] = 0.0
        self.u0 = u0
        self.phi_qp = [sg_inputs.sine_shape_at(m, self.qp[0]) for m in range(1, w.n_vars + 1)]
        self.ones_qp = np.ones(self.qp[0].shape[:2])
        self.G = self.GT = None
        self.stats = {}
        self.checkpoint = None

    def _boundary_mask(self) -> np.ndarray:
        n1 = self.w.n_cells_1d * self.w.fe_degree + 1
        idx = np.arange(self.n_x)
        bnd = np.zeros(self.n_x, dtype=bool)
        for _ in range(self.w.dim):
            i = idx % n1
            bnd |= (i == 0) | (i == n1 - 1)
            idx = idx // n1
        return bnd

    # --- problem set-up for one parameter value ---------------------------------------------------
    def set_parameters(self, theta, a0_cells):
        """Coefficients for (theta, a0): the handles are made once and updated in place afterwards."""
        import sg_inputs
        mus, coef = sg_inputs.adjoint_coef_levels(self.aw, np.asarray(theta, dtype=np.float64),
                                                  np.asarray(a0_cells, dtype=np.float64),
                                                  lambda lvl: self.qp[lvl])
        if self.G is None:
            self.G = sgheat.Problem(self.spec, mus, coef, self.precision)
            specT = sgheat.Spec(**{**self.spec.__dict__, "transpose": 1})
            self.GT = sgheat.Problem(specT, mus, coef, self.precision)
        else:
            self.G.update_coefficients(coef)
            self.GT.update_coefficients(coef)
        self.theta = np.asarray(theta, dtype=np.float64).copy()
        self.a0 = np.asarray(a0_cells, dtype=np.float64).copy()

    def close(self):
        for P in (self.G, self.GT):
            if P is not None:
                P.close()
        self.G = self.GT = None

    # --- helpers ---------------------------------------------------------------------------------
    def _zeros(self):
        import torch
        return torch.zeros(self.n_xi * self.n_t * self.n_x, dtype=torch.float64, device=self.dev)

    def _trace_to_slab(self, trace, out):
        """Slab vector carrying `trace` [N_xi, N_x] as its end-of-slab component (others 0)."""
        out.zero_()
        v = out.view(self.n_xi, self.n_t, self.n_x)
        v[:, self.n_t - 1, :] = trace
        return out

    def _solve(self, P, b, x, info_key):
        x.zero_()
        _, info = P.solve(b, x, rtol=self.rtol, max_iter=self.max_iter)
        self.stats.setdefault(info_key, []).append(info["iterations"])
        return x

    # --- sweeps -----------------------------------------------------------------------------------
    def forward(self, theta, a0_cells):
        """Forward sweep; returns (J, E[Q], Var[Q]) and keeps the slab-end checkpoints."""
        import torch
        self.set_parameters(theta, a0_cells)
        self.stats = {}
        x0 = self._zeros()
        v = x0.view(self.n_xi, self.n_t, self.n_x)
        v[0, self.n_t - 1, :] = torch.from_numpy(self.u0).to(self.dev)
        b = self.G.slab_transfer(x0)                       # B_0
        u = self._zeros()
        self.traces = []
        for n in range(self.aw.n_slabs):
            self._solve(self.G, b, u, "forward_iterations")
            self.traces.append(u.view(self.n_xi, self.n_t, self.n_x)[:, self.n_t - 1, :].clone())
            b = self.G.slab_transfer(u, b)
        self.u_last = u
        self.grad_u = self._zeros()
        EQ, VQ = self.G.qoi_mean_var(u, 1.0, 1.0, grad=self.grad_u)
        self.J = EQ + VQ
        # everything backward() needs, kept apart from the next forward sweep's state
        self.checkpoint = Checkpoint(self.theta, self.a0, self.traces, self.u_last, self.grad_u)
        return self.J, EQ, VQ

    def backward(self, checkpoint=None):
        """Adjoint sweep; returns (dJ/dtheta [M], dJ/da0 [n_cells]) at the parameters of `checkpoint`
        (a forward() result; default: the latest one).  If another forward sweep ran since, the
        coefficients of that checkpoint are set again before the sweep."""
        ck = self.checkpoint if checkpoint is None else checkpoint
        if ck is None:
            raise RuntimeError("backward() needs a forward() sweep first")
        if not (np.array_equal(ck.theta, self.theta) and np.array_equal(ck.a0, self.a0)):
            self.set_parameters(ck.theta, ck.a0)
        self.traces, self.u_last, self.grad_u = ck.traces, ck.u_last, ck.grad_u
        import torch
        M = self.w.n_vars
        n_cells = self.qp[0].shape[0]
        # both gradients accumulate on the device over the slabs; one copy to the host at the end
        dth = torch.zeros(M, dtype=torch.float64, device=self.dev)
        da0 = torch.zeros(n_cells, dtype=torch.float64, device=self.dev)
        rhs = self.grad_u
        rhs_buf = self._zeros()
        lam = self._zeros()
        u = self._zeros()
        b = self._zeros()
        tmp = self._zeros()
        for n in reversed(range(self.aw.n_slabs)):
            self._solve(self.GT, rhs, lam, "adjoint_iterations")
            # recompute U^(n) from the checkpoint of slab n - 1 (or the initial value)
            if n == self.aw.n_slabs - 1:
                u_n = self.u_last
            else:
                if n == 0:
                    t0 = torch.zeros(self.n_xi, self.n_x, dtype=torch.float64, device=self.dev)
                    t0[0] = torch.from_numpy(self.u0).to(self.dev)
                    self._trace_to_slab(t0, tmp)
                else:
                    self._trace_to_slab(self.traces[n - 1], tmp)
                self.G.slab_transfer(tmp, b)
                u_n = self._solve(self.G, b, u, "recompute_iterations")
            for m in range(M):
                self.G.stiffness_form_accumulate(m + 1, self.phi_qp[m], lam, u_n, -1.0, total=dth[m:m + 1])
            self.G.stiffness_form_accumulate(0, self.ones_qp, lam, u_n, -1.0, cells=da0)
            rhs = self.G.slab_transfer(lam, rhs_buf, transpose=True)
        return dth.cpu().numpy(), da0.cpu().numpy()

    def gradient(self, theta, a0_cells):
        J, EQ, VQ = self.forward(theta, a0_cells)
        dth, da0 = self.backward()
        return J, (EQ, VQ), dth, da0


def make_function():
    """torch.autograd.Function computing J(theta, a0) with the adjoint gradient in backward."""
    import torch

    class SlabQoI(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, a0, seq):
            J, _, _ = seq.forward(theta.detach().cpu().numpy(), a0.detach().cpu().numpy())
            ctx.seq = seq
            ctx.checkpoint = seq.checkpoint      # backward uses this sweep's state, not the latest one
            ctx.dtypes = (theta.dtype, theta.device, a0.dtype, a0.device)
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            dth, da0 = ctx.seq.backward(ctx.checkpoint)
            tdt, tdev, adt, adev = ctx.dtypes
            g = float(gJ)
            return (torch.as_tensor(g * dth, dtype=tdt, device=tdev), torch.as_tensor(g * da0, dtype=adt, device=adev),
                    None)

    return SlabQoI
