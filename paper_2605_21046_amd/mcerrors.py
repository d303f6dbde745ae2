"""Monte-Carlo study of the finite-chaos benchmark on one GPU: pathwise slab sequences of a batch of
samples, the estimators at the space-time quadrature points and their error split (Section 5).

Host orchestration over the slab library (libsgheat.so); every vector-sized step runs in its kernels.
The samples are split into sample-batch handles (at most 512 / N_t samples each; by default each
sample is preconditioned with its own diagonal block, since the squared-Gaussian coefficient varies
strongly between samples); each handle marches its samples slab by slab with the pathwise forcing
    F_s^(n) = G_q(xi_s) ( T1^(n) (x) m + sum_mu Psi_mu(xi_s) T2^(n) (x) k_mu )
(sg_separable_vector over the loads of sg_load_vectors, on top of the transfer JJ U^(n-1)), and after
every slab the handles add their samples' values and squares at the quadrature points into one array
(sg_sample_qp_moments), from which sg_moment_errors integrates the errors of the sample mean and
unbiased sample variance against the exact mean phi and variance C2 phi^2 (total errors) and against the
exact sampled estimators g_bar phi and v_g phi^2 (discretisation errors); the pure sampling errors are
|g_bar - 1| ||phi|| and |v_g - C2| ||phi^2|| (eqs. mc-error-mean-L2,mc-error-var-L2, mc-disc-mean-error,
mc-pure-sampling-mean-error, mc-disc-var-error, mc-pure-sampling-var-error), with g_bar and v_g the
sample mean and unbiased sample variance of G_q(xi_s).
"""
from __future__ import annotations

import math

import numpy as np

from . import sgheat


class MCErrorStudy:
    """One sg_inputs.MCErrorWorkload."""

    def __init__(self, ew, precision=sgheat.SG_FP64, rtol: float = 1e-10, max_iter: int = 500, samples=None,
                 diag_blocks: int = 1):
        import torch
        import sg_inputs
        self.ew = ew
        w = ew.base
        self.rtol, self.max_iter = rtol, max_iter
        self.spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, 0, w.n_levels,
                                w.lo, w.hi, w.pre_smooth, w.post_smooth, w.vanka_omega, w.fgmres_restart,
                                diag_blocks=diag_blocks)
        mus, coef = sg_inputs.coef_qp_levels(w, lambda lvl: sgheat.quadrature_points(self.spec, lvl))
        xs = ew.samples() if samples is None else np.asarray(samples, dtype=np.float64)
        self.N = len(xs)
        if self.N < 2:
            raise ValueError("the unbiased variance needs at least two samples")
        bsz = min(ew.batch, sgheat_max_samples(w.n_time))
        self.handles = [sgheat.Problem(self.spec, mus, coef, precision, samples=xs[i:i + bsz])
                        for i in range(0, self.N, bsz)]
        self.nq1, self.ntq = w.fe_degree + 3, w.time_degree + 3
        dev = torch.device("cuda:0")
        P0 = self.handles[0]
        pts = sgheat.gauss_points(self.spec, 0, self.nq1)
        s, gs = sg_inputs.finite_chaos_phi(pts)
        mus_q, a = sg_inputs.finite_chaos_coefficient_modes(pts)
        nf = 1 + len(mus_q)
        fval = np.zeros((nf,) + s.shape)
        fval[0] = s
        fgrad = np.zeros((nf,) + gs.shape)
        for k in range(len(mus_q)):
            fgrad[1 + k] = a[k][..., None] * gs
        self.V = P0.load_vectors(self.nq1, torch.from_numpy(fval).to(dev), torch.from_numpy(fgrad).to(dev))
        self.s_qp = torch.from_numpy(np.ascontiguousarray(s)).to(dev)
        la, lc = sg_inputs.finite_chaos_exact_modes()
        self.C2 = float(np.sum(lc[np.any(la != 0, axis=1)] ** 2))
        self.psi_mu = [P.sample_psi(np.array(mus_q)) for P in self.handles]      # [n_s, n_mu] per handle
        self.G = [P.sample_psi(la) @ lc for P in self.handles]                   # G_q(xi_s) per handle
        g_all = np.concatenate(self.G)
        self.g_bar = float(np.mean(g_all))
        self.v_g = float(np.var(g_all, ddof=1))
        self.st, _ = P0.time_rule(self.ntq)
        self.acc = torch.zeros(P0.qp_moment_length(self.nq1, self.ntq), dtype=torch.float64, device=dev)
        self.info = []

    def close(self):
        for P in self.handles:
            P.close()
        self.handles = []

    def _weights(self, k, n):
        P = self.handles[k]
        t = (n - 1) * self.ew.base.tau + self.ew.base.tau * self.st
        T = P.time_load_weights(np.stack([4.0 * t ** 3, t ** 4]))                # [2, N_t]
        g, pm = self.G[k], self.psi_mu[k]
        W = np.empty((1 + pm.shape[1], len(g), T.shape[1]))
        W[0] = g[:, None] * T[0][None, :]
        W[1:] = (g[:, None] * pm).T[:, :, None] * T[1][None, None, :]
        return W

    def run(self, windows: bool = False, progress=None):
        """March every handle; returns the six errors (dict) of the estimators over all slabs, or with
        windows=True a list of them for every cumulative window of handles (samples 1..n_k, n_k the
        samples of the first k handles), the sampling diagnostic over growing N."""
        import torch
        H = len(self.handles)
        us = [torch.zeros(P.n(0), dtype=torch.float64, device="cuda") for P in self.handles]
        rhs = [torch.zeros_like(u) for u in us]
        n_win = H if windows else 1
        accs = [self.acc] + [torch.zeros_like(self.acc) for _ in range(n_win - 1)]
        counts = np.cumsum([len(g) for g in self.G])
        tg = []
        for j in range(n_win):
            g = np.concatenate(self.G[: j + 1]) if windows else np.concatenate(self.G)
            tg.append((float(np.mean(g)), float(np.var(g, ddof=1))))
        outs = [np.zeros(6) for _ in range(n_win)]
        self.info = []
        for n in range(1, self.ew.n_slabs + 1):
            for a in accs:
                a.zero_()
            for k, P in enumerate(self.handles):
                if n == 1:
                    P.separable_vector(self._weights(k, n), self.V, rhs[k], beta=0.0)
                else:
                    P.slab_transfer(us[k], rhs[k])
                    P.separable_vector(self._weights(k, n), self.V, rhs[k], beta=1.0)
                _, info = P.solve(rhs[k], us[k], rtol=self.rtol, max_iter=self.max_iter)
                self.info.append(info)
                if not info["converged"]:
                    raise sgheat.SgError(sgheat.SG_NOT_CONVERGED, f"slab {n} of batch {k} did not converge")
                # handle k's samples belong to every window that contains it
                for j in (range(k, n_win) if windows else [0]):
                    P.sample_qp_moments(us[k], self.nq1, self.ntq, accs[j])
            if progress is not None:
                progress(n)
            t = (n - 1) * self.ew.base.tau + self.ew.base.tau * self.st
            for j in range(n_win):
                n_tot = int(counts[j]) if windows else self.N
                outs[j] += self.handles[0].moment_errors(accs[j], n_tot, self.nq1, self.s_qp, t ** 4,
                                                         [1.0, tg[j][0]], [self.C2, tg[j][1]])
        self.last = us
        res = []
        for j in range(n_win):
            out, (g_bar, v_g) = outs[j], tg[j]
            res.append({"tot_mean": math.sqrt(out[0]), "disc_mean": math.sqrt(out[1]),
                        "mc_mean": abs(g_bar - 1.0) * math.sqrt(out[4]),
                        "tot_var": math.sqrt(out[2]), "disc_var": math.sqrt(out[3]),
                        "mc_var": abs(v_g - self.C2) * math.sqrt(out[5]),
                        "N": int(counts[j]) if windows else self.N})
        return res if windows else res[0]


def sgheat_max_samples(n_time: int) -> int:
    """Samples one handle holds: N_xi * N_t <= 512 components per cell."""
    return 512 // n_time
