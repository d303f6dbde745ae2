"""Batches of independent stochastic Galerkin problems of mixed chaos degree on one GPU.

Host orchestration over the slab library (libsgheat.so); every numerical step runs in its kernels.
Members share the mesh, the time discretisation and the mean coefficient a_0 and differ in their
total degree p_j and in the factors on the fluctuation modes.  Members are packed into as few
member-batch handles as the library's per-cell component limit (N_xi * N_t <= 512) allows; inside a
handle every G_mu is block diagonal over its members, so one apply, Vanka sweep or V-cycle advances
all of them, and the coefficient fields are read once per cell for the whole handle.

Per handle and slab n: b = (I (x) C_t (x) M_x) U^(n-1) (u_0 in every member's mean mode for n = 1),
U^(n) = AA^{-1} b (one FGMRES over the handle, mean-block V-cycle preconditioner); at the end the
chaos mean and variance of every member (eqs. qoi-mean-chaos, qoi-variance-chaos).
"""
from __future__ import annotations

import math

import numpy as np

from . import sgheat

MAX_COMPONENTS = 512    # N_xi * N_t of one handle


def pack_members(modes, capacity):
    """Greedy first-fit packing of members (mode counts) into bins of at most `capacity` modes,
    largest first; returns lists of member indices, each in ascending order."""
    bins, loads = [], []
    for j in sorted(range(len(modes)), key=lambda j: (-modes[j], j)):
        if modes[j] > capacity:
            raise ValueError(f"member {j} has {modes[j]} modes, more than one handle holds ({capacity})")
        for b in range(len(bins)):
            if loads[b] + modes[j] <= capacity:
                bins[b].append(j)
                loads[b] += modes[j]
                break
        else:
            bins.append([j])
            loads.append(modes[j])
    return [sorted(b) for b in bins]


class MemberBatch:
    """The slab sequences of one sg_inputs.MemberWorkload."""

    def __init__(self, mw, rtol: float = 1e-10, max_iter: int = 500, precision=sgheat.SG_FP64):
        import torch
        import sg_inputs
        self.mw = mw
        self.w = w = mw.base
        self.rtol, self.max_iter = rtol, max_iter
        self.spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, 0, w.n_levels,
                                w.lo, w.hi, w.pre_smooth, w.post_smooth, w.vanka_omega, w.fgmres_restart)
        mus, coef = sg_inputs.coef_qp_levels(w, lambda lvl: sgheat.quadrature_points(self.spec, lvl))
        scales = mw.scales(mus)
        self.modes = [math.comb(w.n_vars + p, p) for p in mw.degrees]
        self.groups = pack_members(self.modes, MAX_COMPONENTS // w.n_time)
        self.handles = [sgheat.Problem(self.spec, mus, coef, precision,
                                       members=([mw.degrees[j] for j in g], scales[g])) for g in self.groups]
        self.n_t = w.n_time
        self.n_x = self.handles[0].shape[2]
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
        for P in self.handles:
            P.close()
        self.handles = []

    def _first_rhs(self, P, g):
        import torch
        x0 = torch.zeros(P.n(0), dtype=torch.float64, device=self.dev)
        v = x0.view(P.shape[0], self.n_t, self.n_x)
        off = 0
        for j in g:
            v[off, self.n_t - 1, :] = self.u0
            off += self.modes[j]
        return P.slab_transfer(x0)

    def run(self, n_slabs: int | None = None, keep_previous: bool = False):
        """March every handle n_slabs slabs; returns the last slab vector of each handle (and keeps the
        one before it in self.previous when keep_previous is set)."""
        import torch
        n_slabs = self.mw.n_slabs if n_slabs is None else n_slabs
        self.info = []
        self.previous = []
        out = []
        for P, g in zip(self.handles, self.groups):
            b = self._first_rhs(P, g)
            u = torch.zeros_like(b)
            for n in range(n_slabs):
                if keep_previous and n == n_slabs - 1:
                    self.previous.append(u.clone())
                u.zero_()
                _, info = P.solve(b, u, rtol=self.rtol, max_iter=self.max_iter)
                self.info.append(info)
                if not info["converged"]:
                    raise sgheat.SgError(sgheat.SG_NOT_CONVERGED, "a slab solve of the member batch did not converge")
                b = P.slab_transfer(u, b)
            out.append(u)
        return out

    def moments(self, us):
        """Chaos mean and variance of every member (workload order), each [n_members, N_t, N_x]."""
        import torch
        J = len(self.modes)
        mean = torch.empty(J, self.n_t, self.n_x, dtype=torch.float64, device=self.dev)
        var = torch.empty_like(mean)
        for P, g, u in zip(self.handles, self.groups, us):
            m, v = P.chaos_moments(u, var=torch.empty(len(g) * self.n_t * self.n_x, dtype=torch.float64,
                                                      device=self.dev))
            mean[g] = m.view(len(g), self.n_t, self.n_x)
            var[g] = v.view(len(g), self.n_t, self.n_x)
        return mean, var

    def member_vector(self, us, j):
        """Slab vector of member j alone, [modes_j * N_t * N_x], from the handles' vectors."""
        for P, g, u in zip(self.handles, self.groups, us):
            if j in g:
                off = sum(self.modes[i] for i in g if i < j)
                return u.view(P.shape[0], -1)[off:off + self.modes[j]].reshape(-1)
        raise IndexError(j)
