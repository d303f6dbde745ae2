"""Pins of the FP64 adjoint oracle (slab sequence, mean/variance QoI, parameter gradient); no GPU.

Each check uses a route other than the adjoint itself: central finite differences of the forward
sweep, tensor Gauss-Hermite quadrature of Q(xi)^2, the textbook right-Radau transfer, and the
invariant that a deterministic coefficient carries no variance.
"""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

import sg_inputs
from oracle import adjoint as adj
from oracle import chaos, timebasis


@pytest.mark.parametrize("name", ["a2", "a3"])
def test_adjoint_gradient_matches_central_differences(name):
    aw = sg_inputs.ADJOINT_WORKLOADS[name]
    th, a0 = aw.theta0(), aw.a0_cells0()
    J, _, dth, da0 = adj.gradient(aw, th, a0)
    assert J == pytest.approx(adj.objective(aw, th, a0), rel=1e-13)
    h = 1e-6
    for m in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[m] += h
        tm[m] -= h
        fd = (adj.objective(aw, tp, a0) - adj.objective(aw, tm, a0)) / (2 * h)
        assert dth[m] == pytest.approx(fd, rel=1e-6)
    for c in [0, len(a0) // 2, len(a0) - 1]:
        ap, am = a0.copy(), a0.copy()
        ap[c] += h
        am[c] -= h
        fd = (adj.objective(aw, th, ap) - adj.objective(aw, th, am)) / (2 * h)
        assert da0[c] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_variance_of_q_matches_gauss_hermite_quadrature():
    """E[Q] and Var[Q] from the triple-product expansion against direct quadrature of Q(xi)."""
    aw = sg_inputs.ADJOINT_WORKLOADS["a2"]
    w = aw.base
    P = adj.build(aw, aw.theta0(), aw.a0_cells0())
    U = adj.forward(P, sg_inputs.initial_value(P.mesh.node_coords()), aw.n_slabs)
    EQ, VQ, _ = adj.qoi(P, U[-1], w.n_vars, w.chaos_degree)
    r = P.n_t - 1
    Ut = U[-1].reshape(P.n_xi, P.n_t, P.n_x)[:, r, :]
    m = Ut @ (P.Mx @ Ut.T)
    x1, w1 = He.hermegauss(12)
    w1 = w1 / math.sqrt(2 * math.pi)
    E1 = E2 = 0.0
    for idx in itertools.product(range(len(x1)), repeat=w.n_vars):
        xi = np.array([x1[i] for i in idx])
        wt = np.prod([w1[i] for i in idx])
        psi = np.array([float(chaos.psi_multi(a, xi[None, :])[0]) for a in P.index_set])
        Q = psi @ m @ psi
        E1 += wt * Q
        E2 += wt * Q * Q
    assert EQ == pytest.approx(E1, rel=1e-12)
    assert VQ == pytest.approx(E2 - E1 * E1, rel=1e-9, abs=1e-18)


def test_deterministic_coefficient_has_no_variance():
    aw = sg_inputs.ADJOINT_WORKLOADS["a2"]
    P = adj.build(aw, np.zeros(aw.base.n_vars), aw.a0_cells0())
    U = adj.forward(P, sg_inputs.initial_value(P.mesh.node_coords()), aw.n_slabs)
    for u in U:
        assert np.max(np.abs(u.reshape(P.n_xi, -1)[1:])) == 0.0
    EQ, VQ, _ = adj.qoi(P, U[-1], aw.base.n_vars, aw.base.chaos_degree)
    assert VQ == 0.0 and EQ > 0.0


def test_transfer_is_right_radau_trace_transport():
    """C_t = v(0) e_r^T (eq. Ct); dG(1) on nodes {1/3, 1}: v_0(0) = 3/2, v_1(0) = -1/2."""
    _, _, C = timebasis.time_matrices(1, 0.1)
    assert np.allclose(C, [[0.0, 1.5], [0.0, -0.5]], atol=1e-14)
    aw = sg_inputs.ADJOINT_WORKLOADS["a2"]
    P = adj.build(aw, aw.theta0(), aw.a0_cells0())
    x = np.random.default_rng(0).standard_normal(P.n)
    x[P.full_boundary_mask()] = 0.0
    y = (adj.transfer_matrix(P) @ x).reshape(P.n_xi, P.n_t, P.n_x)
    xr = x.reshape(P.n_xi, P.n_t, P.n_x)[:, P.n_t - 1, :]
    Mx = P.Mx.toarray()
    Mx[P.bmask, :] = 0.0
    for i, v0 in enumerate([1.5, -0.5]):
        assert np.allclose(y[:, i, :], v0 * (xr @ Mx.T), atol=1e-14)
