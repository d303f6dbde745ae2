"""Pins of the FP64 Monte-Carlo oracle (pathwise slab sequences and sample estimators); no GPU.

Routes other than the pathwise solve itself: a worked example of the estimators, the closed form of
the 8x8-cell workload's coefficient at a sample, spectral convergence of the stochastic Galerkin
solution evaluated at a sample towards the pathwise solution at that sample, and the root-N
behaviour of the sample mean and variance around the Galerkin mean and variance.
"""
import math

import numpy as np
import pytest

import sg_inputs
from oracle import adjoint as adj
from oracle import chaos
from oracle import montecarlo as mc
from oracle.slab import from_workload


def test_estimators_worked_example():
    U = np.array([[1.0, -2.0], [2.0, -2.0], [3.0, -2.0], [4.0, -2.0]])
    assert np.allclose(mc.sample_mean(U), [2.5, -2.0], rtol=0, atol=1e-15)
    assert np.allclose(mc.sample_variance(U), [5.0 / 3.0, 0.0], rtol=1e-15, atol=0)
    assert np.allclose(mc.sample_variance(U, unbiased=False), [1.25, 0.0], rtol=1e-15, atol=0)


def test_sampled_coefficient_closed_form():
    """a(x, xi) = 1 + 0.1 xi_1 sin(pi x) sin(pi y) + 0.05 xi_2 sin(2 pi x) sin(pi y)."""
    w = sg_inputs.SAMPLE_WORKLOADS["m2"].base
    pts = np.random.default_rng(0).uniform(0.0, 1.0, size=(17, 2))
    xi = np.array([0.7, -1.3])
    x, y = pts[:, 0], pts[:, 1]
    ref = 1 + 0.1 * xi[0] * np.sin(math.pi * x) * np.sin(math.pi * y) + 0.05 * xi[1] * np.sin(2 * math.pi * x) * np.sin(math.pi * y)
    assert np.allclose(mc.sampled_coefficient(w, xi, pts), ref, rtol=1e-15, atol=1e-15)


def test_nonpositive_sample_is_rejected():
    w = sg_inputs.SAMPLE_WORKLOADS["m2"].base
    with pytest.raises(ValueError):
        mc.pathwise_problem(w, np.array([-40.0, 0.0]))


def _sg_final(sw, p):
    w = sw.base.with_(chaos_degree=p)
    P = from_workload(w)
    U = adj.forward(P, sg_inputs.initial_value(P.mesh.node_coords()), sw.n_slabs)[-1]
    return P, U.reshape(P.n_xi, -1)


def test_sg_solution_at_a_sample_converges_to_the_pathwise_solution():
    """sum_alpha u_alpha Psi_alpha(xi) -> u(xi) spectrally in p_xi (same space-time discretisation)."""
    sw = sg_inputs.SAMPLE_WORKLOADS["m2"]
    xs = sw.samples()[:3]
    refs = [mc.pathwise_sequence(sw, xi)[-1] for xi in xs]
    prev = None
    for p in [1, 2, 3, 4, 5]:
        P, U = _sg_final(sw, p)
        err = 0.0
        for xi, ref in zip(xs, refs):
            psi = np.array([chaos.psi_multi(a, xi[None])[0] for a in P.index_set])
            err = max(err, np.abs(psi @ U - ref).max() / np.abs(ref).max())
        if prev is not None:
            assert err < prev / 3.0
        prev = err
    assert prev < 5e-6


def test_sample_mean_and_variance_approach_the_galerkin_moments():
    """200 fresh draws: ||mean - E[u]||^2 within 4x its expectation sum(Var)/N; variance within 30%."""
    sw = sg_inputs.SAMPLE_WORKLOADS["m2"]
    N = 200
    xs = np.random.Generator(np.random.PCG64(11)).standard_normal((N, sw.base.n_vars))
    F = mc.batch_final_slabs(sw, xs)
    _, U = _sg_final(sw, 4)
    E, V = U[0], np.sum(U[1:] ** 2, axis=0)
    m, v = mc.sample_mean(F), mc.sample_variance(F)
    assert np.sum((m - E) ** 2) <= 4.0 * np.sum(V) / N
    assert np.linalg.norm(v - V) <= 0.3 * np.linalg.norm(V)
