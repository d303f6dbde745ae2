"""Pins of the FP64 oracle for batches of independent SG problems and for the chaos moments; no GPU.

Routes: Gauss-Hermite quadrature of the chaos expansion (moments), the pathwise solution at the
correspondingly scaled sample (a member's scaled coefficient), and the invariant that the mean
coefficient of every member is the unscaled a_0.
"""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

import sg_inputs
from oracle import chaos
from oracle import members as mb
from oracle import montecarlo as mc
from oracle.slab import from_workload


def test_chaos_moments_match_gauss_hermite_quadrature():
    mw = sg_inputs.MEMBER_WORKLOADS["b2"]
    j = 2                                            # degree 3
    P = mb.member_problem(mw, j)
    u = mb.member_sequence(mw, j)[-1]
    mean, var = mb.chaos_moments(u, P.n_xi)
    U = u.reshape(P.n_xi, -1)
    x1, w1 = He.hermegauss(8)
    w1 = w1 / math.sqrt(2 * math.pi)
    E1 = np.zeros(U.shape[1])
    E2 = np.zeros(U.shape[1])
    for i, k in itertools.product(range(len(x1)), repeat=2):
        xi = np.array([[x1[i], x1[k]]])
        psi = np.array([chaos.psi_multi(a, xi)[0] for a in P.index_set])
        val = psi @ U
        E1 += w1[i] * w1[k] * val
        E2 += w1[i] * w1[k] * val * val
    assert np.allclose(mean, E1, rtol=0, atol=1e-14 * np.abs(E1).max())
    assert np.allclose(var, E2 - E1 * E1, rtol=0, atol=1e-12 * np.abs(var).max())


def test_unit_scales_reproduce_the_single_problem():
    mw = sg_inputs.MEMBER_WORKLOADS["b2"]
    P = mb.member_problem(mw, 1)
    Q = from_workload(mw.base.with_(chaos_degree=mw.degrees[1]))
    assert np.array_equal(P.coef_qp[P.mu0], Q.coef_qp[Q.mu0])      # the shared mean field
    for k in range(len(P.coef_mu)):
        if k != P.mu0:
            s = mw.scales(P.coef_mu)[1, k]
            assert np.allclose(P.coef_qp[k], s * Q.coef_qp[k], rtol=1e-15, atol=0)


def test_member_at_a_sample_matches_the_pathwise_solution_at_the_scaled_sample():
    """Member j with factors s_m, evaluated at xi, approximates the pathwise solution of the unscaled
    coefficient at (s_1 xi_1, s_2 xi_2) (affine coefficient); degree 3 chaos error ~1e-4."""
    mw = sg_inputs.MEMBER_WORKLOADS["b2"]
    j = 2
    P = mb.member_problem(mw, j)
    U = mb.member_sequence(mw, j)[-1].reshape(P.n_xi, -1)
    s = mw.scales(P.coef_mu)[j]
    s_m = np.array([s[k] for k, mu in enumerate(P.coef_mu) if sum(mu) == 1])
    sw = sg_inputs.SampleWorkload(mw.base, 1, mw.n_slabs)
    for xi in [np.array([0.8, -1.1]), np.array([-1.5, 0.3])]:
        psi = np.array([chaos.psi_multi(a, xi[None])[0] for a in P.index_set])
        ref = mc.pathwise_sequence(sw, s_m * xi)[-1]
        assert np.abs(psi @ U - ref).max() <= 2e-4 * np.abs(ref).max()


def test_degree_zero_member_has_no_variance():
    mw = sg_inputs.MEMBER_WORKLOADS["b2"]
    j = mw.degrees.index(0)
    _, var = mb.chaos_moments(mb.member_sequence(mw, j)[-1], 1)
    assert np.all(var == 0.0)


def test_packing_covers_every_member_once_within_capacity():
    from paper_2605_21046_amd.sgbatch import pack_members
    mw = sg_inputs.MEMBER_WORKLOADS["c4"]
    modes = [math.comb(mw.base.n_vars + p, p) for p in mw.degrees]
    bins = pack_members(modes, 256)
    assert sorted(j for b in bins for j in b) == list(range(len(modes)))
    assert all(sum(modes[j] for j in b) <= 256 for b in bins)
    assert len(bins) == math.ceil(sum(modes) / 256)
    with pytest.raises(ValueError):
        pack_members([300], 256)
