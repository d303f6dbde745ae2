"""Pins of the FP64 oracle of the finite-chaos benchmark (forcing, time marching, error norms); no GPU.

Routes other than the oracle's own formulas: the tensor Gauss-Hermite projection of the random
forcing factor (the cross-check the paper itself reports for its analytic projection), closed-form
time integrals of the Lagrange basis, the printed p_xi = 0 variance errors (which depend only on the
exact solution and the norm), the even/odd decoupling of the mean from odd modes, and independence of
the truncation-dominated errors from the space-time resolution.
"""
import itertools
import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He
from numpy.polynomial import polynomial as Pl

import sg_inputs
from oracle import chaos, timebasis
from oracle import finitechaos as fc
from oracle.slab import from_workload

HERE = os.path.dirname(__file__)


def _table():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "finite_chaos_table.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = line.split()
        rows[int(v[0])] = dict(zip(["N_xi", "E_full_L2", "E_full_H1", "E_mean_L2", "E_mean_H1", "E_var_L2", "E_var_H1"],
                                   [int(v[1])] + [float(x) for x in v[2:]]))
    return rows


def test_forcing_weights_match_gauss_hermite_projection():
    """sum_mu d[mu, beta] a_mu(x) = E[a(x, xi) G_q(xi) Psi_beta(xi)] by 8-point tensor quadrature."""
    fw = sg_inputs.finite_chaos_workload(2, 3, 3, 2, 2, 1)
    P = from_workload(fw.base)
    d = fc.forcing_chaos_weights(P, fw)
    x = np.array([[0.3, -0.7], [-0.9, 0.55], [0.0, 1.0]])
    mus, a = sg_inputs.finite_chaos_coefficient_modes(x)
    lhs = d.T @ a                                                  # [beta, point]
    z, wz = He.hermegauss(8)
    wz = wz / math.sqrt(2 * math.pi)
    Lq = chaos.total_degree_set(4, sg_inputs.FINITE_Q)
    rhs = np.zeros_like(lhs)
    for idx in itertools.product(range(8), repeat=4):
        xi = np.array([z[i] for i in idx])
        wt = float(np.prod([wz[i] for i in idx]))
        G = sum(fw.c_alpha(al) * chaos.psi_multi(al, xi[None])[0] for al in Lq)
        af = sg_inputs.finite_chaos_coefficient_at(x, xi)
        psi = np.array([chaos.psi_multi(b, xi[None])[0] for b in P.index_set])
        rhs += wt * G * psi[:, None] * af[None, :]
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_time_loads_closed_form():
    """int_{I_n} 4 t^3 v_i and int_{I_n} t^4 v_i by exact polynomial integration (slab 3 of tau = 0.25)."""
    fw = sg_inputs.finite_chaos_workload(2, 3, 3, 4, 0, 1)
    P = from_workload(fw.base)
    tau, n = 0.25, 3
    T1, T2 = fc.time_loads(P, n, tau)
    nodes = timebasis.right_radau_nodes(3)
    for i in range(4):
        li = Pl.polyfromroots([nodes[j] for j in range(4) if j != i])
        li = li / Pl.polyval(nodes[i], li)
        ts = np.array([(n - 1) * tau, tau])                            # t(s) = t_{n-1} + tau s
        p3 = Pl.polypow(ts, 3)
        p4 = Pl.polypow(ts, 4)
        i1 = Pl.polyint(Pl.polymul(4 * p3, li))
        i2 = Pl.polyint(Pl.polymul(p4, li))
        assert T1[i] == pytest.approx(tau * (Pl.polyval(1.0, i1) - Pl.polyval(0.0, i1)), rel=1e-13, abs=1e-15)
        assert T2[i] == pytest.approx(tau * (Pl.polyval(1.0, i2) - Pl.polyval(0.0, i2)), rel=1e-13, abs=1e-15)


def test_p0_variance_errors_equal_the_printed_values():
    """At p_xi = 0 the discrete variance is 0, so E_var is the norm of the exact variance C2 phi^2."""
    g = _table()[0]
    e = fc.run(sg_inputs.finite_chaos_workload(4, 3, 3, 8, 0, 1))
    assert f"{e['E_var_L2']:.5e}" == f"{g['E_var_L2']:.5e}"
    assert f"{e['E_var_H1']:.5e}" == f"{g['E_var_H1']:.5e}"


def test_mean_error_is_unchanged_by_odd_modes():
    """The coefficient is even in xi, so odd modes decouple from the mean's chain: E_mean(1) = E_mean(0),
    E_mean(3) = E_mean(2) (the pattern the paper reports)."""
    e0 = fc.run(sg_inputs.finite_chaos_workload(4, 3, 3, 8, 0, 1))
    e1 = fc.run(sg_inputs.finite_chaos_workload(4, 3, 3, 8, 1, 1))
    assert e1["E_mean_L2"] == pytest.approx(e0["E_mean_L2"], rel=1e-10)
    assert e1["E_mean_H1"] == pytest.approx(e0["E_mean_H1"], rel=1e-10)
    e2 = fc.run(sg_inputs.finite_chaos_workload(2, 3, 3, 4, 2, 1))
    e3 = fc.run(sg_inputs.finite_chaos_workload(2, 3, 3, 4, 3, 1))
    assert e3["E_mean_L2"] == pytest.approx(e2["E_mean_L2"], rel=1e-10)
    assert e3["E_full_L2"] < e2["E_full_L2"]


def test_truncation_dominated_errors_do_not_depend_on_the_resolution():
    a = fc.run(sg_inputs.finite_chaos_workload(4, 3, 3, 8, 1, 1))
    b = fc.run(sg_inputs.finite_chaos_workload(8, 3, 3, 16, 1, 1))
    for key in ["E_full_L2", "E_mean_L2", "E_var_L2", "E_full_H1"]:
        assert a[key] == pytest.approx(b[key], rel=1e-4)
