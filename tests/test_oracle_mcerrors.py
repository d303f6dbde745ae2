"""Pins of the FP64 oracle of the Monte-Carlo error split on the finite-chaos benchmark; no GPU.

Routes other than the oracle's own sums: closed forms of the pure sampling errors (they only need the
sample mean and variance of G_q and the exact norms of phi and phi^2), the triangle inequalities of
the split, the order of the discretisation error under h = tau refinement (Q3 / dG(3): about 4, the
rate the paper reports qualitatively), and root-N statistics of G_q (E[G_q] = 1, Var[G_q] = C2).
"""
import math

import numpy as np
import pytest

import sg_inputs
from oracle import mcerrors as me
from oracle import montecarlo as mc


def _C2():
    la, lc = sg_inputs.finite_chaos_exact_modes()
    return float(np.sum(lc[np.any(la != 0, axis=1)] ** 2))


def test_pure_sampling_errors_closed_form():
    """||(g_bar - 1) phi|| = |g_bar - 1| / 3 and ||(v_g - C2) phi^2|| = |v_g - C2| sqrt(1/17) 3/4 on (0,1) x D
    (the 6-point rule on 4^2 cells integrates s^2 to ~1e-10 and s^4 to ~1e-7 relative)."""
    ew = sg_inputs.MC_ERROR_WORKLOADS["e2"]
    e = me.error_split(ew)
    g = me.g_q_many(ew.samples())
    gbar = float(np.mean(g))
    vg = float(np.var(g, ddof=1))
    assert e["mc_mean"] == pytest.approx(abs(gbar - 1.0) / 3.0, rel=1e-8)
    assert e["mc_var"] == pytest.approx(abs(vg - _C2()) * math.sqrt(1.0 / 17.0) * 0.75, rel=1e-6)


@pytest.mark.parametrize("name", ["e2", "e3"])
def test_split_triangle_inequalities(name):
    e = me.error_split(sg_inputs.MC_ERROR_WORKLOADS[name])
    assert e["tot_mean"] <= e["disc_mean"] + e["mc_mean"] + 1e-15
    assert e["tot_var"] <= e["disc_var"] + e["mc_var"] + 1e-15
    assert e["disc_mean"] > 0 and e["disc_var"] > 0


def test_discretisation_error_order_four_under_h_equal_tau():
    xs = np.random.default_rng(3).standard_normal((4, 4))
    d = []
    for n in [1, 2, 4]:
        ew = sg_inputs.mc_error_workload(2 * n, 3, 3, 2 * n, 4, 4, 0, 1)
        d.append(me.error_split(ew, xs)["disc_mean"])
    rates = [math.log2(d[i] / d[i + 1]) for i in range(2)]
    assert min(rates) >= 3.7


def test_gq_moments_root_n():
    xs = np.random.Generator(np.random.PCG64(21)).standard_normal((4000, 4))
    g = me.g_q_many(xs)
    N = len(g)
    C2 = _C2()
    assert abs(np.mean(g) - 1.0) <= 4.0 * math.sqrt(C2 / N)
    assert abs(mc.sample_variance(g[:, None])[0] - C2) <= 0.25 * C2
