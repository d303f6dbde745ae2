"""Pins of the oracle's row-by-row route (oracle/rows.py), which checks the full-size operator
applies at sampled rows: on small meshes it must reproduce every row of the slab operator as the
explicit Kronecker assembly (route 1) and the Kronecker identity (route 2) compute it
(Problem tensor-product-slab-system, eq. local_rhs_tensor), Dirichlet rows included.

The cases cover 2D and 3D, Q1..Q4, dG(0)..dG(3), an affine coefficient (the sine modes and the 8x8
workload's field) and the non-affine coefficient of the finite-chaos benchmark (Section 3.2, eq.
diffusion_benchmark: 11 active Hermite modes, some of total degree 2)."""
import numpy as np
import pytest

import sg_inputs
from oracle.rows import RowOracle
from oracle.slab import from_workload

W = sg_inputs.Workload
CASES = [
    W("r2q1", 2, 3, 1, 0, 0.05, 2, 2, 1, "sine"),
    W("r2q2", 2, 3, 2, 1, 0.01, 2, 2, 1, "c1"),
    W("r2q3", 2, 2, 3, 2, 0.02, 3, 1, 1, "sine"),
    W("r2q4", 2, 2, 4, 3, 0.02, 2, 1, 1, "sine"),
    W("r3q1", 3, 3, 1, 1, 0.05, 2, 1, 1, "sine"),
    W("r3q2", 3, 2, 2, 1, 0.05, 4, 1, 1, "sine"),
    W("r3q3", 3, 2, 3, 2, 0.05, 1, 2, 1, "sine"),
    W("r2fin", 2, 3, 2, 1, 1.0 / 64, 4, 2, 1, "finite", lo=-1.0, hi=1.0),
]


def _row_oracle(w):
    mus, _ = sg_inputs.coefficient_modes(w, np.zeros((1, w.dim)))
    return RowOracle(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree, mus,
                     lambda p: sg_inputs.coefficient_modes(w, p)[1], w.lo, w.hi)


@pytest.mark.parametrize("w", CASES, ids=[c.name for c in CASES])
def test_rows_match_both_operator_routes_on_every_row(w):
    P = from_workload(w)
    R = _row_oracle(w)
    x = sg_inputs.uniform_vector(P.n, 7)
    picks = [(a, i, m) for a in range(P.n_xi) for i in range(P.n_t) for m in range(P.n_x)]
    rows = R.rows(x, picks)
    y2 = P.apply_route2(x)
    y1 = P.apply_route1(x)
    scale = np.abs(y1).max()
    assert np.abs(y1 - y2).max() <= 1e-13 * scale
    assert np.abs(rows - y1).max() <= 1e-13 * scale


def test_rows_see_a_planted_change_of_one_coefficient_mode():
    """A perturbation of one non-mean coefficient mode in one cell changes exactly the rows of the
    nodes of that cell, and the row oracle follows route 2 there."""
    w = CASES[5]
    x = sg_inputs.uniform_vector(from_workload(w).n, 8)
    bump = (0.25, 0.5, 0.75)

    def fn(w_, p):
        mus, vals = sg_inputs.coefficient_modes(w_, p)
        inside = np.all((p > 0.5) & (p < 1.0), axis=-1)
        vals = vals.copy()
        vals[2] = vals[2] + 0.3 * inside * (bump[0] + p[..., 0])
        return mus, vals

    P = from_workload(w, coef_fn=fn)
    mus, _ = sg_inputs.coefficient_modes(w, np.zeros((1, w.dim)))
    R = RowOracle(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree, mus,
                  lambda p: fn(w, p)[1])
    picks = [(a, i, m) for a in range(P.n_xi) for i in range(P.n_t) for m in range(P.n_x)]
    y = P.apply_route2(x)
    assert np.abs(R.rows(x, picks) - y).max() <= 1e-13 * np.abs(y).max()
    y0 = from_workload(w).apply_route2(x)
    changed = np.abs(y - y0) > 1e-14 * np.abs(y0).max()
    assert 0 < changed.sum() < changed.size
