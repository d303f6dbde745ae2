"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics (no GPU needed).

Each test checks the oracle against something other than itself: values printed in the paper,
closed forms, textbook matrices, independent quadrature, invariants and brute force on tiny cases.
"""
import math
import os

import numpy as np
import pytest
import scipy.interpolate as si
import scipy.sparse.linalg as spla
from numpy.polynomial import hermite_e as He
from numpy.polynomial import legendre as Leg

import sg_inputs
from oracle import chaos, fem, timebasis
from oracle.krylov import fgmres
from oracle.multigrid import Hierarchy, Level, hierarchy_from_workload, prolongation
from oracle.slab import SlabProblem, from_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------------------------------------------
# Stochastic side (Section 2.6, eq. triple_stoch)
# ------------------------------------------------------------------------------------------------
def test_chaos_dimension_printed_values():
    for p, n in _read_golden("chaos_dims.txt"):
        assert len(chaos.total_degree_set(4, int(p))) == int(n)


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5])
def test_index_set_is_total_degree_graded(M):
    for p in range(7):
        s = chaos.total_degree_set(M, p)
        assert len(s) == math.comb(M + p, p)
        assert len(set(s)) == len(s)
        assert all(sum(a) <= p and min(a) >= 0 for a in s)
        degs = [sum(a) for a in s]
        assert degs == sorted(degs)
        for d in range(p + 1):
            blk = [a for a in s if sum(a) == d]
            assert blk == sorted(blk, reverse=True)
    if M == 2:
        assert chaos.total_degree_set(2, 2) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def test_triple_products_match_gauss_hermite_quadrature():
    # E[psi_a psi_b psi_c] by 40-point Gauss-Hermite (probabilists') quadrature, He via numpy.
    y, w = He.hermegauss(40)
    w = w / math.sqrt(2 * math.pi)

    def psi(n):
        c = np.zeros(n + 1)
        c[n] = 1.0
        return He.hermeval(y, c) / math.sqrt(math.factorial(n))

    worst = 0.0
    for a in range(9):
        for b in range(9):
            for c in range(9):
                q = float(np.sum(w * psi(a) * psi(b) * psi(c)))
                worst = max(worst, abs(q - chaos.hermite_triple_1d(a, b, c)))
    assert worst < 1e-10


def test_galerkin_tensors_structure():
    idx = chaos.total_degree_set(4, 3)
    G0 = chaos.galerkin_tensor((0, 0, 0, 0), idx)
    assert np.array_equal(G0, np.eye(35))
    off = 0
    for m in range(4):
        e = [0] * 4
        e[m] = 1
        G = chaos.galerkin_tensor(tuple(e), idx)
        assert np.array_equal(G, G.T)
        assert np.all(np.diag(G) == 0.0)
        off += int(np.count_nonzero(G))
        # eigenvalues of the multiplication-by-xi_m matrix lie inside the extreme root of He_{p+1}
        root = np.max(He.hermeroots([0] * 4 + [1]))
        assert np.max(np.abs(np.linalg.eigvalsh(G))) <= root + 1e-12
    assert off == 120
    # M = 1: G_{e_1} is the Jacobi matrix of the orthonormal Hermite family; its eigenvalues are
    # exactly the roots of He_{p+1}.
    for p in range(1, 8):
        G = chaos.galerkin_tensor((1,), chaos.total_degree_set(1, p))
        roots = np.sort(He.hermeroots([0] * (p + 1) + [1]))
        assert np.allclose(np.sort(np.linalg.eigvalsh(G)), roots, atol=1e-12)


def test_finite_chaos_table_row_p0_truncation_and_variance():
    """Row p_xi = 0 of Table tab:finite-errors-rates, the parts the discrete solve does not enter: the
    oracle's own error routine, run on a small mesh, gives (i) the variance error, which at p_xi = 0 is
    ||phi^2|| sum_{alpha != 0} c_alpha^2 (no nonzero mode is computed), and (ii) E_full^2 - E_mean^2, the
    truncation part ||phi||^2 sum_{alpha != 0, |alpha| <= q} c_alpha^2 (eq. finite-truncation-error-L2);
    both must equal the printed row (E_full^2 - E_mean^2 formed from the printed columns) to the printed
    digits."""
    import sg_inputs
    from oracle import finitechaos as fc
    g = {k: float(v) for k, v in _read_golden("finite_chaos_p0.txt")}
    e = fc.run(sg_inputs.finite_chaos_workload(4, 3, 3, 8, 0, 1))
    assert e["E_var_L2"] == pytest.approx(g["E_var_L2"], rel=5e-6)
    trunc = e["E_full_L2"] ** 2 - e["E_mean_L2"] ** 2
    assert trunc == pytest.approx(g["E_full_L2"] ** 2 - g["E_mean_L2"] ** 2, rel=2e-5)


@pytest.mark.xfail(strict=True, reason="the printed p_xi = 0 mean error (8.62293e-3) is not reproduced by the "
                   "definitions of Section 3.2 as written (the oracle gives 5.33e-2 at every resolution) nor by "
                   "any other reading tried; the readings and their values are listed in the design notes")
def test_finite_chaos_table_row_p0_mean_error():
    """The printed mean error of row p_xi = 0, computed by the oracle itself (the p_xi = 0 solution is
    the mean-coefficient problem with the projected forcing; truncation-dominated, so a small mesh
    suffices)."""
    import sg_inputs
    from oracle import finitechaos as fc
    g = {k: float(v) for k, v in _read_golden("finite_chaos_p0.txt")}
    e = fc.run(sg_inputs.finite_chaos_workload(4, 3, 3, 8, 0, 1))
    assert e["E_mean_L2"] == pytest.approx(g["E_mean_L2"], rel=0.05)


# ------------------------------------------------------------------------------------------------
# Time side (Section 2.5, eqs. At, Bt, Ct)
# ------------------------------------------------------------------------------------------------
def test_time_matrices_dg0_is_backward_euler():
    A, B, C = timebasis.time_matrices(0, 0.3)
    assert np.allclose(A, [[1.0]]) and np.allclose(B, [[0.3]]) and np.allclose(C, [[1.0]])


def test_time_matrices_dg1_exact_rationals():
    tau = 0.7
    A, B, C = timebasis.time_matrices(1, tau)
    assert np.allclose(timebasis.right_radau_nodes(1), [1 / 3, 1.0], atol=1e-15)
    assert np.allclose(A, [[9 / 8, 3 / 8], [-9 / 8, 5 / 8]], atol=1e-14)
    assert np.allclose(B, tau * np.diag([3 / 4, 1 / 4]), atol=1e-14)
    assert np.allclose(C, [[0.0, 3 / 2], [0.0, -1 / 2]], atol=1e-14)


@pytest.mark.parametrize("r", [0, 1, 2, 3, 4])
def test_time_matrix_invariants(r):
    A, B, C = timebasis.time_matrices(r, 1.0)
    nodes = timebasis.right_radau_nodes(r)
    v0 = np.array([float(timebasis.lagrange_value(nodes, i, np.array(0.0))) for i in range(r + 1)])
    er = np.zeros(r + 1)
    er[-1] = 1.0
    assert np.allclose(A @ np.ones(r + 1), v0, atol=1e-12)                    # A 1 = v(0)
    assert np.allclose(A + A.T, np.outer(v0, v0) + np.outer(er, er), atol=1e-12)  # by parts
    assert np.allclose(B, np.diag(np.diag(B)), atol=1e-13)                    # Radau exactness
    assert np.all(np.diag(B) > 0) and abs(np.trace(B) - 1.0) < 1e-13
    assert np.allclose(C, np.outer(v0, er), atol=1e-13)                       # rank-one transfer


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_dg_stability_function_is_subdiagonal_pade(r):
    """For u' = -lambda u one slab maps u(t_{n-1}) to R(z) u(t_{n-1}), z = lambda tau, and for dG(r)
    R is the (r, r+1) Pade approximant of exp(-z)."""
    A, B, C = timebasis.time_matrices(r, 1.0)
    taylor = [(-1.0) ** k / math.factorial(k) for k in range(2 * r + 2)]
    p, q = si.pade(taylor, r + 1, r)
    er = np.zeros(r + 1)
    er[-1] = 1.0
    for z in [0.01, 0.3, 1.0, 2.5, 10.0]:
        U = np.linalg.solve(A + z * B, C @ er)
        assert abs(U[-1] - p(z) / q(z)) < 1e-11 * max(1.0, abs(p(z) / q(z)))


# ------------------------------------------------------------------------------------------------
# Space side (Section 2.4)
# ------------------------------------------------------------------------------------------------
def test_gll_points_closed_form():
    assert np.allclose(fem.gll_points(1), [0, 1])
    assert np.allclose(fem.gll_points(2), [0, 0.5, 1])
    s5 = 1 / math.sqrt(5)
    assert np.allclose(fem.gll_points(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1])
    s37 = math.sqrt(3 / 7)
    assert np.allclose(fem.gll_points(4), [0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1])


def _textbook_1d(k, h):
    if k == 1:
        return h / 6 * np.array([[2, 1], [1, 2]]), 1 / h * np.array([[1, -1], [-1, 1]])
    if k == 2:
        return (h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]),
                1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]))
    raise ValueError


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_element_matrices_textbook_tensor_form(dim, k):
    n = 3
    m = fem.Mesh(dim, n, k)
    h = 1.0 / n
    M1, K1 = _textbook_1d(k, h)
    Me = m.element_matrices(None)[0]
    Ke = m.element_matrices(np.ones((m.n_cells, m.nq)))[0]
    if dim == 2:
        # local numbering x fastest: index = a_x + (k+1) a_y  ->  kron(y-factor, x-factor)
        M_ref = np.kron(M1, M1)
        K_ref = np.kron(M1, K1) + np.kron(K1, M1)
    else:
        M_ref = np.kron(M1, np.kron(M1, M1))
        K_ref = (np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1))
                 + np.kron(K1, np.kron(M1, M1)))
    assert np.allclose(Me, M_ref, atol=1e-14)
    assert np.allclose(Ke, K_ref, atol=1e-12)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (3, 2), (3, 3)])
def test_global_spatial_matrices_invariants(dim, k):
    m = fem.Mesh(dim, 2, k, -1.0, 1.0)
    M = m.mass()
    K = m.stiffness(1.0 + np.random.default_rng(3).random((m.n_cells, m.nq)))
    one = np.ones(m.n_nodes)
    assert abs(one @ (M @ one) - 2.0 ** dim) < 1e-12               # |D|
    assert np.max(np.abs(K @ one)) < 1e-12                         # constants in the kernel
    assert abs(M - M.T).max() < 1e-15 and abs(K - K.T).max() < 1e-13
    ev = np.linalg.eigvalsh(M.toarray())
    assert ev.min() > 0


def _lagrange_1d_independent(nodes, a):
    vals = np.zeros(len(nodes))
    vals[a] = 1.0
    return si.lagrange(nodes, vals)   # numpy poly1d


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 2), (2, 3)])
def test_stiffness_against_high_order_quadrature(dim, k):
    """A Q1 coefficient makes the (k+1)-point rule exact, so the oracle's assembled K must match an
    independent 8-point-per-direction quadrature of int a grad phi_l . grad phi_m."""
    m = fem.Mesh(dim, 2, k)
    coef = lambda x: 1.0 + 0.5 * x[..., 0] - 0.3 * x[..., 1] + (0.2 * x[..., 2] if dim == 3 else 0.0)
    K = m.stiffness(coef(m.qp_coords())).toarray()
    g, w = Leg.leggauss(8)
    g = 0.5 * (g + 1)
    w = 0.5 * w
    h = m.h
    nodes_ref = m.support
    polys = [_lagrange_1d_independent(nodes_ref, a) for a in range(k + 1)]
    dpolys = [p.deriv() for p in polys]
    Kref = np.zeros_like(K)
    loc = m.local_multi()
    import itertools
    for c in range(m.n_cells):
        cm = m.cell_multi(c)
        dofs = m.cell_dofs(c)
        for qi in itertools.product(range(8), repeat=dim):
            ref = np.array([g[qi[d]] for d in range(dim)])
            x = np.array([m.lo + h * (cm[d] + ref[d]) for d in range(dim)])
            wq = np.prod([w[qi[d]] for d in range(dim)]) * h ** dim
            grads = []
            for am in loc:
                gr = []
                for e in range(dim):
                    val = 1.0
                    for d in range(dim):
                        val *= (dpolys[am[d]](ref[d]) / h) if d == e else polys[am[d]](ref[d])
                    gr.append(val)
                grads.append(np.array(gr))
            a = coef(x)
            for i, gi in enumerate(grads):
                for j, gj in enumerate(grads):
                    Kref[dofs[i], dofs[j]] += wq * a * (gi @ gj)
    assert np.abs(K - Kref).max() < 1e-11 * np.abs(Kref).max()


def test_interpolation_reproduces_coarse_polynomials():
    for dim, k in [(2, 1), (2, 2), (2, 3), (3, 2)]:
        fine, coarse = fem.Mesh(dim, 4, k), fem.Mesh(dim, 2, k)
        I = fem.interpolation_matrix(fine, coarse)
        # a polynomial of degree k in each variable lies in every Q_k space
        f = lambda X: np.prod([(X[:, d] + 0.3) ** k - 0.7 * X[:, d] for d in range(dim)], axis=0)
        assert np.abs(I @ f(coarse.node_coords()) - f(fine.node_coords())).max() < 1e-12


# ------------------------------------------------------------------------------------------------
# The slab operator (Problem tensor-product-slab-system)
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["c1", "t2q1", "t2q3", "t3q1", "t3q2"])
def test_routes_agree(name):
    P = from_workload(sg_inputs.WORKLOADS[name])
    x = sg_inputs.uniform_vector(P.n, sg_inputs.SEED_APPLY_INPUT)
    y1, y2 = P.apply_route1(x), P.apply_route2(x)
    assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y1).max()


def test_pxi0_reduces_to_deterministic_slab():
    w = sg_inputs.WORKLOADS["t2q2"].with_(chaos_degree=0)
    P = from_workload(w)
    import scipy.sparse as sp
    A = sp.kron(sp.csr_matrix(P.At), P.Mx) + sp.kron(sp.csr_matrix(P.Bt), P.K[P.mu0])
    A = P._apply_dirichlet(A, P.n_t)
    x = sg_inputs.uniform_vector(P.n, 5)
    assert np.abs(A @ x - P.apply_route2(x)).max() < 1e-14 * np.abs(A @ x).max() + 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_manufactured_weak_form(dim):
    """u = X(x) T(t) sum_beta c_beta Psi_beta with X in Q_2 (zero on the boundary), T in P_1 and a
    coefficient affine in xi with Q1 modes in x: the oracle's AA U equals the weak form
    E[int_I <d_t u, v> + a(u, v) dt] + E[<u(t_{n-1}^+), v(t_{n-1}^+)>] computed independently
    (8-point Gauss in space and time, 10-point Gauss-Hermite in xi, equispaced Q2 Lagrange basis)."""
    n, k, tau, M, p = (3 if dim == 2 else 2), 2, 0.4, 2, 2
    def coef_fn(w, x):
        mus = [(0, 0), (1, 0), (0, 1)]
        a0 = 1.0 + 0.3 * x[..., 0] + 0.2 * x[..., 1]
        a1 = 0.1 * (1.0 + x[..., 0] * x[..., 1])
        a2 = 0.05 * (1.0 - x[..., 1])
        return mus, np.stack([a0, a1, a2])
    w = sg_inputs.Workload("mf", dim, n, k, 1, tau, M, p, 1, "sine")
    P = from_workload(w, 0, coef_fn)
    idx = P.index_set
    c = np.array([1.0, 0.4, -0.3, 0.2, 0.1, -0.25])
    X = lambda x: np.prod([x[..., d] * (1 - x[..., d]) for d in range(dim)], axis=0)
    def gradX(x):
        out = []
        for e in range(dim):
            v = np.ones(x.shape[:-1])
            for d in range(dim):
                v = v * ((1 - 2 * x[..., d]) if d == e else x[..., d] * (1 - x[..., d]))
            out.append(v)
        return np.stack(out, axis=-1)
    T = lambda s: 0.5 + 1.5 * s          # s = t / tau
    dT = 1.5 / tau
    s_nodes = np.array([1 / 3, 1.0])     # dG(1) right Radau nodes
    U = np.zeros(P.n)
    Xn = X(P.mesh.node_coords())
    for a in range(P.n_xi):
        for i in range(2):
            U[(a * 2 + i) * P.n_x:(a * 2 + i + 1) * P.n_x] = c[a] * T(s_nodes[i]) * Xn
    y = P.apply_route2(U)
    # --- independent weak form ---
    gt, wt = Leg.leggauss(8)
    st = 0.5 * (gt + 1)
    wt = 0.5 * wt
    v = [lambda s: 1.5 * (1 - s), lambda s: 1.5 * s - 0.5]
    int_dT_v = [sum(wt * dT * v[i](st)) * tau + T(0.0) * v[i](0.0) for i in range(2)]
    int_T_v = [sum(wt * T(st) * v[i](st)) * tau for i in range(2)]
    yh, wh = He.hermegauss(10)
    wh = wh / math.sqrt(2 * math.pi)
    def Psi(alpha, xi):
        out = np.ones(xi.shape[:-1])
        for m, am in enumerate(alpha):
            cc = np.zeros(am + 1)
            cc[am] = 1
            out = out * He.hermeval(xi[..., m], cc) / math.sqrt(math.factorial(am))
        return out
    XI = np.stack(np.meshgrid(yh, yh, indexing="ij"), -1).reshape(-1, 2)
    WXI = np.outer(wh, wh).reshape(-1)
    # E[a Psi_beta Psi_alpha] at x, for affine a: = sum over quadrature of a(x, xi) Psi Psi
    PsiTab = np.stack([Psi(al, XI) for al in idx])   # [n_xi, n_quad]
    gx, wx = Leg.leggauss(8)
    gx = 0.5 * (gx + 1)
    wx = 0.5 * wx
    h = P.mesh.h
    rng = np.random.default_rng(0)
    interior = np.flatnonzero(~P.bmask)
    rows = rng.choice(interior, size=min(6, len(interior)), replace=False)
    coords = P.mesh.node_coords()
    import itertools
    for mnode in rows:
        xm = coords[mnode]
        # global basis function phi_m: product of 1D hat-like quadratics on the equispaced nodes
        def phi_1d(d, t):
            # 1D global Q2 basis centred at xm[d] with spacing h/2
            pos = np.round(xm[d] / (h / 2)).astype(int)
            out = np.zeros_like(t)
            for cell in range(n):
                lo_ = cell * h
                local_nodes = lo_ + np.array([0, h / 2, h])
                if not np.any(np.isclose(local_nodes, xm[d])):
                    continue
                a = int(np.argmin(np.abs(local_nodes - xm[d])))
                pl = _lagrange_1d_independent(local_nodes, a)
                inside = (t >= lo_ - 1e-15) & (t <= lo_ + h + 1e-15)
                out = np.where(inside, pl(t), out)
            return out, pos
        acc_mass = 0.0
        acc_stiff = np.zeros((P.n_xi, P.n_xi))
        for cm in itertools.product(range(n), repeat=dim):
            for qi in itertools.product(range(8), repeat=dim):
                x = np.array([h * (cm[d] + gx[qi[d]]) for d in range(dim)])
                wq = np.prod([wx[qi[d]] for d in range(dim)]) * h ** dim
                # phi_m and its gradient at x, restricted to this cell
                vals, ders = [], []
                ok = True
                for d in range(dim):
                    lo_ = cm[d] * h
                    local_nodes = lo_ + np.array([0, h / 2, h])
                    hit = np.isclose(local_nodes, xm[d])
                    if not hit.any():
                        ok = False
                        break
                    pl = _lagrange_1d_independent(local_nodes, int(np.argmax(hit)))
                    vals.append(pl(x[d]))
                    ders.append(pl.deriv()(x[d]))
                if not ok:
                    continue
                phi = np.prod(vals)
                gphi = np.array([np.prod([ders[d] if d == e else vals[d] for d in range(dim)])
                                 for e in range(dim)])
                acc_mass += wq * X(x) * phi
                mus, avals = coef_fn(None, x[None, :])
                a_xi = avals[0, 0] + avals[1, 0] * XI[:, 0] + avals[2, 0] * XI[:, 1]
                E = (PsiTab * a_xi * WXI) @ PsiTab.T                  # E[a Psi_al Psi_be]
                acc_stiff += wq * (gradX(x) @ gphi) * E
        for a in range(P.n_xi):
            for i in range(2):
                ref = c[a] * int_dT_v[i] * acc_mass + int_T_v[i] * (acc_stiff[a] @ c)
                got = y[(a * 2 + i) * P.n_x + mnode]
                assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (a, i, mnode, got, ref)


# ------------------------------------------------------------------------------------------------
# Smoother, cycle and solve
# ------------------------------------------------------------------------------------------------
def test_vanka_single_cell_is_exact():
    for name in ["t2q3", "t3q3"]:
        w = sg_inputs.WORKLOADS[name].with_(n_cells_1d=1, n_levels=1)
        P = from_workload(w)
        lev = Level(P)
        b = sg_inputs.uniform_vector(lev.ndof, 7)
        x = lev.vanka(b, np.zeros_like(b), 1, 1.0)
        assert np.abs(lev.A0 @ x - b).max() < 1e-13 * np.abs(b).max()


def test_one_level_cycle_is_exact_and_two_grid_contracts():
    w = sg_inputs.WORKLOADS["t2q2"].with_(n_levels=1)
    H = hierarchy_from_workload(w)
    lev = H.levels[0]
    b = sg_inputs.uniform_vector(lev.ndof, 8)
    x = H.vcycle_mode(b)
    assert np.abs(lev.A0 @ x - b).max() < 1e-12 * np.abs(b).max()
    w2 = sg_inputs.WORKLOADS["t2q2"]
    H2 = hierarchy_from_workload(w2)
    lev = H2.levels[0]
    e = sg_inputs.uniform_vector(lev.ndof, 9)
    e[lev.bdof] = 0.0
    for _ in range(3):                     # error propagation of one cycle: e <- e - V(A e)
        e_new = e - H2.vcycle_mode(lev.A0 @ e)
        assert np.linalg.norm(e_new) < 0.5 * np.linalg.norm(e)
        e = e_new


def test_restriction_is_transpose_of_prolongation_and_masks_boundary():
    H = hierarchy_from_workload(sg_inputs.WORKLOADS["t2q2"])
    P = H.P[0]
    fine, coarse = H.levels[0], H.levels[1]
    assert np.all(P[fine.bdof].toarray() == 0) and np.all(P[:, coarse.bdof].toarray() == 0)


@pytest.mark.parametrize("name", ["c1", "t3q2"])
def test_fgmres_matches_direct_solve(name):
    w = sg_inputs.WORKLOADS[name]
    P = from_workload(w)
    H = hierarchy_from_workload(w)
    xs = sg_inputs.uniform_vector(P.n, sg_inputs.SEED_SOLVE_TARGET)
    xs[P.full_boundary_mask()] = 0.0
    b = P.apply_route2(xs)
    x, st = fgmres(P.apply_route2, lambda r: H.vcycle(r, P.n_xi), b, rtol=1e-8)
    assert st["converged"] == 1 and st["rel_residual_true"] <= 1e-8
    xd = spla.spsolve(P.assemble_full().tocsc(), b)
    assert np.linalg.norm(xd - xs) <= 1e-12 * np.linalg.norm(xs)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)


def test_diagonal_blocks_of_an_affine_coefficient_are_the_mean_block():
    """[G_{e_m}]_{alpha alpha} = 0, so every per-mode hierarchy equals the mean-block one."""
    from oracle import multigrid
    w = sg_inputs.WORKLOADS["t2q2"]
    H = multigrid.hierarchy_from_workload(w)
    B = multigrid.block_hierarchies_from_workload(w)
    P = from_workload(w)
    r = np.random.default_rng(4).standard_normal(P.n)
    assert np.allclose(B.vcycle(r, P.n_xi), H.vcycle(r, P.n_xi), rtol=0, atol=1e-13 * np.abs(r).max())


def test_diagonal_block_is_the_galerkin_projection_at_fixed_mode():
    """For the non-affine finite-chaos coefficient A_alpha differs from A_0 exactly by
    sum_mu [G_mu]_{alpha alpha} B_t (x) K_mu over mu != 0, with [G_{2 e_k}]_{alpha alpha} = sqrt(2) alpha_k
    (E[He_2/sqrt2 psi_a^2] = sqrt(2) a) and zero for mu = e_k + e_l."""
    import scipy.sparse as sp
    fw = sg_inputs.finite_chaos_workload(2, 2, 1, 2, 2, 1)
    P = from_workload(fw.base)
    for a, alpha in enumerate(P.index_set):
        D = (P.diagonal_block(a) - P.mean_block()).toarray()
        ref = np.zeros_like(D)
        for mu, K in zip(P.coef_mu, P.K):
            if max(mu) == 2 and sum(mu) == 2:
                k = int(np.argmax(mu))
                g = math.sqrt(2.0) * alpha[k]
                Bk = sp.kron(sp.csr_matrix(P.Bt), K).toarray()
                ref += g * Bk
        bm = np.tile(P.bmask, P.n_t)
        ref[bm, :] = 0.0
        ref[:, bm] = 0.0
        assert np.allclose(D, ref, rtol=0, atol=1e-12)
