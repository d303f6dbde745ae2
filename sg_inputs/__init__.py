"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests/benchmark.

This module holds problem sizes, coefficient fields and random vectors only.  It contains none of
the discretisation arithmetic (no quadrature rules, no basis functions, no matrices): callers pass
in the physical coordinates at which a coefficient field is wanted.

Coefficient model (Section 2.7, coefficient expansion): a(x, xi) = sum_mu a_mu(x) Psi_mu(xi).
Every workload here is affine in xi, so the active set is {0, e_1, ..., e_M} and Psi_{e_m} = xi_m.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field, asdict

import numpy as np

# Seeds (fixed so every run sees the same data).
SEED_APPLY_INPUT = 0
SEED_SOLVE_TARGET = 1
SEED_MC_DRAWS = 2


@dataclass(frozen=True)
class Workload:
    """Sizes of one slab problem; the names follow the paper's notation."""
    name: str
    dim: int              # d
    n_cells_1d: int       # finest uniform Cartesian mesh: n_cells_1d^d cells of (lo, hi)^d
    fe_degree: int        # k of Q_k
    time_degree: int      # r of dG(r)
    tau: float            # slab length
    n_vars: int           # M
    chaos_degree: int     # p_xi (total degree)
    n_levels: int         # geometric multigrid levels (level 0 finest)
    field: str            # coefficient field, see coefficient_modes()
    lo: float = 0.0
    hi: float = 1.0
    pre_smooth: int = 1
    post_smooth: int = 1
    vanka_omega: float = 1.0
    fgmres_restart: int = 30

    @property
    def n_chaos(self) -> int:
        return math.comb(self.n_vars + self.chaos_degree, self.chaos_degree)

    @property
    def n_time(self) -> int:
        return self.time_degree + 1

    def n_nodes_1d(self, level: int = 0) -> int:
        return (self.n_cells_1d >> level) * self.fe_degree + 1

    def n_nodes(self, level: int = 0) -> int:
        return self.n_nodes_1d(level) ** self.dim

    def n_dofs(self, level: int = 0) -> int:
        return self.n_chaos * self.n_time * self.n_nodes(level)

    def with_(self, **kw) -> "Workload":
        d = asdict(self)
        d.update(kw)
        return Workload(**d)


WORKLOADS = {
    # 2D unit square, Q2 on 8x8 cells, dG(1), dt = 0.01, M = 2, p_xi = 2 (6 modes): 3468 DoFs.
    "c1": Workload("c1", 2, 8, 2, 1, 0.01, 2, 2, 3, "c1"),
    # 3D unit cube, Q2 on 32^3 cells, dG(1), M = 4, p_xi = 3 (35 modes): 19,223,750 DoFs, 4 levels.
    "c2": Workload("c2", 3, 32, 2, 1, 1.0 / 32, 4, 3, 4, "sine"),
    # 3D unit cube, Q3 on 24^3 cells, dG(2), M = 3, p_xi = 4 (35 modes): 40,846,785 DoFs, 4 levels.
    "c3": Workload("c3", 3, 24, 3, 2, 1.0 / 24, 3, 4, 4, "sine"),
    # Small cases used by the tests (several cells per direction, ragged sizes, every degree).
    "t2q1": Workload("t2q1", 2, 6, 1, 0, 0.05, 2, 2, 2, "sine"),
    "t2q2": Workload("t2q2", 2, 6, 2, 1, 0.02, 2, 2, 2, "sine"),
    "t2q3": Workload("t2q3", 2, 4, 3, 2, 0.02, 3, 2, 2, "sine"),
    "t3q1": Workload("t3q1", 3, 4, 1, 1, 0.05, 2, 1, 2, "sine"),
    "t3q2": Workload("t3q2", 3, 4, 2, 1, 0.05, 3, 2, 2, "sine"),
    "t3q3": Workload("t3q3", 3, 2, 3, 2, 0.05, 2, 2, 1, "sine"),
    "t3q4": Workload("t3q4", 3, 2, 4, 1, 0.05, 2, 1, 1, "sine"),
    "t2q4": Workload("t2q4", 2, 4, 4, 1, 0.02, 2, 2, 2, "sine"),
    # many chaos modes (70) on a small mesh: strips of modes in the Vanka kernel
    "t2q2p4": Workload("t2q2p4", 2, 4, 2, 1, 0.02, 4, 4, 2, "sine"),
    # the discretisations of the two 3D benchmark workloads (same k, r, M, p_xi, field and tau = h) on
    # small meshes whose cell counts per direction are not multiples of the apply's tile widths
    "t3c2": Workload("t3c2", 3, 10, 2, 1, 1.0 / 10, 4, 3, 2, "sine"),
    "t3c3": Workload("t3c3", 3, 5, 3, 2, 1.0 / 5, 3, 4, 1, "sine"),
    # the c3 discretisation on two levels (4 and 2 cells per direction): Vanka sweeps of Q3 dG(2) patches
    "t3v3": Workload("t3v3", 3, 4, 3, 2, 1.0 / 4, 3, 4, 2, "sine"),
    # two-level 3D Q3 and Q4 hierarchies with few modes: the Q3/Q4 restriction and prolongation passes
    "t3m3": Workload("t3m3", 3, 4, 3, 1, 0.05, 1, 1, 2, "sine"),
    "t3m4": Workload("t3m4", 3, 4, 4, 0, 0.05, 1, 1, 2, "sine"),
    # 64 cells per row: one row of cells per wave in the register-form Vanka corrections
    "t2w64": Workload("t2w64", 2, 64, 2, 1, 0.01, 2, 2, 2, "sine"),
    # three-level hierarchies whose lower two levels form one persistent coarse segment
    "t2s3": Workload("t2s3", 2, 8, 3, 2, 0.02, 3, 2, 3, "sine"),
    "t3s2": Workload("t3s2", 3, 4, 2, 1, 0.05, 2, 2, 3, "sine"),
    "t2v2": Workload("t2v2", 2, 8, 2, 1, 0.02, 2, 2, 3, "vmean"),
}


def _sine_shape(m: int, x: np.ndarray) -> np.ndarray:
    """phi_1 = prod_k sin(pi x_k); phi_m (m >= 2) doubles the frequency in direction (m - 2) mod d."""
    d = x.shape[-1]
    out = np.ones(x.shape[:-1])
    for k in range(d):
        freq = 2.0 if (m >= 2 and (m - 2) % d == k) else 1.0
        out = out * np.sin(freq * math.pi * x[..., k])
    return out


def coefficient_modes(w: Workload, x: np.ndarray):
    """Affine coefficient of workload ``w`` at physical points ``x`` (shape [..., d]).

    Returns ``(mu_list, values)`` with ``values[k]`` = a_{mu_k}(x).  The first mode is mu = 0.
    * "c1":   a = 1 + 0.1 xi_1 sin(pi x) sin(pi y) + 0.05 xi_2 sin(2 pi x) sin(pi y)
    * "sine": a = 1 + sum_m (0.1 / m^2) xi_m phi_m(x)
    * "vmean": a = 1 + 0.5 x y + sum_m (0.1 / m^2) xi_m phi_m(x) (a mean that varies between cells)
    * "finite": the non-affine coefficient of the finite-chaos benchmark (M = 4, d = 2), see
      finite_chaos_coefficient_modes.
    """
    x = np.asarray(x, dtype=np.float64)
    M = w.n_vars
    if w.field == "finite":
        return finite_chaos_coefficient_modes(x)
    mus = [tuple([0] * M)]
    vals = [np.ones(x.shape[:-1]) + (0.5 * x[..., 0] * x[..., 1] if w.field == "vmean" else 0.0)]
    for m in range(1, M + 1):
        e = [0] * M
        e[m - 1] = 1
        mus.append(tuple(e))
        if w.field == "c1":
            if m == 1:
                v = 0.1 * np.sin(math.pi * x[..., 0]) * np.sin(math.pi * x[..., 1])
            elif m == 2:
                v = 0.05 * np.sin(2 * math.pi * x[..., 0]) * np.sin(math.pi * x[..., 1])
            else:
                v = np.zeros(x.shape[:-1])
        elif w.field in ("sine", "vmean"):
            v = (0.1 / m ** 2) * _sine_shape(m, x)
        else:
            raise ValueError(f"unknown field {w.field}")
        vals.append(v)
    return mus, np.stack(vals)


# Finite-chaos benchmark (Section 3.2, eqs. diffusion_benchmark and finite-exact-solution-M4-q6):
# D = (-1, 1)^2, T = 1, M = 4, a = d_min + (xi_1 x_1^2 + xi_2 x_1 x_2 + xi_3 x_2^2 + xi_4)^2,
# u = phi(x, t) G_q(xi), phi = t^4 sin(pi (x_1 + 1) / 2) sin(pi (x_2 + 1) / 2),
# G_q = sum_{|alpha| <= q} c_alpha Psi_alpha, c_0 = 1, c_alpha = eta^|alpha|.
FINITE_D_MIN = 0.2
FINITE_ETA = 0.35
FINITE_Q = 6


def _finite_shapes(x: np.ndarray) -> list:
    """g_1..g_4 = x_1^2, x_1 x_2, x_2^2, 1: a = d_min + (sum_k xi_k g_k)^2."""
    x1, x2 = x[..., 0], x[..., 1]
    return [x1 * x1, x1 * x2, x2 * x2, np.ones_like(x1)]


def finite_chaos_coefficient_modes(x: np.ndarray):
    """Hermite modes of a = d_min + (sum_k xi_k g_k)^2 at points x [..., 2]: 11 modes.

    With xi_k^2 = sqrt(2) Psi_{2 e_k} + 1 and xi_k xi_l = Psi_{e_k + e_l} (k != l):
        a_0 = d_min + sum_k g_k^2,  a_{2 e_k} = sqrt(2) g_k^2,  a_{e_k + e_l} = 2 g_k g_l.
    """
    g = _finite_shapes(np.asarray(x, dtype=np.float64))
    mus = [(0, 0, 0, 0)]
    vals = [FINITE_D_MIN + sum(gk * gk for gk in g)]
    for k in range(4):
        mu = [0] * 4
        mu[k] = 2
        mus.append(tuple(mu))
        vals.append(math.sqrt(2.0) * g[k] * g[k])
    for k in range(4):
        for l in range(k + 1, 4):
            mu = [0] * 4
            mu[k] = mu[l] = 1
            mus.append(tuple(mu))
            vals.append(2.0 * g[k] * g[l])
    return mus, np.stack(vals)


def finite_chaos_coefficient_at(x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """a(x, xi) = d_min + (sum_k xi_k g_k(x))^2 at points x [..., 2] for one sample xi [4]."""
    g = _finite_shapes(np.asarray(x, dtype=np.float64))
    s = sum(float(xi[k]) * g[k] for k in range(4))
    return FINITE_D_MIN + s * s


def finite_chaos_phi(x: np.ndarray) -> tuple:
    """Spatial factor sin(pi (x_1 + 1) / 2) sin(pi (x_2 + 1) / 2) and its gradient [..., 2]."""
    x = np.asarray(x, dtype=np.float64)
    h = 0.5 * math.pi
    s1, s2 = np.sin(h * (x[..., 0] + 1)), np.sin(h * (x[..., 1] + 1))
    c1, c2 = np.cos(h * (x[..., 0] + 1)), np.cos(h * (x[..., 1] + 1))
    return s1 * s2, np.stack([h * c1 * s2, h * s1 * c2], axis=-1)


def finite_chaos_exact_modes():
    """Multi-indices of Lambda_q (M = 4, q = 6) and the exact solution's coefficients c_alpha."""
    alphas = [a for a in itertools.product(range(FINITE_Q + 1), repeat=4) if sum(a) <= FINITE_Q]
    c = [1.0 if sum(a) == 0 else FINITE_ETA ** sum(a) for a in alphas]
    return np.array(alphas, dtype=np.int32), np.array(c)


@dataclass(frozen=True)
class FiniteChaosWorkload:
    """The finite-chaos benchmark discretised with ``base`` (dim 2, domain (-1, 1)^2, field "finite",
    tau = T / n_slabs) at stochastic degree ``base.chaos_degree``."""
    base: Workload
    n_slabs: int

    def c_alpha(self, alpha) -> float:
        n = sum(alpha)
        return 0.0 if n > FINITE_Q else (1.0 if n == 0 else FINITE_ETA ** n)


def finite_chaos_workload(n_cells_1d: int, fe_degree: int, time_degree: int, n_slabs: int, p_xi: int,
                          n_levels: int) -> FiniteChaosWorkload:
    w = Workload(f"fc{n_cells_1d}q{fe_degree}r{time_degree}p{p_xi}", 2, n_cells_1d, fe_degree, time_degree,
                 1.0 / n_slabs, 4, p_xi, n_levels, "finite", lo=-1.0, hi=1.0)
    return FiniteChaosWorkload(w, n_slabs)


def uniform_vector(n: int, seed: int) -> np.ndarray:
    """FP64 vector of ``n`` entries drawn from U[-1, 1] with numpy's PCG64 generator."""
    return np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, size=n)


def coef_qp_levels(w: Workload, points_fn):
    """Coefficient values for every multigrid level, in the layout the slab library takes.

    ``points_fn(level)`` returns the physical quadrature points of that level as an array
    [n_cells, n_points, d]; each side (oracle or HIP library) supplies its own.
    Returns (mu_list, coef) with coef[level] of shape [n_mu, n_cells, n_points].
    """
    mus, out = None, []
    for level in range(w.n_levels):
        pts = np.asarray(points_fn(level))
        m, vals = coefficient_modes(w, pts)
        mus = m
        out.append(np.ascontiguousarray(vals, dtype=np.float64))
    return mus, out


def interior_target(w: Workload, seed: int = SEED_SOLVE_TARGET) -> np.ndarray:
    """Solve target x* for the benchmark: U[-1, 1] on interior nodes, 0 on the Dirichlet boundary.

    Layout [N_xi][N_t][n_nodes] with nodes lexicographic, x fastest, on (n_cells_1d k + 1)^d nodes.
    """
    n1 = w.n_nodes_1d(0)
    idx = np.arange(n1)
    inner1 = (idx > 0) & (idx < n1 - 1)
    inner = inner1
    for _ in range(w.dim - 1):
        inner = np.outer(inner1, inner).reshape(-1)
    x = uniform_vector(w.n_dofs(0), seed).reshape(w.n_chaos * w.n_time, -1)
    x[:, ~inner] = 0.0
    return x.reshape(-1)


# ---- adjoint workloads: a sequence of slabs, a parametrised coefficient, an initial value ------------
SEED_ADJOINT_A0 = 3


@dataclass(frozen=True)
class AdjointWorkload:
    """Slab sequence for the mean/variance QoI gradient: ``n_slabs`` slabs of ``base.tau``.

    Coefficient a(x, xi) = a_0(x) + sum_m theta_m phi_m(x) xi_m with a_0 constant on each finest cell
    (seeded 1 + a0_spread U[-1, 1]), phi_m the sine shapes; initial value u_0 = prod_k sin(pi x_k) in
    the mean mode; no forcing.
    """
    base: Workload
    n_slabs: int
    a0_spread: float = 0.2

    def theta0(self) -> np.ndarray:
        return np.array([0.1 / m ** 2 for m in range(1, self.base.n_vars + 1)])

    def a0_cells0(self) -> np.ndarray:
        n = self.base.n_cells_1d ** self.base.dim
        u = np.random.Generator(np.random.PCG64(SEED_ADJOINT_A0)).uniform(-1.0, 1.0, size=n)
        return 1.0 + self.a0_spread * u


ADJOINT_WORKLOADS = {
    # 3D Q2 on 16^3 cells, dG(1), tau = 0.01, 10 slabs, M = 3, p_xi = 3 (20 modes), 3-level GMG
    "c5": AdjointWorkload(Workload("c5", 3, 16, 2, 1, 0.01, 3, 3, 3, "sine"), 10),
    # small cases for the tests
    "a2": AdjointWorkload(Workload("a2", 2, 4, 2, 1, 0.02, 2, 2, 2, "sine"), 3),
    "a3": AdjointWorkload(Workload("a3", 3, 2, 2, 1, 0.02, 2, 2, 1, "sine"), 2),
}


def cell_means_to_coarse(a_cells: np.ndarray, dim: int, n: int) -> np.ndarray:
    """Per-cell values on n^d cells -> the mean over the 2^d children on (n/2)^d cells."""
    a = np.asarray(a_cells, dtype=np.float64).reshape((n,) * dim)   # [z][y][x] (x fastest in memory)
    for ax in range(dim):
        sl = [slice(None)] * dim
        sl0, sl1 = list(sl), list(sl)
        sl0[ax] = slice(0, None, 2)
        sl1[ax] = slice(1, None, 2)
        a = 0.5 * (a[tuple(sl0)] + a[tuple(sl1)])
    return a.reshape(-1)


def adjoint_coef_levels(aw: AdjointWorkload, theta, a0_cells, points_fn):
    """Coefficient values for every level in the slab library's layout, for parameters (theta, a0).

    Level 0 carries a_0 per cell; coarser levels the mean of the children.  Returns (mu_list, coef)
    with coef[level] of shape [M + 1, n_cells(level), n_points].
    """
    w = aw.base
    M = w.n_vars
    mus = [tuple([0] * M)] + [tuple(1 if j == m else 0 for j in range(M)) for m in range(M)]
    out = []
    a0 = np.asarray(a0_cells, dtype=np.float64)
    for level in range(w.n_levels):
        n = w.n_cells_1d >> level
        pts = np.asarray(points_fn(level))                 # [n_cells, n_points, d]
        vals = np.empty((M + 1,) + pts.shape[:2])
        vals[0] = a0[:, None]
        for m in range(1, M + 1):
            vals[m] = theta[m - 1] * _sine_shape(m, pts)
        out.append(vals)
        if level + 1 < w.n_levels:
            a0 = cell_means_to_coarse(a0, w.dim, n)
    return mus, out


def sine_shape_at(m: int, pts: np.ndarray) -> np.ndarray:
    """phi_m at the given points (the derivative field of a_{e_m} with respect to theta_m)."""
    return _sine_shape(m, np.asarray(pts, dtype=np.float64))


def initial_value(x: np.ndarray) -> np.ndarray:
    """u_0(x) = prod_k sin(pi x_k) (mean mode of the initial value)."""
    x = np.asarray(x, dtype=np.float64)
    return np.prod(np.sin(math.pi * x), axis=-1)


@dataclass(frozen=True)
class SampleWorkload:
    """A batch of pathwise (Monte-Carlo) problems: the slab sequence of ``base`` (``n_slabs`` slabs of
    ``base.tau``, initial value u_0 = prod_k sin(pi x_k), no forcing) with the coefficient of
    ``base.field`` evaluated at ``n_samples`` draws xi ~ N(0, I_M) from the PCG64 stream ``seed``.
    ``base.chaos_degree`` is not used."""
    base: Workload
    n_samples: int
    n_slabs: int
    seed: int = SEED_MC_DRAWS

    def samples(self) -> np.ndarray:
        g = np.random.Generator(np.random.PCG64(self.seed))
        return g.standard_normal((self.n_samples, self.base.n_vars))


SAMPLE_WORKLOADS = {
    # 256 samples of the 8x8-cell workload's coefficient on 2D Q2 64^2 cells, dG(1), tau = 0.01,
    # 20 slabs, 4-level GMG: 256 x 2 x 16641 = 8,520,192 DoFs per slab
    "c4": SampleWorkload(Workload("c4", 2, 64, 2, 1, 0.01, 2, 0, 4, "c1"), 256, 20),
    # small cases for the tests
    "m2": SampleWorkload(Workload("m2", 2, 4, 2, 1, 0.02, 2, 0, 2, "c1"), 12, 3, seed=5),
    "m3": SampleWorkload(Workload("m3", 3, 2, 2, 1, 0.02, 3, 0, 1, "sine"), 5, 2, seed=6),
    "m2q3": SampleWorkload(Workload("m2q3", 2, 4, 3, 2, 0.02, 2, 0, 2, "sine"), 7, 2, seed=7),
}


SEED_MEMBER_SCALES = 8


@dataclass(frozen=True)
class MemberWorkload:
    """A batch of independent stochastic Galerkin problems sharing the mesh, the time discretisation
    and the mean coefficient: member j has total degree ``degrees[j]`` and the coefficient
    a_0 + sum_m s_{j,m} a_{e_m} xi_m with s_{j,m} ~ U[0.5, 1.5] (PCG64 stream ``seed``); the slab
    sequence of ``base`` (``n_slabs`` slabs, u_0 = prod_k sin(pi x_k) in the mean mode, no forcing)."""
    base: Workload
    degrees: tuple
    n_slabs: int
    seed: int = SEED_MEMBER_SCALES

    def scales(self, coef_mu) -> np.ndarray:
        """[n_members, n_coef_modes]: 1 for mu = 0, the member's factor s_{j,m} for mu = e_m."""
        g = np.random.Generator(np.random.PCG64(self.seed))
        s = g.uniform(0.5, 1.5, size=(len(self.degrees), self.base.n_vars))
        out = np.ones((len(self.degrees), len(coef_mu)))
        for k, mu in enumerate(coef_mu):
            if sum(mu) == 1:
                out[:, k] = s[:, int(np.argmax(mu))]
            elif sum(mu) > 1:
                raise ValueError("member scales are defined for affine coefficients")
        return out


MEMBER_WORKLOADS = {
    # 64 SG problems, 16 each of degree 1, 2, 3, 4 (3 / 6 / 10 / 15 modes), on the 64^2-cell Q2 mesh
    # of the sample batch, dG(1), tau = 0.01, 20 slabs, 4-level GMG
    "c4": MemberWorkload(Workload("c4sg", 2, 64, 2, 1, 0.01, 2, 0, 4, "c1"), (1,) * 16 + (2,) * 16 + (3,) * 16 + (4,) * 16, 20),
    # small cases for the tests
    "b2": MemberWorkload(Workload("b2", 2, 4, 2, 1, 0.02, 2, 0, 2, "c1"), (1, 2, 3, 0, 2), 3, seed=9),
    "b3": MemberWorkload(Workload("b3", 3, 2, 2, 1, 0.02, 3, 0, 1, "sine"), (1, 2), 2, seed=10),
}


@dataclass(frozen=True)
class MCErrorWorkload:
    """Monte-Carlo study of the finite-chaos benchmark: pathwise problems (coefficient and forcing of
    Section 3.2 at xi^(s)) discretised with ``base`` (field "finite", dim 2, (-1, 1)^2, chaos degree
    unused), ``n_slabs`` slabs of tau = T / n_slabs, ``n_samples`` draws xi ~ N(0, I_4) from the PCG64
    stream ``seed``, solved ``batch`` samples per handle."""
    base: Workload
    n_slabs: int
    n_samples: int
    batch: int
    seed: int

    def samples(self) -> np.ndarray:
        g = np.random.Generator(np.random.PCG64(self.seed))
        return g.standard_normal((self.n_samples, 4))


def mc_error_workload(n_cells_1d: int, fe_degree: int, time_degree: int, n_slabs: int, n_samples: int, batch: int,
                      seed: int, n_levels: int) -> MCErrorWorkload:
    w = Workload(f"mc{n_cells_1d}q{fe_degree}r{time_degree}", 2, n_cells_1d, fe_degree, time_degree, 1.0 / n_slabs, 4,
                 0, n_levels, "finite", lo=-1.0, hi=1.0)
    return MCErrorWorkload(w, n_slabs, n_samples, batch, seed)


MC_ERROR_WORKLOADS = {
    # 2D Q3 on 32^2 cells of (-1,1)^2 (h = 1/16), dG(3), tau = 1/16 (16 slabs), 512 samples in 4 handles
    "c6": mc_error_workload(32, 3, 3, 16, 512, 128, 12, 4),
    # the same discretisation and draw stream with 2048 samples in 16 handles (its first 512 samples
    # are c6's): the cumulative windows N = 128, 256, ..., 2048 give the root-N diagnostic
    "c7": mc_error_workload(32, 3, 3, 16, 2048, 128, 12, 4),
    # small cases for the tests
    "e2": mc_error_workload(4, 3, 3, 2, 6, 3, 13, 2),
    "e3": mc_error_workload(4, 2, 1, 3, 5, 5, 14, 2),
}
