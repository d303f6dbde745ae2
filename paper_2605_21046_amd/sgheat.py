"""Python binding of libsgheat.so (include/sgheat.h): argument marshalling only.

Every numerical step runs in the library's gfx950 kernels; PyTorch provides device memory and
the current HIP stream.  Importing this module loads the library and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SGHEAT_LIB", os.path.join(_HERE, "libsgheat.so"))

SG_OK, SG_NOT_CONVERGED = 0, 1
SG_FP64, SG_MIXED = 0, 1
_STATUS = {0: "SG_OK", 1: "SG_NOT_CONVERGED", -1: "SG_EINVAL", -2: "SG_ENOMEM", -3: "SG_EHIP",
           -4: "SG_ESINGULAR", -5: "SG_EUNSUPPORTED"}
EXPORTS = ["sg_create", "sg_destroy", "sg_vector_length", "sg_operator_apply", "sg_operator_apply_noalloc", "sg_vanka_smooth",
           "gmg_vcycle", "fgmres_solve_slab", "sg_quadrature_points", "sg_node_coordinates", "sg_update_coefficients", "sg_operator_apply_T",
           "sg_slab_transfer", "sg_stiffness_form_cells", "sg_stiffness_form_accumulate", "sg_qoi_mean_var", "sg_sample_statistics", "sg_chaos_moments", "sg_gauss_points", "sg_index_set", "sg_chaos_projection",
           "sg_time_rule", "sg_time_load_weights", "sg_load_vectors", "sg_separable_vector", "sg_separable_error",
           "sg_sample_psi", "sg_sample_qp_moments", "sg_moment_errors", "sg_autotune", "sg_set_vcycle_graph", "sg_set_vcycle_segment", "sg_last_error"]


class SgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class ProblemDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells_1d", ctypes.c_int), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("fe_degree", ctypes.c_int), ("time_degree", ctypes.c_int),
                ("tau", ctypes.c_double), ("n_vars", ctypes.c_int), ("chaos_degree", ctypes.c_int),
                ("n_coef_modes", ctypes.c_int), ("coef_mu", ctypes.POINTER(ctypes.c_int)),
                ("coef_qp", ctypes.POINTER(ctypes.c_double)), ("n_levels", ctypes.c_int),
                ("pre_smooth", ctypes.c_int), ("post_smooth", ctypes.c_int), ("vanka_omega", ctypes.c_double),
                ("fgmres_restart", ctypes.c_int), ("precision", ctypes.c_int), ("n_samples", ctypes.c_int),
                ("samples", ctypes.POINTER(ctypes.c_double)), ("n_members", ctypes.c_int),
                ("member_degree", ctypes.POINTER(ctypes.c_int)), ("member_scale", ctypes.POINTER(ctypes.c_double)),
                ("diag_blocks", ctypes.c_int), ("transpose", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("vcycles", ctypes.c_int),
                ("applies", ctypes.c_int), ("converged", ctypes.c_int), ("rel_residual_true", ctypes.c_double),
                ("t_apply_ms", ctypes.c_double), ("t_prec_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("work_proxy", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.sg_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(P)]
    lib.sg_destroy.argtypes = [P]
    lib.sg_vector_length.argtypes = [P, I, ctypes.POINTER(ctypes.c_longlong)]
    lib.sg_operator_apply.argtypes = [P, V, V, V]
    lib.sg_vanka_smooth.argtypes = [P, I, V, V, I, V]
    lib.gmg_vcycle.argtypes = [P, V, V, V]
    lib.fgmres_solve_slab.argtypes = [P, V, V, D, I, ctypes.POINTER(SolveInfo), V]
    lib.sg_quadrature_points.argtypes = [ctypes.POINTER(ProblemDesc), I, ctypes.POINTER(ctypes.c_double)]
    lib.sg_node_coordinates.argtypes = [ctypes.POINTER(ProblemDesc), I, ctypes.POINTER(ctypes.c_double)]
    lib.sg_update_coefficients.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.sg_operator_apply_T.argtypes = [P, V, V, V]
    lib.sg_slab_transfer.argtypes = [P, I, V, V, V]
    lib.sg_stiffness_form_cells.argtypes = [P, I, ctypes.POINTER(ctypes.c_double), V, V, V, V]
    lib.sg_stiffness_form_accumulate.argtypes = [P, I, ctypes.POINTER(ctypes.c_double), V, V, D, V, V, V]
    lib.sg_qoi_mean_var.argtypes = [P, V, D, D, ctypes.POINTER(ctypes.c_double), V, V]
    lib.sg_sample_statistics.argtypes = [P, V, V, V, V]
    lib.sg_chaos_moments.argtypes = [P, V, V, V, V]
    PD, PI = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.sg_gauss_points.argtypes = [ctypes.POINTER(ProblemDesc), I, I, PD]
    lib.sg_index_set.argtypes = [P, PI]
    lib.sg_chaos_projection.argtypes = [P, I, PI, PD, PD]
    lib.sg_time_rule.argtypes = [P, I, PD, PD]
    lib.sg_time_load_weights.argtypes = [P, I, I, PD, PD]
    lib.sg_load_vectors.argtypes = [P, I, I, V, V, V, V]
    lib.sg_separable_vector.argtypes = [P, I, PD, V, D, V, V]
    lib.sg_separable_error.argtypes = [P, V, I, V, V, I, PD, PD, D, PD, V]
    lib.sg_sample_psi.argtypes = [P, I, PI, PD]
    lib.sg_autotune.argtypes = [P, I, PI, V]
    lib.sg_set_vcycle_graph.argtypes = [P, I]
    lib.sg_set_vcycle_segment.argtypes = [P, I, PI]
    lib.sg_sample_qp_moments.argtypes = [P, V, I, I, V, V]
    lib.sg_moment_errors.argtypes = [P, V, ctypes.c_longlong, I, V, I, PD, PD, PD, PD, V]
    lib.sg_last_error.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f != "sg_last_error":
            getattr(lib, f).restype = ctypes.c_int
    return lib


_lib = load_library()


def _check(status: int, allow_not_converged: bool = False) -> int:
    if status == SG_OK or (allow_not_converged and status == SG_NOT_CONVERGED):
        return status
    raise SgError(status, _lib.sg_last_error().decode())


@dataclass
class Spec:
    """Sizes of one slab problem (names as in the paper)."""
    dim: int
    n_cells_1d: int
    fe_degree: int
    time_degree: int
    tau: float
    n_vars: int
    chaos_degree: int
    n_levels: int
    lo: float = 0.0
    hi: float = 1.0
    pre_smooth: int = 1
    post_smooth: int = 1
    vanka_omega: float = 1.0
    fgmres_restart: int = 30
    transpose: int = 0
    diag_blocks: int = 0


def _desc(spec, precision=SG_FP64):
    d = ProblemDesc()
    for name in ["dim", "n_cells_1d", "fe_degree", "time_degree", "n_vars", "chaos_degree", "n_levels",
                 "pre_smooth", "post_smooth", "fgmres_restart", "transpose", "diag_blocks"]:
        setattr(d, name, int(getattr(spec, name)))
    for name in ["lo", "hi", "tau", "vanka_omega"]:
        setattr(d, name, float(getattr(spec, name)))
    d.precision = int(precision)
    return d


def quadrature_points(spec, level: int) -> np.ndarray:
    """Physical Gauss points of a level, [n_cells, (k+1)^d, d] (where coef_qp is sampled)."""
    d = _desc(spec)
    n = spec.n_cells_1d >> level
    npts = (spec.fe_degree + 1) ** spec.dim
    out = np.zeros((n ** spec.dim, npts, spec.dim))
    _check(_lib.sg_quadrature_points(ctypes.byref(d), level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def gauss_points(spec, level: int, nq1: int) -> np.ndarray:
    """Physical points of the nq1-point Gauss rule per direction, [n_cells, nq1^d, d]."""
    d = _desc(spec)
    n = spec.n_cells_1d >> level
    out = np.zeros((n ** spec.dim, nq1 ** spec.dim, spec.dim))
    _check(_lib.sg_gauss_points(ctypes.byref(d), level, nq1, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def node_coordinates(spec, level: int) -> np.ndarray:
    """Physical node coordinates of a level, [n_nodes, d] (lexicographic, x fastest)."""
    d = _desc(spec)
    n1 = (spec.n_cells_1d >> level) * spec.fe_degree + 1
    out = np.zeros((n1 ** spec.dim, spec.dim))
    _check(_lib.sg_node_coordinates(ctypes.byref(d), level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def _ptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Problem:
    """One slab problem on the GPU (a handle of libsgheat.so)."""

    def __init__(self, spec, coef_mu, coef_qp_levels, precision=SG_FP64, samples=None, members=None):
        """samples: None for the stochastic Galerkin operator, or [n_samples, n_vars] points xi^(s) for a
        batch of pathwise problems (block s = the deterministic slab system at a(x, xi^(s))).
        members: None, or (degrees [J], scales [J, n_coef_modes]) for a batch of J independent SG
        problems (member j: total degree degrees[j], coefficient sum_mu scales[j, mu] a_mu)."""
        self.spec = spec
        mus = np.ascontiguousarray(np.asarray(coef_mu, dtype=np.int32).reshape(-1, spec.n_vars))
        coef = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64).reshape(-1) for c in coef_qp_levels]))
        d = _desc(spec, precision)
        d.n_coef_modes = mus.shape[0]
        d.coef_mu = mus.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.coef_qp = coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        n_modes = math_comb(spec.n_vars + spec.chaos_degree, spec.chaos_degree)
        if samples is not None:
            xi = np.ascontiguousarray(np.asarray(samples, dtype=np.float64).reshape(-1, spec.n_vars))
            d.n_samples = xi.shape[0]
            d.samples = xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            n_modes = xi.shape[0]
        self.member_modes = [n_modes]
        if members is not None:
            deg = np.ascontiguousarray(np.asarray(members[0], dtype=np.int32).reshape(-1))
            sc = np.ascontiguousarray(np.asarray(members[1], dtype=np.float64).reshape(deg.size, mus.shape[0]))
            d.n_members = deg.size
            d.member_degree = deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
            d.member_scale = sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self.member_modes = [math_comb(spec.n_vars + int(p), int(p)) for p in deg]
            n_modes = sum(self.member_modes)
        h = ctypes.c_void_p()
        _check(_lib.sg_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.precision = precision
        self.n_samples = 0 if samples is None else n_modes
        self.n_mu = mus.shape[0]
        self.shape = (n_modes, spec.time_degree + 1, (spec.n_cells_1d * spec.fe_degree + 1) ** spec.dim)

    def update_coefficients(self, coef_qp_levels):
        """New coefficient values (same modes and layout as at construction); keeps the allocations."""
        coef = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64).reshape(-1) for c in coef_qp_levels]))
        _check(_lib.sg_update_coefficients(self._h, coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n(self, level: int = 0) -> int:
        v = ctypes.c_longlong()
        _check(_lib.sg_vector_length(self._h, level, ctypes.byref(v)))
        return v.value

    def apply(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        n = self.n(0)
        _check(_lib.sg_operator_apply(self._h, _ptr(x, n, "x"), _ptr(y, n, "y"), _stream(stream)))
        return y

    def apply_noalloc(self, x, y, stream=None):
        """y = AA x through sg_operator_apply_noalloc (no device allocation; y must be given)."""
        n = self.n(0)
        _check(_lib.sg_operator_apply_noalloc(self._h, _ptr(x, n, "x"), _ptr(y, n, "y"), _stream(stream)))
        return y

    def apply_T(self, x, y=None, stream=None):
        """y = AA^T x (AA x for a handle made with transpose=1)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        n = self.n(0)
        _check(_lib.sg_operator_apply_T(self._h, _ptr(x, n, "x"), _ptr(y, n, "y"), _stream(stream)))
        return y

    def slab_transfer(self, x, y=None, transpose=False, stream=None):
        """y = (I (x) C_t (x) M_x) x, or with C_t^T."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        n = self.n(0)
        _check(_lib.sg_slab_transfer(self._h, int(bool(transpose)), _ptr(x, n, "x"), _ptr(y, n, "y"), _stream(stream)))
        return y

    def stiffness_form_cells(self, mu_index, coef_qp, lam, u, out=None, stream=None):
        """out[K] = lam^T (G_mu (x) B_t (x) K_{c|K}) u for the field c given at the level-0 Gauss points."""
        import torch
        n = self.n(0)
        n_cells = self.spec.n_cells_1d ** self.spec.dim
        c = np.ascontiguousarray(np.asarray(coef_qp, dtype=np.float64).reshape(n_cells, -1))
        if out is None:
            out = torch.empty(n_cells, dtype=torch.float64, device=lam.device)
        _check(_lib.sg_stiffness_form_cells(self._h, int(mu_index), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            _ptr(lam, n, "lam"), _ptr(u, n, "u"), _ptr(out, n_cells, "out"),
                                            _stream(stream)))
        return out

    def stiffness_form_accumulate(self, mu_index, coef_qp, lam, u, scale, cells=None, total=None, stream=None):
        """cells[K] += scale out[K] and total[0] += scale sum_K out[K] on the device, with out[K] as in
        stiffness_form_cells (either target may be None, not both)."""
        n = self.n(0)
        n_cells = self.spec.n_cells_1d ** self.spec.dim
        c = np.ascontiguousarray(np.asarray(coef_qp, dtype=np.float64).reshape(n_cells, -1))
        _check(_lib.sg_stiffness_form_accumulate(
            self._h, int(mu_index), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(lam, n, "lam"),
            _ptr(u, n, "u"), float(scale), None if cells is None else _ptr(cells, n_cells, "cells"),
            None if total is None else _ptr(total, 1, "total"), _stream(stream)))

    def qoi_mean_var(self, u, w_mean=1.0, w_var=1.0, grad=None, stream=None):
        """(E[Q], Var[Q]) of Q = int_D u(T)^2 and, if grad is a tensor, dJ/du for J = w_mean E + w_var Var."""
        n = self.n(0)
        q = (ctypes.c_double * 2)()
        g = _ptr(grad, n, "grad") if grad is not None else None
        _check(_lib.sg_qoi_mean_var(self._h, _ptr(u, n, "u"), float(w_mean), float(w_var), q, g, _stream(stream)))
        return float(q[0]), float(q[1])

    def sample_statistics(self, u, mean=None, var=None, stream=None):
        """Sample mean and unbiased sample variance over the batch, each [N_t * n_nodes] (var optional)."""
        import torch
        n = self.n(0)
        m = self.shape[1] * self.shape[2]
        if mean is None:
            mean = torch.empty(m, dtype=torch.float64, device=u.device)
        v = _ptr(var, m, "var") if var is not None else None
        _check(_lib.sg_sample_statistics(self._h, _ptr(u, n, "u"), _ptr(mean, m, "mean"), v, _stream(stream)))
        return mean, var

    def chaos_moments(self, u, mean=None, var=None, stream=None):
        """Per member: mean (first mode) and variance (sum of squares of the other modes), each
        [n_members * N_t * n_nodes] (var optional)."""
        import torch
        n = self.n(0)
        m = len(self.member_modes) * self.shape[1] * self.shape[2]
        if mean is None:
            mean = torch.empty(m, dtype=torch.float64, device=u.device)
        v = _ptr(var, m, "var") if var is not None else None
        _check(_lib.sg_chaos_moments(self._h, _ptr(u, n, "u"), _ptr(mean, m, "mean"), v, _stream(stream)))
        return mean, var

    # --- prescribed solutions and forcing ------------------------------------------------------------
    def index_set(self) -> np.ndarray:
        out = np.zeros((self.shape[0], self.spec.n_vars), dtype=np.int32)
        _check(_lib.sg_index_set(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return out

    def chaos_projection(self, src_alpha, src_c) -> np.ndarray:
        """out[mu, beta] = sum_s src_c[s] E[Psi_mu Psi_{src_alpha[s]} Psi_beta] (coefficient modes x modes)."""
        a = np.ascontiguousarray(np.asarray(src_alpha, dtype=np.int32).reshape(-1, self.spec.n_vars))
        c = np.ascontiguousarray(np.asarray(src_c, dtype=np.float64).reshape(-1))
        out = np.zeros((self.n_mu, self.shape[0]))
        _check(_lib.sg_chaos_projection(self._h, a.shape[0], a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(c),
                                        _dp(out)))
        return out

    def time_rule(self, ntq: int):
        s, w = np.zeros(ntq), np.zeros(ntq)
        _check(_lib.sg_time_rule(self._h, ntq, _dp(s), _dp(w)))
        return s, w

    def time_load_weights(self, gvals) -> np.ndarray:
        g = np.ascontiguousarray(np.atleast_2d(np.asarray(gvals, dtype=np.float64)))
        out = np.zeros((g.shape[0], self.shape[1]))
        _check(_lib.sg_time_load_weights(self._h, g.shape[1], g.shape[0], _dp(g), _dp(out)))
        return out

    def load_vectors(self, nq1, fval=None, fgrad=None, n_fields=None, out=None, stream=None):
        """Spatial loads [n_fields, n_nodes] of fields at the nq1-point Gauss rule (device tensors)."""
        import torch
        nf = n_fields if n_fields is not None else (fval if fval is not None else fgrad).shape[0]
        n_cells = self.spec.n_cells_1d ** self.spec.dim
        nq = nq1 ** self.spec.dim
        if out is None:
            out = torch.empty(nf, self.shape[2], dtype=torch.float64, device="cuda")
        fv = _ptr(fval, nf * n_cells * nq, "fval") if fval is not None else None
        fg = _ptr(fgrad, nf * n_cells * nq * self.spec.dim, "fgrad") if fgrad is not None else None
        _check(_lib.sg_load_vectors(self._h, nq1, nf, fv, fg, _ptr(out, nf * self.shape[2], "out"), _stream(stream)))
        return out

    def separable_vector(self, W, V, y, beta=0.0, stream=None):
        """y = beta y + sum_t W[t] (x) V[t], W [n_terms, N_xi, N_t] (host), V [n_terms, n_nodes] (device)."""
        Wc = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(-1, self.shape[0], self.shape[1]))
        nt = Wc.shape[0]
        _check(_lib.sg_separable_vector(self._h, nt, _dp(Wc), _ptr(V, nt * self.shape[2], "V"), float(beta),
                                        _ptr(y, self.n(0), "y"), _stream(stream)))
        return y

    def separable_error(self, u, nq1, s_qp, gs_qp, theta, c, C2, stream=None) -> np.ndarray:
        """The 8 error sums of one slab against theta(t) s(x) sum_a c_a Psi_a (see the header)."""
        n_cells = self.spec.n_cells_1d ** self.spec.dim
        nq = nq1 ** self.spec.dim
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        assert cc.size == self.shape[0]
        out = np.zeros(8)
        _check(_lib.sg_separable_error(self._h, _ptr(u, self.n(0), "u"), nq1, _ptr(s_qp, n_cells * nq, "s_qp"),
                                       _ptr(gs_qp, n_cells * nq * self.spec.dim, "gs_qp"), th.size, _dp(th), _dp(cc),
                                       float(C2), _dp(out), _stream(stream)))
        return out

    def set_vcycle_segment(self, enable: bool = True) -> int:
        """Coarse levels of the V-cycle as one persistent launch or kernel by kernel (the default);
        returns the first level the segment covers (-1: the hierarchy has none)."""
        lvl = ctypes.c_int(-1)
        _check(_lib.sg_set_vcycle_segment(self._h, 1 if enable else 0, ctypes.byref(lvl)))
        return lvl.value

    def vcycle_segment_level(self) -> int:
        """First level of the coarse segment while it runs as one launch, else -1."""
        lvl = ctypes.c_int(-1)
        _check(_lib.sg_set_vcycle_segment(self._h, -1, ctypes.byref(lvl)))
        return lvl.value

    def set_vcycle_graph(self, enable: bool = True):
        """Replay the V-cycle from a HIP graph (captured on first use) instead of launching its kernels."""
        _check(_lib.sg_set_vcycle_graph(self._h, int(bool(enable))))

    def autotune(self, reps: int = 20, stream=None) -> dict:
        """Time the cell kernel's workgroup tiles (and the V-cycle with and without the coarse segment)
        on this handle and keep the fastest; returns the choices."""
        L = self.spec.n_levels
        out = np.zeros((2, 2, L), dtype=np.int32)
        _check(_lib.sg_autotune(self._h, int(reps), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _stream(stream)))
        return {"fp64_full": int(out[0, 1, 0]), "fp64_mean": out[0, 0].tolist(),
                "fp32_mean": out[1, 0].tolist() if self.precision == SG_MIXED else None,
                "segment_level": self.vcycle_segment_level()}

    # --- Monte-Carlo estimators at quadrature points --------------------------------------------------
    def sample_psi(self, alphas) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(alphas, dtype=np.int32).reshape(-1, self.spec.n_vars))
        out = np.zeros((self.n_samples, a.shape[0]))
        _check(_lib.sg_sample_psi(self._h, a.shape[0], a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out)))
        return out

    def qp_moment_length(self, nq1, ntq) -> int:
        return (self.spec.n_cells_1d ** self.spec.dim) * nq1 ** self.spec.dim * ntq * 2

    def sample_qp_moments(self, u, nq1, ntq, acc, stream=None):
        _check(_lib.sg_sample_qp_moments(self._h, _ptr(u, self.n(0), "u"), nq1, ntq,
                                         _ptr(acc, self.qp_moment_length(nq1, ntq), "acc"), _stream(stream)))
        return acc

    def moment_errors(self, acc, n_tot, nq1, s_qp, theta, mean_targets, var_targets, stream=None) -> np.ndarray:
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        mt = np.ascontiguousarray(np.asarray(mean_targets, dtype=np.float64))
        vt = np.ascontiguousarray(np.asarray(var_targets, dtype=np.float64))
        out = np.zeros(6)
        n_cells = self.spec.n_cells_1d ** self.spec.dim
        _check(_lib.sg_moment_errors(self._h, _ptr(acc, self.qp_moment_length(nq1, th.size), "acc"), int(n_tot), nq1,
                                     _ptr(s_qp, n_cells * nq1 ** self.spec.dim, "s_qp"), th.size, _dp(th), _dp(mt),
                                     _dp(vt), _dp(out), _stream(stream)))
        return out

    def vanka_smooth(self, level, b, x, sweeps=1, stream=None):
        n = self.n(level)
        _check(_lib.sg_vanka_smooth(self._h, level, _ptr(b, n, "b"), _ptr(x, n, "x"), sweeps, _stream(stream)))
        return x

    def vcycle(self, r, z=None, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(r)
        n = self.n(0)
        _check(_lib.gmg_vcycle(self._h, _ptr(r, n, "r"), _ptr(z, n, "z"), _stream(stream)))
        return z

    def solve(self, b, x=None, rtol=1e-8, max_iter=1000, stream=None):
        import torch
        if x is None:
            x = torch.zeros_like(b)
        n = self.n(0)
        info = SolveInfo()
        st = _lib.fgmres_solve_slab(self._h, _ptr(b, n, "b"), _ptr(x, n, "x"), float(rtol), int(max_iter),
                                    ctypes.byref(info), _stream(stream))
        _check(st, allow_not_converged=True)
        return x, info.as_dict()


def math_comb(a, b):
    import math
    return math.comb(a, b)


def problem_from_workload(w, precision=SG_FP64, **overrides):
    """Problem for an sg_inputs.Workload, with coefficients sampled at this library's Gauss points."""
    import sg_inputs
    spec = Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree, w.n_levels,
                w.lo, w.hi, w.pre_smooth, w.post_smooth, w.vanka_omega, w.fgmres_restart)
    for k, v in overrides.items():
        setattr(spec, k, v)
    mus, coef = sg_inputs.coef_qp_levels(w, lambda lvl: quadrature_points(spec, lvl))
    return Problem(spec, mus, coef, precision)
