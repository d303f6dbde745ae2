// C ABI of libsgheat.so (declared in include/sgheat.h): handle set-up and the host orchestration of
// the slab operator, the Vanka smoother, the geometric-multigrid V-cycle and flexible GMRES.
//
// Everything numerical runs in the gfx950 kernels of kernels_*.hip; this file only validates
// arguments, builds small host tables (1D bases, time matrices, chaos coupling lists, transfer
// stencils), inverts the coarsest-level matrix once, and enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sgheat.h"
#include "basis.hpp"
#include "kernels.hpp"
#include "krylov.hpp"
#include "forcing.hpp"

using namespace sg;

namespace {

thread_local std::string g_last_error;

sg_status fail(sg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define SG_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(SG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

#define SG_TRY(call)                                                                                   \
    do {                                                                                               \
        sg_status s_ = (call);                                                                         \
        if (s_ != SG_OK) return s_;                                                                    \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    ~DevBuf() { if (p) (void)hipFree(p); }
    sg_status alloc(size_t count, const char* what) {
        if (p && n == count) return SG_OK;   // same size: keep the allocation
        if (p) (void)hipFree(p);
        p = nullptr;
        n = count;
        if (count == 0) return SG_OK;
        if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(SG_ENOMEM, std::string("device allocation failed: ") + what);
        }
        return SG_OK;
    }
    sg_status upload(const T* host, size_t count, const char* what) {
        SG_TRY(alloc(count, what));
        if (count) SG_HIP(hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice));
        return SG_OK;
    }
};

struct Level {
    Grid g{};
    double h = 0.0;
    Tables<double> tab64{};
    Tables<float> tab32{};
    DevBuf<double> coef64;   // level 0: every mode; other levels: the mean mode only
    DevBuf<float> coef32;
    DevBuf<double> inv64;    // patch inverses [slots][vanka_inv_stride(npp)] (fragment layout)
    DevBuf<float> inv32;
    int inv_classes = 0;     // 1: one inverse per position class (inverse_slot), 3^d slots; 0: one per cell
    bool mean_const = false;                 // mean coefficient one constant: mean block as a Kronecker sum
    DevBuf<double> mb64, kb64;               // its assembled 1D mass / stiffness bands [n1][2k+1] (K times c)
    DevBuf<float> mb32, kb32;
    // and its Vanka corrections by fast diagonalisation: per-direction transforms of the first / inner /
    // last cell [3][k+1][k+1] and inverted time blocks per position class [3^d][(k+1)^d][N_t][N_t]
    DevBuf<double> fdmS64, fdmT64;
    DevBuf<float> fdmS32, fdmT32;
    DevBuf<int> class_cells; // a representative cell of every position class
    DevBuf<double> E64;      // levels of the coarse segment: element stiffness of the mean coefficient
    DevBuf<double> Me64;     // and the element mass
    // transfer stencils between this level (fine) and level + 1 (coarse)
    int wp = 0, wr = 0;
    DevBuf<int> p_idx, r_idx;
    DevBuf<double> p_w64, r_w64;
    DevBuf<float> p_w32, r_w32;
    // work vectors of the V-cycle
    DevBuf<double> b64, x64, r64;
    DevBuf<float> b32, x32, r32;
    long long len = 0;       // N_xi * N_t * n_nodes
};

}  // namespace

struct sg_handle_s {
    sg_problem_desc d{};
    int device = -1;                    // the GPU the handle's buffers live on
    std::vector<int> coef_mu;
    std::vector<double> samples;   // sample-batch handles: [n_samples][n_vars]
    std::vector<int> member_degree;     // member batches: [n_members]
    std::vector<double> member_scale;   // [n_members][n_mu]
    std::vector<int> member_off;        // first mode of every member, n_members + 1 entries
    DevBuf<int> moff;                   // member_off on the device
    int NP = 0, NT = 0, n_xi = 0, n_mu = 0, npp = 0;
    Coupling cpl;
    bool mixed = false;
    std::vector<double> At, Bt;
    std::vector<Level> lv;
    // coupling lists
    DevBuf<int> cptr, cbeta, cmu, cptr_m, cbeta_m, cmu_m;
    DevBuf<double> cw64, cw_m64;
    DevBuf<float> cw32, cw_m32;
    // per-mode diagonal blocks (desc.diag_blocks): weights dw[alpha][mu] = [G_mu]_{alpha alpha} and the
    // diagonal coupling lists of the block operator
    bool diag = false;
    std::vector<double> dw;
    DevBuf<int> cptr_d, cbeta_d, cmu_d;
    DevBuf<double> cw_d64, acomb;
    DevBuf<float> cw_d32;
    int n_ent_d = 0;
    // coarsest level
    int nint = 0;
    DevBuf<double> coarse_invT;
    DevBuf<int> coarse_dofs;
    // transfer temporaries
    DevBuf<double> t64a, t64b;
    DevBuf<float> t32a, t32b;
    // Krylov workspace
    int restart = 30;
    DevBuf<double> V, Z, w1, w2, partial, dscal;
    // cell-local results in the broken node layout (shared by every operator call; FP32 calls reuse it)
    DevBuf<double> sbuf;
    std::vector<double> hbuf;
    long long N = 0;
    // operator variants on level 0: 1D tables, the other orientation of A_t, the end-of-slab
    // transfer, scratch for the bilinear forms and the quantity of interest
    std::vector<double> tS, tD, tDn, tgw, radau0, Me1;   // radau0[i] = v_i(0+); Me1: unit-cell mass
    Tables<double> tabT64{};
    DevBuf<double> zcoef, fcoef, qpart, qout, qC;
    DevBuf<double> elem_E, elem_M;             // element matrices of the patch set-up (reused)
    DevBuf<double> sepW, errC, errPart, errOut;  // separable weights, error-sum work arrays
    DevBuf<double> momPart;                      // moment-error partial sums
    int tuned_cpb[2][2][16] = {};                // apply cells per workgroup from sg_autotune: [FP32][full][level]
    // V-cycle replayed from a HIP graph (sg_set_vcycle_graph): captured on the level-0 work vectors
    bool graph_on = false;
    int seg_level = -1;          // first level of the coarse segment run as one launch (-1: none)
    bool seg_on = false;
    int graph_calls = 0;
    hipGraph_t vgraph = nullptr;
    hipGraphExec_t vgraph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    void drop_graph() {
        if (vgraph_exec) (void)hipGraphExecDestroy(vgraph_exec);
        if (vgraph) (void)hipGraphDestroy(vgraph);
        vgraph_exec = nullptr;
        vgraph = nullptr;
        graph_calls = 0;
    }
    std::vector<hipEvent_t> ev_pool;          // timing events of the solver, created once and reused
    // recorded on the caller's stream at the end of every asynchronous call: calls on one handle are
    // ordered by the caller, so once it completes no earlier work of the handle is pending either
    hipEvent_t last_work = nullptr;
    // cell-wise forms: the last field of every mode as given (host) and scaled on the device, and the
    // mode whose field sits in fcoef (whose other modes stay zero)
    std::vector<std::vector<double>> form_raw;
    DevBuf<double> form_fields, form_cells;
    int form_active = -1;
    ~sg_handle_s() {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        if (last_work) (void)hipEventDestroy(last_work);
    }
    // waits for the handle's last asynchronous call, not for the whole device
    void quiesce() {
        if (last_work) (void)hipEventSynchronize(last_work);
    }
    std::vector<double> hstage;
    std::vector<double> trip;                 // E[Psi_a Psi_b Psi_eps], [n_xi][n_xi][n_eps]
    int n_eps = 0;
};

namespace {

// Records the handle's completion event on the caller's stream when an entry point returns (not
// while the stream is being captured into a graph: the caller's graph owns that work).
struct WorkMark {
    sg_handle h;
    hipStream_t s;
    ~WorkMark() {
        if (!h || !h->last_work) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
            (void)hipEventRecord(h->last_work, s);
    }
};

int ipow_h(int b, int e) {
    int r = 1;
    while (e--) r *= b;
    return r;
}

template <typename T>
void fill_tables(Tables<T>* tb, const std::vector<double>& S, const std::vector<double>& D,
                 const std::vector<double>& w, const std::vector<double>& At, const std::vector<double>& Bt, int N1,
                 int NT, double vol) {
    std::memset(tb, 0, sizeof(*tb));
    for (int i = 0; i < N1 * N1; ++i) {
        tb->S[i] = (T)S[i];
        tb->D[i] = (T)D[i];
    }
    for (int i = 0; i < N1; ++i) tb->w[i] = (T)w[i];
    for (int i = 0; i < NT; ++i) {
        tb->Bt[i] = (T)Bt[i];
        for (int j = 0; j < NT; ++j) tb->As[i * NT + j] = (T)(At[i * NT + j] / Bt[i]);
    }
    tb->vol = (T)vol;
}

sg_status validate(const sg_problem_desc* d) {
    if (!d) return fail(SG_EINVAL, "desc is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(SG_EINVAL, "dim must be 2 or 3");
    if (d->fe_degree < 1 || d->fe_degree > 4) return fail(SG_EINVAL, "fe_degree must be in 1..4");
    if (d->time_degree < 0 || d->time_degree > 3) return fail(SG_EINVAL, "time_degree must be in 0..3");
    if (d->n_cells_1d < 1) return fail(SG_EINVAL, "n_cells_1d must be >= 1");
    if (!(d->hi > d->lo)) return fail(SG_EINVAL, "hi must exceed lo");
    if (!(d->tau > 0.0)) return fail(SG_EINVAL, "tau must be positive");
    if (d->n_vars < 1 || d->chaos_degree < 0) return fail(SG_EINVAL, "n_vars >= 1 and chaos_degree >= 0 required");
    if (d->n_coef_modes < 1 || !d->coef_mu || !d->coef_qp) return fail(SG_EINVAL, "coefficient arrays missing");
    if (d->n_levels < 1 || d->n_levels > 12) return fail(SG_EINVAL, "n_levels must be in 1..12");
    if (d->n_cells_1d % (1 << (d->n_levels - 1)) != 0)
        return fail(SG_EINVAL, "n_cells_1d must be divisible by 2^(n_levels-1)");
    if (d->pre_smooth < 0 || d->post_smooth < 0) return fail(SG_EINVAL, "smoothing counts must be >= 0");
    if (d->fgmres_restart < 1 || d->fgmres_restart > 64) return fail(SG_EINVAL, "fgmres_restart must be in 1..64");
    if (d->precision != SG_FP64 && d->precision != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
    if (d->transpose != 0 && d->transpose != 1) return fail(SG_EINVAL, "transpose must be 0 or 1");
    if (d->n_samples < 0 || (d->n_samples > 0 && !d->samples)) return fail(SG_EINVAL, "samples missing");
    if (d->n_members < 0 || (d->n_members > 0 && (!d->member_degree || !d->member_scale)))
        return fail(SG_EINVAL, "member_degree / member_scale missing");
    if (d->n_members > 0 && d->n_samples > 0) return fail(SG_EINVAL, "n_samples and n_members are exclusive");
    if (d->diag_blocks != 0 && d->diag_blocks != 1) return fail(SG_EINVAL, "diag_blocks must be 0 or 1");
    return SG_OK;
}

// 1D prolongation stencil from a coarse level with nc cells to the fine level with 2 nc cells:
// fine node f takes sum_a l_a(t) * coarse node (c k + a); rows and columns of Dirichlet nodes are 0.
void prolong_1d(int nc, int k, const std::vector<double>& gll, std::vector<int>* idx, std::vector<double>* w) {
    const int nf1 = 2 * nc * k + 1, nc1 = nc * k + 1;
    idx->assign((size_t)nf1 * (k + 1), 0);
    w->assign((size_t)nf1 * (k + 1), 0.0);
    for (int f = 0; f < nf1; ++f) {
        const int cellf = std::min(f / k, 2 * nc - 1);
        const int af = f - cellf * k;
        const double xf = (cellf + gll[af]) * 0.5;   // in coarse-cell units
        int c = (int)std::floor(xf);
        if (c > nc - 1) c = nc - 1;
        const double t = xf - c;
        for (int a = 0; a <= k; ++a) {
            const int ci = c * k + a;
            double v = lagrange_value(gll, a, t);
            if (f == 0 || f == nf1 - 1 || ci == 0 || ci == nc1 - 1) v = 0.0;
            if (std::fabs(v) < 1e-15) v = 0.0;
            (*idx)[f * (k + 1) + a] = ci;
            (*w)[f * (k + 1) + a] = v;
        }
    }
}

// Position classes of the patch inverses are used unless SGHEAT_PATCH_CLASSES=0 (a measurement switch:
// one inverse per cell even where they coincide).
bool patch_classes_disabled() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("SGHEAT_PATCH_CLASSES");
        v = (e && std::atoi(e) == 0) ? 1 : 0;
    }
    return v == 1;
}

// The mean block of a level with a constant mean coefficient is applied as a Kronecker sum of assembled
// 1D matrices unless SGHEAT_MEAN_STENCIL=0 (a measurement switch: the element route everywhere).
bool mean_stencil_disabled() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("SGHEAT_MEAN_STENCIL");
        v = (e && std::atoi(e) == 0) ? 1 : 0;
    }
    return v == 1;
}

// Levels with a constant mean coefficient compute their Vanka corrections by fast diagonalisation unless
// SGHEAT_VANKA_FDM=0 (a measurement switch: the dense position-class inverses instead).  Read at every
// smoothing call, so a process can compare both.
bool vanka_fdm_disabled() {
    const char* e = std::getenv("SGHEAT_VANKA_FDM");
    return e && std::strcmp(e, "0") == 0;     // ("lds" keeps it on and picks the kernel's LDS form)
}

// Generalised symmetric-definite eigenproblem A s = lambda B s of order m (row-major, B positive
// definite): S (column i = eigenvector i, S^T B S = I, S^T A S = diag(lambda)), by the Cholesky factor
// B = L L^T and cyclic Jacobi rotations of the symmetric C = L^{-1} A L^{-T} (Golub and Van Loan,
// Matrix Computations, the symmetric Schur decomposition of Section 8.5).  false if B is not positive
// definite.
bool sym_gen_eig(int m, const std::vector<double>& A, const std::vector<double>& B, std::vector<double>& S,
                 std::vector<double>& lam) {
    std::vector<double> L((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = B[(size_t)i * m + j];
            for (int q = 0; q < j; ++q) v -= L[(size_t)i * m + q] * L[(size_t)j * m + q];
            if (i == j) {
                if (!(v > 0.0)) return false;
                L[(size_t)i * m + i] = std::sqrt(v);
            } else {
                L[(size_t)i * m + j] = v / L[(size_t)j * m + j];
            }
        }
    // Y = L^{-1} A (forward substitution, column by column), C = L^{-1} Y^T (A symmetric: C = C^T)
    auto lsolve = [&](std::vector<double>& X) {   // X <- L^{-1} X, X row-major m x m
        for (int c = 0; c < m; ++c)
            for (int i = 0; i < m; ++i) {
                double v = X[(size_t)i * m + c];
                for (int q = 0; q < i; ++q) v -= L[(size_t)i * m + q] * X[(size_t)q * m + c];
                X[(size_t)i * m + c] = v / L[(size_t)i * m + i];
            }
    };
    std::vector<double> C(A);
    lsolve(C);
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) std::swap(C[(size_t)i * m + j], C[(size_t)j * m + i]);
    lsolve(C);
    for (int i = 0; i < m; ++i)                   // symmetrise the rounding
        for (int j = i + 1; j < m; ++j) {
            const double v = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
            C[(size_t)i * m + j] = C[(size_t)j * m + i] = v;
        }
    std::vector<double> V((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double v = C[(size_t)i * m + j] * C[(size_t)i * m + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = C[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double tau = (C[(size_t)q * m + q] - C[(size_t)p * m + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                for (int i = 0; i < m; ++i) {     // C <- C J
                    const double a = C[(size_t)i * m + p], b = C[(size_t)i * m + q];
                    C[(size_t)i * m + p] = c * a - sn * b;
                    C[(size_t)i * m + q] = sn * a + c * b;
                }
                for (int j = 0; j < m; ++j) {     // C <- J^T C
                    const double a = C[(size_t)p * m + j], b = C[(size_t)q * m + j];
                    C[(size_t)p * m + j] = c * a - sn * b;
                    C[(size_t)q * m + j] = sn * a + c * b;
                }
                for (int i = 0; i < m; ++i) {     // V <- V J
                    const double a = V[(size_t)i * m + p], b = V[(size_t)i * m + q];
                    V[(size_t)i * m + p] = c * a - sn * b;
                    V[(size_t)i * m + q] = sn * a + c * b;
                }
            }
    }
    lam.assign(m, 0.0);
    for (int i = 0; i < m; ++i) lam[i] = C[(size_t)i * m + i];
    // S = L^{-T} V (back substitution)
    S.assign((size_t)m * m, 0.0);
    for (int c = 0; c < m; ++c)
        for (int i = m - 1; i >= 0; --i) {
            double v = V[(size_t)i * m + c];
            for (int q = i + 1; q < m; ++q) v -= L[(size_t)q * m + i] * S[(size_t)q * m + c];
            S[(size_t)i * m + c] = v / L[(size_t)i * m + i];
        }
    return true;
}

// Tables of the fast-diagonalisation Vanka kernel for a level of n cells with constant mean
// coefficient: the assembled 1D bands (stiffness times the coefficient) restricted to the interior
// nodes of the first, an inner and the last cell, their generalised eigenvectors Sv[3][k+1][k+1]
// (zero rows for Dirichlet nodes) and the inverted time blocks Tt[3^d][(k+1)^d][N_t][N_t] of
// A_t + lambda_e B_t, lambda_e the sum of the 1D eigenvalues of eigen index e (zero blocks for unused
// indices).  false if a restricted mass matrix is not positive definite or a time block is singular.
bool fdm_tables(int dim, int n, int k, int NT, const std::vector<double>& At, const std::vector<double>& Bt,
                const std::vector<double>& mb, const std::vector<double>& kb, std::vector<double>& Sv,
                std::vector<double>& Tt) {
    const int N1 = k + 1, n1 = n * k + 1, W = 2 * k + 1;
    Sv.assign((size_t)3 * N1 * N1, 0.0);
    std::vector<double> lam((size_t)3 * N1, 0.0);
    int nint[3] = {0, 0, 0};
    for (int v = 0; v < 3; ++v) {
        const int pos = v == 0 ? 0 : (v == 1 ? std::min(1, n - 1) : n - 1);
        std::vector<int> in;
        for (int a = 0; a < N1; ++a) {
            const int gi = pos * k + a;
            if (gi != 0 && gi != n1 - 1) in.push_back(a);
        }
        const int m = (int)in.size();
        nint[v] = m;
        if (m == 0) continue;
        std::vector<double> M((size_t)m * m), Kr((size_t)m * m), S, l;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const int gi = pos * k + in[i], gj = pos * k + in[j];
                M[(size_t)i * m + j] = mb[(size_t)gi * W + (gj - gi + k)];
                Kr[(size_t)i * m + j] = kb[(size_t)gi * W + (gj - gi + k)];
            }
        if (!sym_gen_eig(m, Kr, M, S, l)) return false;
        for (int i = 0; i < m; ++i) {
            lam[(size_t)v * N1 + i] = l[i];
            for (int r = 0; r < m; ++r) Sv[((size_t)v * N1 + in[r]) * N1 + i] = S[(size_t)r * m + i];
        }
    }
    const int ncls = ipow_h(3, dim), NP = ipow_h(N1, dim);
    Tt.assign((size_t)ncls * NP * NT * NT, 0.0);
    for (int cls = 0; cls < ncls; ++cls)
        for (int e = 0; e < NP; ++e) {
            double lsum = 0.0;
            bool used = true;
            for (int d = 0, cr = cls, er = e; d < dim; ++d, cr /= 3, er /= N1) {
                used &= er % N1 < nint[cr % 3];
                lsum += lam[(size_t)(cr % 3) * N1 + er % N1];
            }
            if (!used) continue;
            // Gauss-Jordan with partial pivoting on [A_t + lambda B_t | I]
            std::vector<double> a((size_t)NT * 2 * NT, 0.0);
            for (int i = 0; i < NT; ++i) {
                for (int j = 0; j < NT; ++j) a[(size_t)i * 2 * NT + j] = At[(size_t)i * NT + j] + (i == j ? lsum * Bt[i] : 0.0);
                a[(size_t)i * 2 * NT + NT + i] = 1.0;
            }
            for (int c = 0; c < NT; ++c) {
                int piv = c;
                for (int i = c + 1; i < NT; ++i)
                    if (std::fabs(a[(size_t)i * 2 * NT + c]) > std::fabs(a[(size_t)piv * 2 * NT + c])) piv = i;
                if (a[(size_t)piv * 2 * NT + c] == 0.0) return false;
                for (int j = 0; j < 2 * NT; ++j) std::swap(a[(size_t)c * 2 * NT + j], a[(size_t)piv * 2 * NT + j]);
                const double ip = 1.0 / a[(size_t)c * 2 * NT + c];
                for (int j = 0; j < 2 * NT; ++j) a[(size_t)c * 2 * NT + j] *= ip;
                for (int i = 0; i < NT; ++i) {
                    if (i == c) continue;
                    const double f = a[(size_t)i * 2 * NT + c];
                    for (int j = 0; j < 2 * NT; ++j) a[(size_t)i * 2 * NT + j] -= f * a[(size_t)c * 2 * NT + j];
                }
            }
            for (int i = 0; i < NT; ++i)
                for (int j = 0; j < NT; ++j)
                    Tt[(((size_t)cls * NP + e) * NT + i) * NT + j] = a[(size_t)i * 2 * NT + NT + j];
        }
    return true;
}

// Assembled 1D mass and stiffness matrices of Q_k on n cells of width h, in band storage
// band[i][d] = M1[i][i - k + d] (zero beyond the mesh): the Gauss-quadrature integrals of the GLL
// basis on every cell, summed over the cells sharing a node.
void assemble_1d_bands(int n, int k, double h, const std::vector<double>& S, const std::vector<double>& Dn,
                       const std::vector<double>& gw, std::vector<double>& mb, std::vector<double>& kb) {
    const int N1 = k + 1, n1 = n * k + 1, W = 2 * k + 1;
    mb.assign((size_t)n1 * W, 0.0);
    kb.assign((size_t)n1 * W, 0.0);
    for (int c = 0; c < n; ++c)
        for (int a = 0; a < N1; ++a)
            for (int b = 0; b < N1; ++b) {
                double m = 0.0, st = 0.0;
                for (int q = 0; q < N1; ++q) {
                    m += gw[q] * S[q * N1 + a] * S[q * N1 + b];
                    st += gw[q] * Dn[q * N1 + a] * Dn[q * N1 + b];
                }
                const int i = c * k + a, j = c * k + b;
                mb[(size_t)i * W + (j - i + k)] += h * m;
                kb[(size_t)i * W + (j - i + k)] += st / h;
            }
}

// Everything that depends on the coefficient values: the pre-scaled coefficients of every level,
// the Vanka patch inverses and the coarsest-level inverse.  Called by sg_create and
// sg_update_coefficients; the device arrays keep their allocations between calls.
sg_status set_coefficients(sg_handle h, const double* coef_qp) {
    const sg_problem_desc& d = h->d;
    const int dim = d.dim, k = d.fe_degree, N1 = k + 1, L = d.n_levels;
    const std::vector<double>& S = h->tS;
    const std::vector<double>& Dn = h->tDn;
    const std::vector<double>& gw = h->tgw;
    const std::vector<double>& Me1 = h->Me1;
    if (d.n_samples > 0) {
        // every pathwise coefficient a(x, xi^(s)) = sum_mu Psi_mu(xi^(s)) a_mu(x) must be positive at the
        // finest level's Gauss points (the sample problems are then uniformly elliptic)
        const size_t per_mode = (size_t)h->lv[0].g.n_cells * h->NP;
        for (int smp = 0; smp < d.n_samples; ++smp) {
            const int* pp = h->cpl.ptr.data() + (size_t)smp * h->n_mu;
            for (size_t q = 0; q < per_mode; ++q) {
                double a = 0.0;
                for (int mi = 0; mi < h->n_mu; ++mi) a += h->cpl.w[pp[mi]] * coef_qp[(size_t)mi * per_mode + q];
                if (!(a > 0.0))
                    return fail(SG_EINVAL, "the coefficient of sample " + std::to_string(smp) +
                                               " is not positive at every Gauss point");
            }
        }
    }
    size_t coef_off = 0;
    std::vector<std::vector<double>> c64_levels(h->diag ? L : 0);   // host copies for the per-mode blocks
    for (int l = 0; l < L; ++l) {
        Level& lv = h->lv[l];
        // coefficients, pre-scaled by the Gauss weight and h^(d-2)
        const size_t per_mode = (size_t)lv.g.n_cells * h->NP;
        const bool all_modes = (l == 0) || h->diag;   // per-mode blocks need every mode on every level
        const int nm = all_modes ? h->n_mu : 1;
        std::vector<double> c64((size_t)nm * per_mode);
        const double hs = std::pow(lv.h, dim - 2);
        for (int mi = 0; mi < nm; ++mi) {
            const int mu = all_modes ? mi : h->cpl.mu0;
            const double* src = coef_qp + coef_off + (size_t)mu * per_mode;
            for (size_t c = 0; c < (size_t)lv.g.n_cells; ++c)
                for (int q = 0; q < h->NP; ++q) {
                    double wq = hs;
                    for (int dd = 0, qq = q; dd < dim; ++dd, qq /= N1) wq *= gw[qq % N1];
                    c64[mi * per_mode + c * h->NP + q] = src[c * h->NP + q] * wq;
                }
        }
        // a mean coefficient equal to one constant c at every Gauss point of the level: the mean block
        // is the Kronecker sum of the 1D matrices (stiffness scaled by c)
        {
            const double* s0 = coef_qp + coef_off + (size_t)h->cpl.mu0 * per_mode;
            bool cst = !h->diag;
            for (size_t q = 1; cst && q < per_mode; ++q) cst = s0[q] == s0[0];
            lv.mean_const = cst;
            if (cst) {
                std::vector<double> mb, kb;
                assemble_1d_bands(lv.g.n, k, lv.h, S, Dn, gw, mb, kb);
                for (double& v : kb) v *= s0[0];
                SG_TRY(lv.mb64.upload(mb.data(), mb.size(), "mean-block bands"));
                SG_TRY(lv.kb64.upload(kb.data(), kb.size(), "mean-block bands"));
                std::vector<double> fS, fT;
                if (!fdm_tables(dim, lv.g.n, k, h->NT, h->At, h->Bt, mb, kb, fS, fT))
                    return fail(SG_ESINGULAR, "a Vanka patch matrix is singular");
                SG_TRY(lv.fdmS64.upload(fS.data(), fS.size(), "Vanka transforms"));
                SG_TRY(lv.fdmT64.upload(fT.data(), fT.size(), "Vanka transforms"));
                if (h->mixed) {
                    std::vector<float> m32(mb.begin(), mb.end()), k32(kb.begin(), kb.end());
                    SG_TRY(lv.mb32.upload(m32.data(), m32.size(), "mean-block bands"));
                    SG_TRY(lv.kb32.upload(k32.data(), k32.size(), "mean-block bands"));
                    std::vector<float> s32(fS.begin(), fS.end()), t32(fT.begin(), fT.end());
                    SG_TRY(lv.fdmS32.upload(s32.data(), s32.size(), "Vanka transforms"));
                    SG_TRY(lv.fdmT32.upload(t32.data(), t32.size(), "Vanka transforms"));
                }
            }
        }
        coef_off += (size_t)h->n_mu * per_mode;
        if (h->diag) c64_levels[l] = c64;
        // With the mean coefficient identical in every cell (bitwise), the patch matrix of a cell depends
        // only on where the cell sits (first, inner or last along every direction): one inverse per
        // position class then serves every cell, bitwise what each cell's own inversion gives.
        {
            const double* m0 = c64.data() + (size_t)(all_modes ? h->cpl.mu0 : 0) * per_mode;
            bool same = !h->diag && !patch_classes_disabled();
            for (size_t c = 1; same && c < (size_t)lv.g.n_cells; ++c)
                for (int q = 0; q < h->NP; ++q)
                    if (m0[c * h->NP + q] != m0[q]) { same = false; break; }
            lv.inv_classes = same ? 1 : 0;
        }
        SG_TRY(lv.coef64.upload(c64.data(), c64.size(), "coefficients"));
        if (h->mixed) {
            std::vector<float> c32(c64.begin(), c64.end());
            SG_TRY(lv.coef32.upload(c32.data(), c32.size(), "coefficients"));
        }
    }

    // Vanka patch inverses on every level (device)
    {
        PatchTime pt{};
        for (int i = 0; i < h->NT; ++i) {
            pt.Bt[i] = h->Bt[i];
            for (int j = 0; j < h->NT; ++j) pt.At[i * h->NT + j] = h->At[i * h->NT + j];
        }
        ElemTables et{};
        for (int i = 0; i < N1 * N1; ++i) {
            et.S[i] = S[i];
            et.Dn[i] = Dn[i];
        }
        DevBuf<int> status;
        int zero = 0;
        SG_TRY(status.upload(&zero, 1, "status"));
        for (int l = 0; l < L; ++l) {
            Level& lv = h->lv[l];
            DevBuf<double>& E = h->elem_E;
            DevBuf<double>& Me = h->elem_M;
            if (E.n < (size_t)lv.g.n_cells * h->NP * h->NP)
                SG_TRY(E.alloc((size_t)lv.g.n_cells * h->NP * h->NP, "element matrices"));
            std::vector<double> Mel(Me1);
            const double vol = std::pow(lv.h, dim);
            for (double& v : Mel) v *= vol;
            SG_TRY(Me.upload(Mel.data(), Mel.size(), "element matrices"));
            // inverses in the fragment layout of the patch products (zero in the padding columns); one per
            // cell, or one per position class (a representative cell of each is inverted)
            int nclass = 1;
            for (int dd = 0; dd < dim; ++dd) nclass *= 3;
            if (lv.inv_classes) {
                std::vector<int> rep(nclass);
                for (int c = 0; c < nclass; ++c) {
                    long long cell = 0, m = 1;
                    for (int dd = 0, cr = c; dd < dim; ++dd, cr /= 3) {
                        const int pos = cr % 3 == 0 ? 0 : (cr % 3 == 2 ? lv.g.n - 1 : std::min(1, lv.g.n - 1));
                        cell += m * pos;
                        m *= lv.g.n;
                    }
                    rep[c] = (int)cell;
                }
                SG_TRY(lv.class_cells.upload(rep.data(), rep.size(), "patch classes"));
            }
            const size_t nslot = lv.inv_classes ? (size_t)nclass : (size_t)lv.g.n_cells;
            const size_t ninv = nslot * vanka_inv_stride(h->npp);
            const bool want32 = h->mixed && l < L - 1;
            const int nblk = h->diag ? h->n_xi : 1;             // one set of patch inverses per mode
            SG_TRY(lv.inv64.alloc(ninv * nblk, "patch inverses"));
            if (want32) SG_TRY(lv.inv32.alloc(ninv * nblk, "patch inverses"));
            SG_HIP(launch_fill<double>(lv.inv64.p, 0.0, (long long)(ninv * nblk), nullptr));
            if (want32) SG_HIP(launch_fill<float>(lv.inv32.p, 0.0f, (long long)(ninv * nblk), nullptr));
            const size_t per_mode = (size_t)lv.g.n_cells * h->NP;
            std::vector<double> acomb(h->diag ? per_mode : 0);
            for (int a = 0; a < nblk; ++a) {
                const double* c0 = lv.coef64.p + ((l == 0 || h->diag) ? (size_t)h->cpl.mu0 * per_mode : 0);
                if (h->diag) {
                    // a_alpha = sum_mu [G_mu]_{alpha alpha} a_mu at this level's Gauss points (pre-scaled)
                    std::fill(acomb.begin(), acomb.end(), 0.0);
                    for (int mi = 0; mi < h->n_mu; ++mi) {
                        const double wv = h->dw[(size_t)a * h->n_mu + mi];
                        if (wv == 0.0) continue;
                        const double* src = c64_levels[l].data() + (size_t)mi * per_mode;
                        for (size_t q = 0; q < per_mode; ++q) acomb[q] += wv * src[q];
                    }
                    SG_TRY(h->acomb.upload(acomb.data(), acomb.size(), "block coefficient"));
                    c0 = h->acomb.p;
                }
                SG_HIP(launch_elem_stiffness(dim, k, lv.g, c0, et, E.p, nullptr));
                if (h->seg_level >= 0 && l >= h->seg_level) {
                    // the coarse segment applies A_0 from the element matrices of these levels
                    const size_t ne = (size_t)lv.g.n_cells * h->NP * h->NP;
                    SG_TRY(lv.E64.alloc(ne, "segment element matrices"));
                    SG_HIP(hipMemcpy(lv.E64.p, E.p, ne * sizeof(double), hipMemcpyDeviceToDevice));
                    SG_TRY(lv.Me64.upload(Mel.data(), Mel.size(), "segment element matrices"));
                }
                SG_HIP(launch_patch_invert(dim, k, h->NT, lv.g, E.p, Me.p, pt, lv.inv64.p + a * ninv,
                                           want32 ? lv.inv32.p + a * ninv : nullptr, status.p, nullptr,
                                           lv.inv_classes ? lv.class_cells.p : nullptr, (int)nslot));
                SG_HIP(hipStreamSynchronize(nullptr));   // set-up runs on the null stream
            }
        }
        int st = 0;
        SG_HIP(hipMemcpy(&st, status.p, sizeof(int), hipMemcpyDeviceToHost));
        if (st) return fail(SG_ESINGULAR, "a Vanka patch matrix is singular");
    }

    // coarsest level: dense A_0 on interior DoFs, assembled on the host and inverted on the device
    // (Gauss-Jordan elimination with partial pivoting, FP64)
    {
        const Level& lc = h->lv[L - 1];
        const int n = lc.g.n, n1 = lc.g.n1;
        std::vector<int> interior_node(lc.g.n_nodes, -1);
        std::vector<int> inodes;
        for (long long node = 0; node < lc.g.n_nodes; ++node) {
            bool bnd = false;
            long long r = node;
            for (int dd = 0; dd < dim; ++dd) {
                const int id = r % n1;
                r /= n1;
                bnd |= (id == 0 || id == n1 - 1);
            }
            if (!bnd) {
                interior_node[node] = (int)inodes.size();
                inodes.push_back((int)node);
            }
        }
        const int ni = (int)inodes.size();
        h->nint = ni * h->NT;
        if (h->nint > 12000) return fail(SG_EINVAL, "coarsest level too large for the dense solve; add levels");
        const int nblk = h->diag ? h->n_xi : 1;                   // one coarsest inverse per mode
        if (h->diag && (double)nblk * h->nint * h->nint * 8.0 > 16e9)
            return fail(SG_EUNSUPPORTED, "per-mode coarsest-level inverses need more than 16 GB; add levels");
        size_t off = 0;
        for (int l = 0; l < L - 1; ++l) off += (size_t)h->n_mu * h->lv[l].g.n_cells * h->NP;
        const size_t cper = (size_t)lc.g.n_cells * h->NP;
        std::vector<double> craw(h->diag ? cper : 0);
        if (h->nint > 0) SG_TRY(h->coarse_invT.alloc((size_t)nblk * h->nint * h->nint, "coarse inverse"));
        for (int blk = 0; blk < nblk; ++blk) {
            std::vector<double> A((size_t)h->nint * h->nint, 0.0);
            const double* c0 = coef_qp + off + (size_t)h->cpl.mu0 * cper;
            if (h->diag) {
                std::fill(craw.begin(), craw.end(), 0.0);
                for (int mi = 0; mi < h->n_mu; ++mi) {
                    const double wv = h->dw[(size_t)blk * h->n_mu + mi];
                    if (wv == 0.0) continue;
                    const double* src = coef_qp + off + (size_t)mi * cper;
                    for (size_t q = 0; q < cper; ++q) craw[q] += wv * src[q];
                }
                c0 = craw.data();
            }
            const double vol = std::pow(lc.h, dim), hs = std::pow(lc.h, dim - 2);
            // reference stiffness integrands Kref[q][a][b] = w_q h^(d-2) sum_e dphi_a/dx_e dphi_b/dx_e (x_q)
            const int NP = h->NP;
            std::vector<double> Kref((size_t)NP * NP * NP);
            for (int q = 0; q < NP; ++q) {
                double wq = hs;
                for (int dd = 0, qq = q; dd < dim; ++dd, qq /= N1) wq *= gw[qq % N1];
                for (int a = 0; a < NP; ++a)
                    for (int b = 0; b < NP; ++b) {
                        double gsum = 0.0;
                        for (int e = 0; e < dim; ++e) {
                            double va = 1.0, vb = 1.0;
                            for (int dd = 0, qq = q, aa = a, bb = b; dd < dim; ++dd, qq /= N1, aa /= N1, bb /= N1) {
                                va *= (dd == e ? Dn : S)[(qq % N1) * N1 + aa % N1];
                                vb *= (dd == e ? Dn : S)[(qq % N1) * N1 + bb % N1];
                            }
                            gsum += va * vb;
                        }
                        Kref[((size_t)q * NP + a) * NP + b] = wq * gsum;
                    }
            }
            std::vector<double> Ke((size_t)NP * NP);
            for (long long cell = 0; cell < lc.g.n_cells; ++cell) {
                int cc[3] = {0, 0, 0};
                long long r = cell;
                for (int dd = 0; dd < dim; ++dd) { cc[dd] = r % n; r /= n; }
                std::vector<int> nodes(NP);
                for (int a = 0; a < NP; ++a) {
                    long long node = 0, mul = 1;
                    for (int dd = 0, aa = a; dd < dim; ++dd, aa /= N1) { node += (cc[dd] * k + aa % N1) * mul; mul *= n1; }
                    nodes[a] = interior_node[node];
                }
                std::fill(Ke.begin(), Ke.end(), 0.0);
                for (int q = 0; q < NP; ++q) {
                    const double cq = c0[cell * NP + q];
                    const double* kr = &Kref[(size_t)q * NP * NP];
                    for (size_t ab = 0; ab < (size_t)NP * NP; ++ab) Ke[ab] += cq * kr[ab];
                }
                for (int a = 0; a < h->NP; ++a) {
                    if (nodes[a] < 0) continue;
                    for (int b = 0; b < h->NP; ++b) {
                        if (nodes[b] < 0) continue;
                        const double m = Me1[(size_t)a * h->NP + b] * vol, kv = Ke[(size_t)a * h->NP + b];
                        for (int i = 0; i < h->NT; ++i)
                            for (int j = 0; j < h->NT; ++j) {
                                const size_t row = (size_t)i * ni + nodes[a], col = (size_t)j * ni + nodes[b];
                                A[row * h->nint + col] += h->At[i * h->NT + j] * m + (i == j ? h->Bt[i] * kv : 0.0);
                            }
                    }
                }
            }
            // Gauss-Jordan inverse on the device (the matrix is a few thousand rows at most)
            if (h->nint > 0) {
                DevBuf<double> Ad, col;
                DevBuf<int> perm, status;
                int zero = 0;
                SG_TRY(Ad.upload(A.data(), A.size(), "coarse matrix"));
                SG_TRY(col.alloc(h->nint, "coarse pivots"));
                SG_TRY(perm.alloc(h->nint, "coarse pivots"));
                SG_TRY(status.upload(&zero, 1, "status"));
                SG_HIP(launch_dense_invert(Ad.p, h->nint, col.p, perm.p, status.p,
                                           h->coarse_invT.p + (size_t)blk * h->nint * h->nint, nullptr));
                int st = 0;
                SG_HIP(hipMemcpy(&st, status.p, sizeof(int), hipMemcpyDeviceToHost));
                if (st) return fail(SG_ESINGULAR, "coarsest-level matrix is singular");
            }
        }
        std::vector<int> dofs(h->nint);
        for (int i = 0; i < h->NT; ++i)
            for (int a = 0; a < ni; ++a) dofs[i * ni + a] = i * (int)lc.g.n_nodes + inodes[a];
        SG_TRY(h->coarse_dofs.upload(dofs.data(), dofs.size(), "coarse dofs"));
    }

    return SG_OK;
}

sg_status build(sg_handle h) {
    const sg_problem_desc& d = h->d;
    const int dim = d.dim, k = d.fe_degree, N1 = k + 1;
    h->NP = ipow_h(N1, dim);
    h->NT = d.time_degree + 1;
    h->mixed = d.precision == SG_MIXED;
    std::string err;
    bool ok;
    if (d.n_samples > 0) {
        ok = build_sample_coupling(d.n_vars, d.n_samples, h->samples.data(), d.n_coef_modes, h->coef_mu.data(),
                                   &h->cpl, &err);
    } else if (d.n_members > 0) {
        ok = build_batch_coupling(d.n_vars, d.n_members, h->member_degree.data(), h->member_scale.data(),
                                  d.n_coef_modes, h->coef_mu.data(), &h->cpl, &h->member_off, &err);
    } else {
        ok = build_coupling(d.n_vars, d.chaos_degree, d.n_coef_modes, h->coef_mu.data(), &h->cpl, &err);
        h->member_off = {0, h->cpl.n_xi};
    }
    if (!ok) return fail(SG_EINVAL, err);
    if (d.n_samples == 0) SG_TRY(h->moff.upload(h->member_off.data(), h->member_off.size(), "member offsets"));
    h->n_xi = h->cpl.n_xi;
    h->n_mu = d.n_coef_modes;
    h->npp = h->NT * h->NP;
    // one thread per (cell, component) in the operator kernel: up to 512 threads per workgroup (256 for
    // more than 27 points per cell), or one cell per workgroup of up to 1024 threads in 2D
    const int nc = h->n_xi * h->NT;
    const int maxt = h->NP > 27 ? 256 : 512;
    const bool wide = nc > maxt;
    if (nc > (dim == 2 ? 1024 : maxt))
        return fail(SG_EUNSUPPORTED, dim == 2 ? "N_xi * N_t must be <= 1024 in 2D"
                                              : (maxt == 512 ? "N_xi * N_t must be <= 512 in 3D for k <= 2"
                                                             : "N_xi * N_t must be <= 256 in 3D for k >= 3"));
    if (h->npp > 256) return fail(SG_EUNSUPPORTED, "Vanka patches larger than 256 DoFs are not supported");
    {
        const size_t n_ent_max = wide ? 1 : h->cpl.beta.size();   // wide workgroups read the entries from memory
        const size_t lds_apply = (size_t)(h->n_xi * h->NT + h->n_mu) * h->NP * sizeof(double) + n_ent_max * 16;
        const size_t lds_vanka = vanka_lds_bytes(h->npp, sizeof(double));
        if (lds_apply > 160 * 1024 || lds_vanka > 160 * 1024)
            return fail(SG_EUNSUPPORTED, "problem too large for one workgroup's LDS (N_xi * N_t * (k+1)^d)");
    }
    if (!time_matrices(d.time_degree, d.tau, &h->At, &h->Bt))
        return fail(SG_EINVAL, "time matrices: B_t is not diagonal");
    if (d.transpose) {   // adjoint slab operator: A_t^T (every other factor is symmetric)
        const std::vector<double> a = h->At;
        for (int i = 0; i < h->NT; ++i)
            for (int j = 0; j < h->NT; ++j) h->At[i * h->NT + j] = a[j * h->NT + i];
    }
    {
        const std::vector<double> tn = right_radau_points(d.time_degree);
        h->radau0.resize(h->NT);
        for (int i = 0; i < h->NT; ++i) h->radau0[i] = lagrange_value(tn, i, 0.0);
    }

    // coupling lists (full operator and mean block)
    {
        std::vector<int> cmu_h(h->cpl.beta.size());
        for (int row = 0; row < h->n_xi * h->n_mu; ++row)
            for (int e = h->cpl.ptr[row]; e < h->cpl.ptr[row + 1]; ++e) cmu_h[e] = row % h->n_mu;
        std::vector<float> w32(h->cpl.w.begin(), h->cpl.w.end());
        SG_TRY(h->cptr.upload(h->cpl.ptr.data(), h->cpl.ptr.size(), "coupling"));
        SG_TRY(h->cbeta.upload(h->cpl.beta.data(), h->cpl.beta.size(), "coupling"));
        SG_TRY(h->cmu.upload(cmu_h.data(), cmu_h.size(), "coupling"));
        SG_TRY(h->cw64.upload(h->cpl.w.data(), h->cpl.w.size(), "coupling"));
        SG_TRY(h->cw32.upload(w32.data(), w32.size(), "coupling"));
        std::vector<int> pm(h->n_xi + 1), bm(h->n_xi), mm(h->n_xi, 0);
        std::vector<double> wm(h->n_xi, 1.0);
        std::vector<float> wm32(h->n_xi, 1.0f);
        for (int a = 0; a <= h->n_xi; ++a) pm[a] = a;
        for (int a = 0; a < h->n_xi; ++a) bm[a] = a;
        SG_TRY(h->cptr_m.upload(pm.data(), pm.size(), "coupling"));
        SG_TRY(h->cbeta_m.upload(bm.data(), bm.size(), "coupling"));
        SG_TRY(h->cmu_m.upload(mm.data(), mm.size(), "coupling"));
        SG_TRY(h->cw_m64.upload(wm.data(), wm.size(), "coupling"));
        SG_TRY(h->cw_m32.upload(wm32.data(), wm32.size(), "coupling"));
        h->diag = d.diag_blocks == 1;
        if (h->diag) {
            // the (alpha, alpha) entry of every (alpha, mu) row: the diagonal block's coefficient weights
            h->dw.assign((size_t)h->n_xi * h->n_mu, 0.0);
            std::vector<int> pd(1, 0), bd, md;
            std::vector<double> wd;
            for (int a = 0; a < h->n_xi; ++a)
                for (int mi = 0; mi < h->n_mu; ++mi) {
                    const int row = a * h->n_mu + mi;
                    for (int e = h->cpl.ptr[row]; e < h->cpl.ptr[row + 1]; ++e)
                        if (h->cpl.beta[e] == a) h->dw[(size_t)a * h->n_mu + mi] += h->cpl.w[e];
                    const double wv = h->dw[(size_t)a * h->n_mu + mi];
                    if (wv != 0.0) {
                        bd.push_back(a);
                        md.push_back(mi);
                        wd.push_back(wv);
                    }
                    pd.push_back((int)bd.size());
                }
            h->n_ent_d = (int)bd.size();
            std::vector<float> wd32(wd.begin(), wd.end());
            SG_TRY(h->cptr_d.upload(pd.data(), pd.size(), "diagonal coupling"));
            SG_TRY(h->cbeta_d.upload(bd.data(), bd.size(), "diagonal coupling"));
            SG_TRY(h->cmu_d.upload(md.data(), md.size(), "diagonal coupling"));
            SG_TRY(h->cw_d64.upload(wd.data(), wd.size(), "diagonal coupling"));
            SG_TRY(h->cw_d32.upload(wd32.data(), wd32.size(), "diagonal coupling"));
        }
    }

    // 1D tables
    std::vector<double> gw;
    const std::vector<double> gq = gauss_points(N1, &gw);
    const std::vector<double> gll = gll_points(k);
    std::vector<double> S(N1 * N1), D(N1 * N1), Dn(N1 * N1);
    for (int q = 0; q < N1; ++q)
        for (int a = 0; a < N1; ++a) {
            S[q * N1 + a] = lagrange_value(gll, a, gq[q]);
            D[q * N1 + a] = lagrange_deriv(gq, a, gq[q]);
            Dn[q * N1 + a] = lagrange_deriv(gll, a, gq[q]);
        }

    h->tS = S;
    h->tD = D;
    h->tDn = Dn;
    h->tgw = gw;

    // levels
    const int L = d.n_levels;
    h->lv.resize(L);
    for (int l = 0; l < L; ++l) {
        Level& lv = h->lv[l];
        const int n = d.n_cells_1d >> l;
        lv.g.n = n;
        lv.g.n1 = n * k + 1;
        lv.g.n_nodes = 1;
        lv.g.n_cells = 1;
        for (int i = 0; i < dim; ++i) {
            lv.g.n_nodes *= lv.g.n1;
            lv.g.n_cells *= n;
        }
        lv.h = (d.hi - d.lo) / n;
        lv.len = (long long)h->n_xi * h->NT * lv.g.n_nodes;
        fill_tables(&lv.tab64, S, D, gw, h->At, h->Bt, N1, h->NT, std::pow(lv.h, dim));
        fill_tables(&lv.tab32, S, D, gw, h->At, h->Bt, N1, h->NT, std::pow(lv.h, dim));
        if (l == 0) {
            std::vector<double> at(h->NT * h->NT);
            for (int i = 0; i < h->NT; ++i)
                for (int j = 0; j < h->NT; ++j) at[i * h->NT + j] = h->At[j * h->NT + i];
            fill_tables(&h->tabT64, S, D, gw, at, h->Bt, N1, h->NT, std::pow(lv.h, dim));
        }
        // work vectors
        SG_TRY(lv.b64.alloc(lv.len, "level vectors"));
        SG_TRY(lv.x64.alloc(lv.len, "level vectors"));
        SG_TRY(lv.r64.alloc(lv.len, "level vectors"));
        if (h->mixed) {
            SG_TRY(lv.b32.alloc(lv.len, "level vectors"));
            SG_TRY(lv.x32.alloc(lv.len, "level vectors"));
            SG_TRY(lv.r32.alloc(lv.len, "level vectors"));
        }
    }
    h->N = h->lv[0].len;

    // element mass matrix (identical on every cell of a level up to h^d)
    std::vector<double> Me1((size_t)h->NP * h->NP);
    for (int a = 0; a < h->NP; ++a)
        for (int b = 0; b < h->NP; ++b) {
            double s = 0.0;
            for (int q = 0; q < h->NP; ++q) {
                double v = 1.0;
                for (int dd = 0, qq = q, aa = a, bb = b; dd < dim; ++dd, qq /= N1, aa /= N1, bb /= N1)
                    v *= gw[qq % N1] * S[(qq % N1) * N1 + aa % N1] * S[(qq % N1) * N1 + bb % N1];
                s += v;
            }
            Me1[(size_t)a * h->NP + b] = s;
        }

    h->Me1 = Me1;
    // The coarse segment (levels from the first one of at most 512 cells, below the finest, down to the
    // coarsest) runs as one launch when its per-mode scratch fits the cell-local buffer.
    h->seg_level = -1;
    if (!h->diag) {
        for (int l = 1; l + 1 < L; ++l) {
            if (h->lv[l].g.n_cells > 512) continue;
            if (L - l > kSegMaxLevels) break;
            const long long nf = h->lv[l].g.n1, nc = h->lv[l + 1].g.n1;
            const long long tmp = (long long)h->NT * (dim == 3 ? nf * nf * nc : nf * nc);
            const long long need = (long long)h->n_xi * segment_scratch_per_mode(h->NT, h->NP, h->lv[l].g.n_cells, tmp);
            const long long have = (long long)h->n_xi * h->NT * h->lv[0].g.n_cells * h->NP;   // doubles
            if (need <= have) h->seg_level = l;
            break;
        }
    }
    // kernel by kernel until sg_set_vcycle_segment or sg_autotune (which times both) says otherwise
    h->seg_on = false;
    SG_TRY(set_coefficients(h, d.coef_qp));

    // transfer stencils and temporaries
    size_t tmax = 0;
    for (int l = 0; l + 1 < L; ++l) {
        Level& lf = h->lv[l];
        const int nc = h->lv[l + 1].g.n, nc1 = h->lv[l + 1].g.n1, nf1 = lf.g.n1;
        std::vector<int> pidx;
        std::vector<double> pw;
        prolong_1d(nc, k, gll, &pidx, &pw);
        lf.wp = k + 1;
        // transpose: for each coarse node the fine nodes with a nonzero weight
        std::vector<std::vector<std::pair<int, double>>> cols(nc1);
        for (int f = 0; f < nf1; ++f)
            for (int a = 0; a <= k; ++a) {
                const double v = pw[f * (k + 1) + a];
                if (v != 0.0) cols[pidx[f * (k + 1) + a]].push_back({f, v});
            }
        int wr = 1;
        for (auto& c : cols) wr = std::max<int>(wr, (int)c.size());
        lf.wr = wr;
        std::vector<int> ridx((size_t)nc1 * wr, 0);
        std::vector<double> rw((size_t)nc1 * wr, 0.0);
        for (int c = 0; c < nc1; ++c)
            for (size_t e = 0; e < cols[c].size(); ++e) {
                ridx[c * wr + e] = cols[c][e].first;
                rw[c * wr + e] = cols[c][e].second;
            }
        SG_TRY(lf.p_idx.upload(pidx.data(), pidx.size(), "transfer"));
        SG_TRY(lf.p_w64.upload(pw.data(), pw.size(), "transfer"));
        SG_TRY(lf.r_idx.upload(ridx.data(), ridx.size(), "transfer"));
        SG_TRY(lf.r_w64.upload(rw.data(), rw.size(), "transfer"));
        std::vector<float> pw32(pw.begin(), pw.end()), rw32(rw.begin(), rw.end());
        SG_TRY(lf.p_w32.upload(pw32.data(), pw32.size(), "transfer"));
        SG_TRY(lf.r_w32.upload(rw32.data(), rw32.size(), "transfer"));
        size_t inter = (size_t)h->n_xi * h->NT * nf1 * (size_t)(dim == 3 ? (size_t)nf1 * nc1 : nc1);
        tmax = std::max(tmax, inter);
    }
    if (tmax) {
        SG_TRY(h->t64a.alloc(tmax, "transfer temporaries"));
        SG_TRY(h->t64b.alloc(tmax, "transfer temporaries"));
        if (h->mixed) {
            SG_TRY(h->t32a.alloc(tmax, "transfer temporaries"));
            SG_TRY(h->t32b.alloc(tmax, "transfer temporaries"));
        }
    }
    // Krylov workspace
    h->restart = d.fgmres_restart;
    SG_TRY(h->V.alloc((size_t)(h->restart + 1) * h->N, "Krylov basis"));
    SG_TRY(h->Z.alloc((size_t)h->restart * h->N, "Krylov basis"));
    SG_TRY(h->w1.alloc(h->N, "Krylov work"));
    SG_TRY(h->w2.alloc(h->N, "Krylov work"));
    SG_TRY(h->partial.alloc((size_t)kDotBlocks * (2 * h->restart + 2), "partials"));
    SG_TRY(h->dscal.alloc(3 * 80, "scalars"));
    SG_TRY(h->sbuf.alloc((size_t)h->n_xi * h->NT * h->lv[0].g.n_cells * h->NP, "cell-local results"));
    SG_HIP(hipStreamSynchronize(nullptr));
    return SG_OK;
}

// ---- operator helpers -------------------------------------------------------------------------------
template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static const Tables<double>* tab(const Level& l) { return &l.tab64; }
    static const double* coef(const Level& l) { return l.coef64.p; }
    static const double* cw(const sg_handle h) { return h->cw64.p; }
    static const double* cwm(const sg_handle h) { return h->cw_m64.p; }
    static const double* cwd(const sg_handle h) { return h->cw_d64.p; }
    static const double* inv(const Level& l) { return l.inv64.p; }
    static const double* fdmS(const Level& l) { return l.fdmS64.p; }
    static const double* fdmT(const Level& l) { return l.fdmT64.p; }
    static double* b(Level& l) { return l.b64.p; }
    static double* x(Level& l) { return l.x64.p; }
    static double* r(Level& l) { return l.r64.p; }
    static double* ta(sg_handle h) { return h->t64a.p; }
    static double* tb(sg_handle h) { return h->t64b.p; }
    static const double* pw(const Level& l) { return l.p_w64.p; }
    static const double* rw(const Level& l) { return l.r_w64.p; }
};
template <>
struct Prec<float> {
    static const Tables<float>* tab(const Level& l) { return &l.tab32; }
    static const float* coef(const Level& l) { return l.coef32.p; }
    static const float* cw(const sg_handle h) { return h->cw32.p; }
    static const float* cwm(const sg_handle h) { return h->cw_m32.p; }
    static const float* cwd(const sg_handle h) { return h->cw_d32.p; }
    static const float* inv(const Level& l) { return l.inv32.p; }
    static const float* fdmS(const Level& l) { return l.fdmS32.p; }
    static const float* fdmT(const Level& l) { return l.fdmT32.p; }
    static float* b(Level& l) { return l.b32.p; }
    static float* x(Level& l) { return l.x32.p; }
    static float* r(Level& l) { return l.r32.p; }
    static float* ta(sg_handle h) { return h->t32a.p; }
    static float* tb(sg_handle h) { return h->t32b.p; }
    static const float* pw(const Level& l) { return l.p_w32.p; }
    static const float* rw(const Level& l) { return l.r_w32.p; }
};

// Cells per workgroup of the apply kernel: chosen from the kernel's occupancy unless the
// SGHEAT_APPLY_CPB environment variable fixes it (a tuning override).
int apply_cpb_override() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("SGHEAT_APPLY_CPB");
        v = e ? std::max(0, std::atoi(e)) : 0;
    }
    return v;
}

// Cells per z chunk of the marching 3D apply kernel: chosen from the mesh size unless the
// SGHEAT_APPLY_LZ environment variable fixes it (a tuning override).
int apply_lz_override() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("SGHEAT_APPLY_LZ");
        v = e ? std::max(0, std::atoi(e)) : 0;
    }
    return v;
}

template <typename T>
ApplyOp<T> make_op(const sg_handle h, int level, bool full) {
    const Level& lv = h->lv[level];
    ApplyOp<T> op{};
    op.dim = h->d.dim;
    op.k = h->d.fe_degree;
    op.nt = h->NT;
    op.g = lv.g;
    op.n_xi = h->n_xi;
    op.coef_mode_stride = lv.g.n_cells * h->NP;
    op.tables = Prec<T>::tab(lv);
    if (full) {
        op.n_mu = h->n_mu;
        op.coef = Prec<T>::coef(lv);
        op.cptr = h->cptr.p;
        op.cbeta = h->cbeta.p;
        op.cmu = h->cmu.p;
        op.cw = Prec<T>::cw(h);
    } else {
        op.n_mu = 1;
        op.coef = Prec<T>::coef(lv) + ((level == 0 || h->diag) ? (size_t)h->cpl.mu0 * op.coef_mode_stride : 0);
        op.cptr = h->cptr_m.p;
        op.cbeta = h->cbeta_m.p;
        op.cmu = h->cmu_m.p;
        op.cw = Prec<T>::cwm(h);
    }
    op.mean = !full;
    op.level = level;
    op.n_ent = full ? (int)h->cpl.beta.size() : h->n_xi;
    // compile-time Hermite tables describe a single total-degree problem only
    op.affine = h->cpl.affine && h->d.n_vars <= 8 && h->d.n_samples == 0 && h->d.n_members == 0;
    op.chaos_m = h->d.n_vars;
    op.chaos_p = h->d.chaos_degree;
    op.mu0 = h->cpl.mu0;
    for (int m = 0; m < 8; ++m) op.mum[m] = -1;
    for (int k = 0; k < h->n_mu; ++k) {
        int nz = -1, cnt = 0;
        for (int m = 0; m < h->d.n_vars; ++m)
            if (h->coef_mu[k * h->d.n_vars + m] != 0) { nz = m; ++cnt; }
        if (cnt == 1 && nz < 8 && h->coef_mu[k * h->d.n_vars + nz] == 1) op.mum[nz] = k;
    }
    op.cells_per_block = apply_cpb_override();
    if (op.cells_per_block == 0 && level < 16) op.cells_per_block = h->tuned_cpb[sizeof(T) == 4][full][level];
    op.merge = 1;
    op.used_cpb = nullptr;
    op.lz = apply_lz_override();
    op.used_lz = nullptr;
    return op;
}

// The operator of the preconditioner's diagonal blocks on one level: the mean block I (x) A_0, or with
// per-mode blocks the block-diagonal operator diag_alpha(A_alpha) (the (alpha, alpha) coupling entries).
template <typename T>
ApplyOp<T> make_block_op(const sg_handle h, int level) {
    if (!h->diag) return make_op<T>(h, level, false);
    ApplyOp<T> op = make_op<T>(h, level, true);
    op.cptr = h->cptr_d.p;
    op.cbeta = h->cbeta_d.p;
    op.cmu = h->cmu_d.p;
    op.cw = Prec<T>::cwd(h);
    op.n_ent = h->n_ent_d;
    op.affine = false;
    op.cells_per_block = apply_cpb_override();
    if (op.cells_per_block == 0 && level < 16) op.cells_per_block = h->tuned_cpb[sizeof(T) == 4][0][level];
    return op;
}

template <typename T>
T* sbuf_as(sg_handle h) {
    return reinterpret_cast<T*>(h->sbuf.p);
}

sg_status vcycle_fixed(sg_handle h, hipStream_t s);

// Time the operator (cell kernel + gather) for every feasible cells-per-workgroup value on one level
// and keep the fastest (median of `reps` event-timed launches each).
template <typename T>
sg_status autotune_apply(sg_handle h, int level, bool full, int reps, hipStream_t s) {
    Level& lv = h->lv[level];
    ApplyOp<T> op = full ? make_op<T>(h, level, true) : make_block_op<T>(h, level);
    T* x = Prec<T>::x(lv);
    SG_HIP(hipMemsetAsync(x, 0, sizeof(T) * lv.len, s));
    std::vector<hipEvent_t> ev(reps + 1);
    for (auto& e : ev) SG_HIP(hipEventCreate(&e));
    int best = 0;
    float best_ms = 0.0f;
    sg_status st = SG_OK;
    static const int kCand[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    for (int cpb : kCand) {
        if (cpb > lv.g.n) break;
        op.cells_per_block = cpb;
        // the cell kernel and its gather together (the merged layout's gain is in the gather)
        int used = 1, used_lz = 1;
        op.used_cpb = &used;
        op.used_lz = &used_lz;
        hipError_t err = launch_apply<T>(op, x, sbuf_as<T>(h), s);
        if (err == hipErrorInvalidConfiguration) continue;     // more threads or LDS than one workgroup has
        if (err != hipSuccess) { st = fail(SG_EHIP, std::string("autotune: ") + hipGetErrorString(err)); break; }
        const int sx = apply_segment(op, used), sz = apply_zsegment(op, used_lz);
        auto once = [&]() {
            (void)launch_apply<T>(op, x, sbuf_as<T>(h), s);
            (void)launch_node_gather<T>(GATHER_SET, op.dim, op.k, op.g, h->n_xi * h->NT, sbuf_as<T>(h), x, nullptr,
                                        Prec<T>::r(lv), T(0), sx, sz, s);
        };
        once();
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps; ++r) {
            once();
            (void)hipEventRecord(ev[r + 1], s);
        }
        if (hipEventSynchronize(ev[reps]) != hipSuccess) { st = fail(SG_EHIP, "autotune: event"); break; }
        std::vector<float> t(reps);
        for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], ev[r], ev[r + 1]);
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        const float med = t[reps / 2];
        if (best == 0 || med < best_ms) { best = cpb; best_ms = med; }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (st == SG_OK && level < 16) h->tuned_cpb[sizeof(T) == 4][full][level] = best;
    return st;
}

// Time `reps` V-cycles on the level-0 work vectors with the coarse segment as one launch and kernel by
// kernel (median of each) and keep the faster.
sg_status autotune_segment(sg_handle h, int reps, hipStream_t s) {
    if (h->seg_level < 0) return SG_OK;
    Level& l0 = h->lv[0];
    if (h->mixed) SG_HIP(launch_fill<float>(l0.b32.p, 0.0f, l0.len, s));
    else SG_HIP(launch_fill<double>(l0.b64.p, 0.0, l0.len, s));
    std::vector<hipEvent_t> ev(reps + 1);
    for (auto& e : ev) SG_HIP(hipEventCreate(&e));
    float med[2] = {0.0f, 0.0f};
    sg_status st = SG_OK;
    for (int on = 0; on < 2 && st == SG_OK; ++on) {
        h->seg_on = on == 1;
        st = vcycle_fixed(h, s);
        if (st != SG_OK) break;
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps && st == SG_OK; ++r) {
            st = vcycle_fixed(h, s);
            (void)hipEventRecord(ev[r + 1], s);
        }
        if (st != SG_OK) break;
        if (hipEventSynchronize(ev[reps]) != hipSuccess) { st = fail(SG_EHIP, "autotune: event"); break; }
        std::vector<float> t(reps);
        for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], ev[r], ev[r + 1]);
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        med[on] = t[reps / 2];
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (st == SG_OK) h->seg_on = med[1] < med[0];
    return st;
}

// FGMRES orthogonalises by classical Gram-Schmidt with the reorthogonalisation delayed into the next
// step (DCGS2) unless SGHEAT_FGMRES_CGS2=1 (a measurement switch: both passes of classical Gram-Schmidt
// with reorthogonalisation in every step).  Read at every solve.
bool fgmres_classic_cgs2() {
    const char* e = std::getenv("SGHEAT_FGMRES_CGS2");
    return e && std::strcmp(e, "1") == 0;
}

// y = A x (b == nullptr) or y = b - A x, for the operator described by op; the cell-local results go
// to `cells` (default: the handle's buffer)
template <typename T>
sg_status op_apply(sg_handle h, const ApplyOp<T>& op, const T* x, T* y, const T* b, hipStream_t s,
                   T* cells = nullptr) {
    if (op.mean && !h->diag && !cells && op.level >= 0 && h->lv[op.level].mean_const && !mean_stencil_disabled()) {
        const Level& lv = h->lv[op.level];
        StencilArgs sa{};
        sa.dim = h->d.dim;
        sa.k = h->d.fe_degree;
        sa.nt = h->NT;
        sa.n1 = lv.g.n1;
        sa.n_xi = h->n_xi;
        sa.Mb = sizeof(T) == 8 ? (const void*)lv.mb64.p : (const void*)lv.mb32.p;
        sa.Kb = sizeof(T) == 8 ? (const void*)lv.kb64.p : (const void*)lv.kb32.p;
        for (int i = 0; i < h->NT * h->NT; ++i) sa.At[i] = h->At[i];
        for (int i = 0; i < h->NT; ++i) sa.Bt[i] = h->Bt[i];
        sa.x = x;
        sa.b = b;
        sa.y = y;
        StencilArgs probe = sa;
        if (stencil_fits(probe, (int)sizeof(T))) {
            SG_HIP(launch_mean_stencil<T>(sa, s));
            return SG_OK;
        }
    }
    ApplyOp<T> o = op;
    int cpb = 1, lz = 1;
    o.used_cpb = &cpb;
    o.used_lz = &lz;
    T* sb = cells ? cells : sbuf_as<T>(h);
    SG_HIP(launch_apply<T>(o, x, sb, s));
    SG_HIP(launch_node_gather<T>(b ? GATHER_RESIDUAL : GATHER_SET, op.dim, op.k, op.g, h->n_xi * h->NT, sb, x, b, y,
                                 T(0), apply_segment(o, cpb), apply_zsegment(o, lz), s));
    return SG_OK;
}

// ---- scratch of the allocation-free apply -----------------------------------------------------------
// The cell-local results of sg_operator_apply_noalloc live in this file-scope device array (each GPU
// the library runs on holds its own copy until the process ends).  In host code the name `scratch`
// is a host-side stand-in, not device memory: host code uses only the device address resolved by
// hipGetSymbolAddress, once per device at set-up (sg_create), with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (the current device); resolved once per device.
sg_status resolve_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SG_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return SG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(SG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    return SG_OK;
}

void* scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

template <typename T>
sg_status smooth_level(sg_handle h, int l, const T* b, T* x, int sweeps, bool x_is_zero, hipStream_t s) {
    Level& lv = h->lv[l];
    const ApplyOp<T> op = make_block_op<T>(h, l);
    const T* inv = Prec<T>::inv(lv);
    for (int it = 0; it < sweeps; ++it) {
        const T* r = b;   // with x = 0 the residual b - A_0 x is b itself
        if (!(x_is_zero && it == 0)) {
            SG_TRY(op_apply<T>(h, op, x, Prec<T>::r(lv), b, s));
            r = Prec<T>::r(lv);
        }
        int sx = h->d.fe_degree;                  // x segment length of the corrections' broken layout
        if (h->diag)
            SG_HIP(launch_vanka_cells_modes<T>(h->d.dim, h->d.fe_degree, h->NT, lv.g, h->n_xi, inv, r, sbuf_as<T>(h), s));
        else if (lv.mean_const && !vanka_fdm_disabled())
            SG_HIP(launch_vanka_fdm<T>(h->d.dim, h->d.fe_degree, h->NT, lv.g, h->n_xi, Prec<T>::fdmS(lv),
                                       Prec<T>::fdmT(lv), r, sbuf_as<T>(h), &sx, s));
        else
            SG_HIP(launch_vanka_cells<T>(h->d.dim, h->d.fe_degree, h->NT, lv.g, h->n_xi, inv, r, sbuf_as<T>(h),
                                         lv.inv_classes, s));
        SG_HIP(launch_node_gather<T>(GATHER_VANKA, h->d.dim, h->d.fe_degree, lv.g, h->n_xi * h->NT, sbuf_as<T>(h),
                                     nullptr, b, x, (T)h->d.vanka_omega, sx, h->d.fe_degree, s));
    }
    return SG_OK;
}

int dims_of(const Grid& g, int dim, int* out) {
    for (int i = 0; i < 3; ++i) out[i] = i < dim ? g.n1 : 1;
    return 0;
}

// b_c = R r_f (restriction), fine level l -> coarse level l+1
template <typename T>
sg_status restrict_to(sg_handle h, int l, const T* rf, T* bc, hipStream_t s) {
    const int dim = h->d.dim, nc = h->n_xi * h->NT;
    const Level& lf = h->lv[l];
    const Level& lc = h->lv[l + 1];
    int cur[3];
    dims_of(lf.g, dim, cur);
    const T* in = rf;
    T* bufs[2] = {Prec<T>::ta(h), Prec<T>::tb(h)};
    for (int dir = 0; dir < dim; ++dir) {
        int out[3] = {cur[0], cur[1], cur[2]};
        out[dir] = lc.g.n1;
        T* o = (dir == dim - 1) ? bc : bufs[dir % 2];
        SG_HIP(launch_transfer_1d<T>(dim, nc, cur, out, dir, lf.r_idx.p, Prec<T>::rw(lf), lf.wr, in, o, false, s));
        in = o;
        for (int i = 0; i < 3; ++i) cur[i] = out[i];
    }
    return SG_OK;
}

// x_f += P x_c (prolongation), coarse level l+1 -> fine level l
template <typename T>
sg_status prolong_add(sg_handle h, int l, const T* xc, T* xf, hipStream_t s) {
    const int dim = h->d.dim, nc = h->n_xi * h->NT;
    const Level& lf = h->lv[l];
    const Level& lc = h->lv[l + 1];
    int cur[3];
    dims_of(lc.g, dim, cur);
    const T* in = xc;
    T* bufs[2] = {Prec<T>::ta(h), Prec<T>::tb(h)};
    for (int dir = 0; dir < dim; ++dir) {
        int out[3] = {cur[0], cur[1], cur[2]};
        out[dir] = lf.g.n1;
        const bool last = dir == dim - 1;
        T* o = last ? xf : bufs[dir % 2];
        SG_HIP(launch_transfer_1d<T>(dim, nc, cur, out, dir, lf.p_idx.p, Prec<T>::pw(lf), lf.wp, in, o, last, s));
        in = o;
        for (int i = 0; i < 3; ++i) cur[i] = out[i];
    }
    return SG_OK;
}

// Levels l .. L-1 of the cycle in one launch (kernels_segment.hip): one workgroup per mode.
template <typename T>
sg_status vcycle_segment(sg_handle h, int l0, const T* b, T* x, hipStream_t s) {
    const int L = h->d.n_levels;
    SegArgs a{};
    a.dim = h->d.dim;
    a.k = h->d.fe_degree;
    a.nt = h->NT;
    a.np = h->NP;
    a.n_xi = h->n_xi;
    a.nlev = L - l0;
    long long tmp = 0;
    for (int i = 0; i < a.nlev; ++i) {
        Level& lv = h->lv[l0 + i];
        SegLevelArgs& q = a.lv[i];
        q.g = lv.g;
        q.inv = Prec<T>::inv(lv);
        q.classes = lv.inv_classes;
        q.E = lv.E64.p;
        q.Me = lv.Me64.p;
        q.b = i == 0 ? const_cast<T*>(b) : Prec<T>::b(lv);
        q.x = i == 0 ? x : Prec<T>::x(lv);
        q.r = Prec<T>::r(lv);
        if (l0 + i < L - 1) {
            q.r_idx = lv.r_idx.p;
            q.r_w = Prec<T>::rw(lv);
            q.wr = lv.wr;
            q.p_idx = lv.p_idx.p;
            q.p_w = Prec<T>::pw(lv);
            q.wp = lv.wp;
            // the largest intermediate of a 1D pass between this level and the next, one mode
            const long long nf = lv.g.n1, nc = h->lv[l0 + i + 1].g.n1;
            tmp = std::max(tmp, (long long)h->NT * (h->d.dim == 3 ? nf * nf * nc : nf * nc));
        }
    }
    for (int i = 0; i < h->NT * h->NT; ++i) a.At[i] = h->At[i];
    for (int i = 0; i < h->NT; ++i) a.Bt[i] = h->Bt[i];
    a.omega = h->d.vanka_omega;
    a.pre = h->d.pre_smooth;
    a.post = h->d.post_smooth;
    a.coarse_invT = h->coarse_invT.p;
    a.nint = h->nint;
    a.coarse_dofs = h->coarse_dofs.p;
    a.tmp_len = tmp;
    a.scratch_per_mode = segment_scratch_per_mode(h->NT, h->NP, h->lv[l0].g.n_cells, tmp);
    a.scratch = h->sbuf.p;
    SG_HIP(launch_vcycle_segment<T>(a, s));
    return SG_OK;
}

template <typename T>
sg_status vcycle_level(sg_handle h, int l, const T* b, T* x, hipStream_t s) {
    const int L = h->d.n_levels;
    Level& lv = h->lv[l];
    if (h->seg_on && l == h->seg_level) return vcycle_segment<T>(h, l, b, x, s);
    if (l == L - 1) {
        SG_HIP(launch_coarse_solve<T>(h->coarse_invT.p, h->diag ? (long long)h->nint * h->nint : 0, h->nint,
                                      h->coarse_dofs.p, h->n_xi, (long long)h->NT * lv.g.n_nodes,
                                      b, x, s));
        return SG_OK;
    }
    SG_HIP(launch_fill<T>(x, T(0), lv.len, s));
    SG_TRY(smooth_level<T>(h, l, b, x, h->d.pre_smooth, true, s));
    const ApplyOp<T> op = make_block_op<T>(h, l);
    SG_TRY(op_apply<T>(h, op, x, Prec<T>::r(lv), b, s));
    Level& lc = h->lv[l + 1];
    SG_TRY(restrict_to<T>(h, l, Prec<T>::r(lv), Prec<T>::b(lc), s));
    SG_TRY(vcycle_level<T>(h, l + 1, Prec<T>::b(lc), Prec<T>::x(lc), s));
    SG_TRY(prolong_add<T>(h, l, Prec<T>::x(lc), x, s));
    SG_TRY(smooth_level<T>(h, l, b, x, h->d.post_smooth, false, s));
    return SG_OK;
}

// The V-cycle on the level-0 work vectors (b -> x), the part a graph replays.
sg_status vcycle_fixed(sg_handle h, hipStream_t s) {
    Level& l0 = h->lv[0];
    if (!h->mixed) return vcycle_level<double>(h, 0, l0.b64.p, l0.x64.p, s);
    return vcycle_level<float>(h, 0, l0.b32.p, l0.x32.p, s);
}

// Capture vcycle_fixed into a graph on the handle's own stream (nothing runs during capture).
sg_status capture_vcycle(sg_handle h) {
    if (!h->cap_stream) SG_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    SG_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    const sg_status st = vcycle_fixed(h, h->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (st != SG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess || !g) return fail(SG_EHIP, std::string("V-cycle capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SG_EHIP, std::string("V-cycle graph: ") + hipGetErrorString(ie));
    }
    h->vgraph = g;
    h->vgraph_exec = ex;
    return SG_OK;
}

sg_status vcycle(sg_handle h, const double* r, double* z, hipStream_t s) {
    Level& l0 = h->lv[0];
    if (!h->graph_on) {
        if (!h->mixed) return vcycle_level<double>(h, 0, r, z, s);
        SG_HIP((launch_convert<double, float>(r, l0.b32.p, l0.len, s)));
        SG_TRY(vcycle_level<float>(h, 0, l0.b32.p, l0.x32.p, s));
        SG_HIP((launch_convert<float, double>(l0.x32.p, z, l0.len, s)));
        return SG_OK;
    }
    // graph path: r into the level-0 work vector, the captured cycle, the result out
    if (!h->mixed) SG_HIP(hipMemcpyAsync(l0.b64.p, r, sizeof(double) * l0.len, hipMemcpyDeviceToDevice, s));
    else SG_HIP((launch_convert<double, float>(r, l0.b32.p, l0.len, s)));
    if (h->graph_calls++ == 0) {
        SG_TRY(vcycle_fixed(h, s));            // first call eagerly (fills the launch caches), then capture
        SG_TRY(capture_vcycle(h));
    } else {
        SG_HIP(hipGraphLaunch(h->vgraph_exec, s));
    }
    if (!h->mixed) SG_HIP(hipMemcpyAsync(z, l0.x64.p, sizeof(double) * l0.len, hipMemcpyDeviceToDevice, s));
    else SG_HIP((launch_convert<float, double>(l0.x32.p, z, l0.len, s)));
    return SG_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

// ---- operator variants on level 0: adjoint orientation, slab transfer, bilinear forms, QoI --------

// Level-0 tables with the time matrix `at` in place of A_t (row i is divided by B_t[i] as for A_t).
Tables<double> tables_with(const sg_handle h, const std::vector<double>& at) {
    Tables<double> tb{};
    fill_tables(&tb, h->tS, h->tD, h->tgw, at, h->Bt, h->d.fe_degree + 1, h->NT, std::pow(h->lv[0].h, h->d.dim));
    return tb;
}

// A zero mean-coefficient array of level 0 (mass-only variants).
sg_status zero_coef(sg_handle h, hipStream_t s) {
    const size_t n = (size_t)h->lv[0].g.n_cells * h->NP;
    if (!h->zcoef.p) {
        SG_TRY(h->zcoef.alloc(n, "zero coefficient"));
        SG_HIP(launch_fill<double>(h->zcoef.p, 0.0, (long long)n, s));
    }
    return SG_OK;
}

// Level-0 operator variant: time tables `tb`, coefficient modes `coef` (the mean mode alone when
// !full); cell-local results go to sbuf and, with y, are gathered into y.
sg_status variant_apply(sg_handle h, const Tables<double>* tb, const double* coef, bool full, const double* x,
                        double* y, GatherOp gop, hipStream_t s, bool per_cell = false) {
    ApplyOp<double> op = make_op<double>(h, 0, full);
    op.tables = tb;
    op.coef = coef;
    op.merge = per_cell ? 0 : 1;     // per-cell results (for cell-wise forms) need the unmerged layout
    int cpb = 1, lz = 1;
    op.used_cpb = &cpb;
    op.used_lz = &lz;
    SG_HIP(launch_apply<double>(op, x, h->sbuf.p, s));
    if (y)
        SG_HIP(launch_node_gather<double>(gop, h->d.dim, h->d.fe_degree, h->lv[0].g, h->n_xi * h->NT, h->sbuf.p, x,
                                          nullptr, y, 0.0, apply_segment(op, cpb), apply_zsegment(op, lz), s));
    return SG_OK;
}

// E[Psi_a Psi_b Psi_eps] for a, b in the handle's index set and eps of total degree <= 2 p_xi.
void build_triple_table(sg_handle h) {
    if (!h->trip.empty()) return;
    const int M = h->d.n_vars, p = h->d.chaos_degree, nx = h->n_xi;
    const std::vector<std::vector<int>> A = total_degree_set(M, p);
    const std::vector<std::vector<int>> E = total_degree_set(M, 2 * p);
    h->n_eps = (int)E.size();
    h->trip.assign((size_t)nx * nx * h->n_eps, 0.0);
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < nx; ++b)
            for (int e = 0; e < h->n_eps; ++e) {
                double v = 1.0;
                for (int m = 0; m < M && v != 0.0; ++m) v *= hermite_triple_1d(A[a][m], A[b][m], E[e][m]);
                h->trip[((size_t)a * nx + b) * h->n_eps + e] = v;
            }
}

double dev_dot_sync(sg_handle h, const double* a, const double* b, long long n, hipStream_t s, sg_status* st) {
    double out = 0.0;
    *st = SG_OK;
    if (launch_multidot(a, 0, 1, b, n, h->partial.p, kDotBlocks, s) != hipSuccess ||
        launch_reduce_partials(h->partial.p, kDotBlocks, 1, h->dscal.p, s) != hipSuccess ||
        hipMemcpyAsync(&out, h->dscal.p, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        *st = fail(SG_EHIP, "dot product failed");
    }
    return out;
}

}  // namespace

extern "C" {

sg_status sg_create(const sg_problem_desc* desc, sg_handle* out) {
    if (!out) return fail(SG_EINVAL, "out is NULL");
    *out = nullptr;
    SG_TRY(validate(desc));
    std::unique_ptr<sg_handle_s> h(new (std::nothrow) sg_handle_s());
    if (!h) return fail(SG_ENOMEM, "host allocation failed");
    h->d = *desc;
    h->coef_mu.assign(desc->coef_mu, desc->coef_mu + (size_t)desc->n_coef_modes * desc->n_vars);
    h->d.coef_mu = h->coef_mu.data();
    if (desc->n_samples > 0) h->samples.assign(desc->samples, desc->samples + (size_t)desc->n_samples * desc->n_vars);
    h->d.samples = nullptr;   // host array not retained
    if (desc->n_members > 0) {
        h->member_degree.assign(desc->member_degree, desc->member_degree + desc->n_members);
        h->member_scale.assign(desc->member_scale, desc->member_scale + (size_t)desc->n_members * desc->n_coef_modes);
    }
    h->d.member_degree = nullptr;
    h->d.member_scale = nullptr;
    try {
        sg_status s = build(h.get());
        h->d.coef_qp = nullptr;   // host array not retained
        if (s != SG_OK) return s;
    } catch (const std::bad_alloc&) {
        return fail(SG_ENOMEM, "host allocation failed during set-up");
    }
    SG_HIP(hipGetDevice(&h->device));
    SG_TRY(resolve_scratch(h->device));
    SG_HIP(hipEventCreateWithFlags(&h->last_work, hipEventDisableTiming));
    *out = h.release();
    return SG_OK;
}

sg_status sg_destroy(sg_handle h) {
    if (!h) return SG_OK;
    h->quiesce();
    delete h;
    return SG_OK;
}

sg_status sg_vector_length(sg_handle h, int level, long long* n) {
    if (!h || !n) return fail(SG_EINVAL, "null argument");
    if (level < 0 || level >= h->d.n_levels) return fail(SG_EINVAL, "level out of range");
    *n = h->lv[level].len;
    return SG_OK;
}

sg_status sg_operator_apply(sg_handle h, const double* x, double* y, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !x || !y) return fail(SG_EINVAL, "null argument");
    if (overlap(x, y, h->N * sizeof(double))) return fail(SG_EINVAL, "x and y overlap");
    const ApplyOp<double> op = make_op<double>(h, 0, true);
    SG_TRY(op_apply<double>(h, op, x, y, nullptr, (hipStream_t)hip_stream));
    return SG_OK;
}

sg_status sg_operator_apply_noalloc(sg_handle h, const double* x, double* y, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !x || !y) return fail(SG_EINVAL, "null argument");
    if (overlap(x, y, h->N * sizeof(double))) return fail(SG_EINVAL, "x and y overlap");
    // the cell-local results take at most n_xi N_t n_cells (k+1)^d doubles (the per-cell layout)
    const size_t need = (size_t)h->n_xi * h->NT * (size_t)h->lv[0].g.n_cells * h->NP * sizeof(double);
    if (need > kScratchBytes)
        return fail(SG_EINVAL, "the operator's cell-local results (" + std::to_string(need) +
                                   " bytes) exceed the allocation-free apply's scratch of " +
                                   std::to_string(kScratchBytes) + " bytes; use sg_operator_apply");
    double* cells = static_cast<double*>(scratch_of(h->device));
    if (!cells) return fail(SG_EHIP, "scratch address of the handle's device is not resolved");
    const ApplyOp<double> op = make_op<double>(h, 0, true);
    SG_TRY(op_apply<double>(h, op, x, y, nullptr, (hipStream_t)hip_stream, cells));
    return SG_OK;
}

sg_status sg_vanka_smooth(sg_handle h, int level, const double* b, double* x, int sweeps, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !b || !x) return fail(SG_EINVAL, "null argument");
    if (level < 0 || level >= h->d.n_levels) return fail(SG_EINVAL, "level out of range");
    if (sweeps < 0) return fail(SG_EINVAL, "sweeps must be >= 0");
    Level& lv = h->lv[level];
    if (overlap(b, x, lv.len * sizeof(double))) return fail(SG_EINVAL, "b and x overlap");
    hipStream_t s = (hipStream_t)hip_stream;
    const bool use32 = h->mixed && level < h->d.n_levels - 1;
    if (!use32) return smooth_level<double>(h, level, b, x, sweeps, false, s);
    SG_HIP((launch_convert<double, float>(b, lv.b32.p, lv.len, s)));
    SG_HIP((launch_convert<double, float>(x, lv.x32.p, lv.len, s)));
    SG_TRY(smooth_level<float>(h, level, lv.b32.p, lv.x32.p, sweeps, false, s));
    SG_HIP((launch_convert<float, double>(lv.x32.p, x, lv.len, s)));
    return SG_OK;
}

sg_status gmg_vcycle(sg_handle h, const double* r, double* z, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !r || !z) return fail(SG_EINVAL, "null argument");
    if (overlap(r, z, h->N * sizeof(double))) return fail(SG_EINVAL, "r and z overlap");
    return vcycle(h, r, z, (hipStream_t)hip_stream);
}

sg_status fgmres_solve_slab(sg_handle h, const double* b, double* x, double rtol, int max_iter, sg_solve_info* info,
                            void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !b || !x) return fail(SG_EINVAL, "null argument");
    if (!(rtol > 0.0) || max_iter < 1) return fail(SG_EINVAL, "rtol > 0 and max_iter >= 1 required");
    if (overlap(b, x, h->N * sizeof(double))) return fail(SG_EINVAL, "b and x overlap");
    hipStream_t s = (hipStream_t)hip_stream;
    const long long n = h->N;
    const int m = h->restart;
    sg_solve_info inf{};
    // timing marks from the handle's event pool (grown on first use, reused by later solves)
    size_t ev_used = 0;
    auto mark = [&](std::vector<hipEvent_t>& v) -> hipError_t {
        if (ev_used == h->ev_pool.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            h->ev_pool.push_back(e);
        }
        hipEvent_t e = h->ev_pool[ev_used++];
        v.push_back(e);
        return hipEventRecord(e, s);
    };
    std::vector<hipEvent_t> ev_apply, ev_prec, ev_total;
    SG_HIP(mark(ev_total));
    const ApplyOp<double> op = make_op<double>(h, 0, true);
    double* V = h->V.p;
    double* Z = h->Z.p;
    sg_status st;
    const double bnorm = std::sqrt(dev_dot_sync(h, b, b, n, s, &st));
    if (st != SG_OK) return st;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    double hscal[3 * 80];
    sg_status result = SG_NOT_CONVERGED;
    if (bnorm == 0.0) {
        SG_HIP(launch_fill<double>(x, 0.0, n, s));
        inf.converged = 1;
        result = SG_OK;
    } else {
        while (true) {
            // true residual r = b - AA x into V[0]
            SG_HIP(mark(ev_apply));
            SG_TRY(op_apply<double>(h, op, x, V, b, s));
            SG_HIP(mark(ev_apply));
            inf.applies++;
            const double beta = std::sqrt(dev_dot_sync(h, V, V, n, s, &st));
            if (st != SG_OK) return st;
            inf.rel_residual_true = beta / bnorm;
            if (beta / bnorm <= rtol) { inf.converged = 1; result = SG_OK; break; }
            if (inf.iterations >= max_iter) break;
            inf.restarts++;
            SG_HIP(launch_axpby(1.0 / beta, V, 0.0, nullptr, V, n, s));
            std::fill(H.begin(), H.end(), 0.0);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int kdim = 0;
            if (!fgmres_classic_cgs2()) {
                // DCGS2: V[j] enters step j as the tentative vector u_j (orthogonal once to V[0..j-1]); the
                // step's dot pass also yields its reorthogonalisation coefficients a, its update pass writes
                // the final v_j = (u_j - V a) / nu_j over it and the next tentative vector
                // u_{j+1} = w - V b - e v_j.  Column j-1 of H (A z_{j-1} = ... + u_j) is completed here:
                // h_{i,j-1} += a_i, h_{j,j-1} = nu_j; column j is tested with the provisional
                // h_{j+1,j} = |u_{j+1}| and kept that way if the iteration ends there.
                double* d_r = h->dscal.p;                 // [a (j), b (j), u.u, u.w]
                double* d_s = h->dscal.p + 2 * kDcgsMaxBasis + 2;   // |u_{j+1}|^2
                std::vector<double> col(m + 1);
                for (int j = 0; j < m; ++j) {
                    double* uj = V + (size_t)j * n;
                    double* zj = Z + (size_t)j * n;
                    SG_HIP(mark(ev_prec));
                    SG_TRY(vcycle(h, uj, zj, s));
                    SG_HIP(mark(ev_prec));
                    inf.vcycles++;
                    SG_HIP(mark(ev_apply));
                    SG_TRY(op_apply<double>(h, op, zj, h->w1.p, nullptr, s));
                    SG_HIP(mark(ev_apply));
                    inf.applies++;
                    SG_HIP(launch_dcgs_dots(V, n, j, uj, h->w1.p, n, h->partial.p, kDotBlocks, s));
                    SG_HIP(launch_reduce_partials(h->partial.p, kDotBlocks, 2 * j + 2, d_r, s));
                    SG_HIP(launch_dcgs_update(V, n, j, d_r, uj, h->w1.p, V + (size_t)(j + 1) * n, n, h->partial.p,
                                              kDotBlocks, s));
                    SG_HIP(launch_reduce_partials(h->partial.p, kDotBlocks, 1, d_s, s));
                    SG_HIP(hipMemcpyAsync(hscal, h->dscal.p, sizeof(double) * (2 * kDcgsMaxBasis + 3),
                                          hipMemcpyDeviceToHost, s));
                    SG_HIP(hipStreamSynchronize(s));
                    const double* ra = hscal;
                    const double* rb = hscal + j;
                    double ss = 0.0, ab = 0.0;            // the device's sums, in the same order
                    for (int i = 0; i < j; ++i) {
                        ss += ra[i] * ra[i];
                        ab += ra[i] * rb[i];
                    }
                    const double nu2 = hscal[2 * j] - ss;
                    const double nu = nu2 > 0.0 ? std::sqrt(nu2) : 0.0;
                    const double e = nu > 0.0 ? (hscal[2 * j + 1] - ab) / nu : 0.0;
                    const double un2 = hscal[2 * kDcgsMaxBasis + 2];
                    const double un = un2 > 0.0 ? std::sqrt(un2) : 0.0;
                    auto rotate_column = [&](int c) {         // rotations of columns < c, then its own
                        for (int i = 0; i < c; ++i) {
                            const double t = cs[i] * H[(size_t)i * m + c] + sn[i] * H[(size_t)(i + 1) * m + c];
                            H[(size_t)(i + 1) * m + c] = -sn[i] * H[(size_t)i * m + c] + cs[i] * H[(size_t)(i + 1) * m + c];
                            H[(size_t)i * m + c] = t;
                        }
                        const double den = std::hypot(H[(size_t)c * m + c], H[(size_t)(c + 1) * m + c]);
                        cs[c] = den > 0.0 ? H[(size_t)c * m + c] / den : 1.0;
                        sn[c] = den > 0.0 ? H[(size_t)(c + 1) * m + c] / den : 0.0;
                        H[(size_t)c * m + c] = den;
                        H[(size_t)(c + 1) * m + c] = 0.0;
                        g[c + 1] = -sn[c] * g[c];
                        g[c] = cs[c] * g[c];
                    };
                    if (j == 0) {
                        if (!(nu > 0.0)) break;               // no basis (a non-finite residual): kdim = 0
                        g[0] = beta * nu;                     // r = beta u_0 = beta nu_0 v_0
                    } else {
                        for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] += ra[i];
                        H[(size_t)j * m + (j - 1)] = nu;
                        rotate_column(j - 1);
                        if (nu == 0.0) break;                 // A z_{j-1} lies in span V[0..j-1]: kdim = j
                    }
                    for (int i = 0; i < j; ++i) H[(size_t)i * m + j] = rb[i];
                    H[(size_t)j * m + j] = e;
                    H[(size_t)(j + 1) * m + j] = un;
                    // provisional test of column j (on copies of the column and of g)
                    for (int i = 0; i <= j + 1; ++i) col[i] = H[(size_t)i * m + j];
                    for (int i = 0; i < j; ++i) {
                        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                        col[i] = t;
                    }
                    const double den = std::hypot(col[j], col[j + 1]);
                    const double res = den > 0.0 ? std::fabs(col[j + 1] / den * g[j]) : std::fabs(g[j]);
                    inf.iterations++;
                    kdim = j + 1;
                    if (nu == 0.0 || un == 0.0 || res / bnorm <= rtol || inf.iterations >= max_iter || j + 1 == m) {
                        rotate_column(j);
                        break;
                    }
                }
            } else
            for (int j = 0; j < m; ++j) {
                double* vj = V + (size_t)j * n;
                double* zj = Z + (size_t)j * n;
                SG_HIP(mark(ev_prec));
                SG_TRY(vcycle(h, vj, zj, s));
                SG_HIP(mark(ev_prec));
                inf.vcycles++;
                SG_HIP(mark(ev_apply));
                SG_TRY(op_apply<double>(h, op, zj, h->w1.p, nullptr, s));
                SG_HIP(mark(ev_apply));
                inf.applies++;
                const int kk = j + 1;
                double* d_h1 = h->dscal.p;
                double* d_h2 = h->dscal.p + 80;       // h2, then |w'|^2
                double* vnext = V + (size_t)(j + 1) * n;
                // CGS2: h1 = V^T w; w' = w - V h1 with h2 = V^T w' and |w'|^2 in the same pass;
                // v = (w' - V h2) / hn with hn^2 = |w'|^2 - |h2|^2 (Pythagoras: V orthonormal), so the new
                // basis vector is written normalised in the last pass
                SG_HIP(launch_multidot(V, n, kk, h->w1.p, n, h->partial.p, kDotBlocks, s));
                SG_HIP(launch_reduce_partials(h->partial.p, kDotBlocks, kk, d_h1, s));
                SG_HIP(launch_update_dot(V, n, kk, d_h1, h->w1.p, h->w2.p, n, h->partial.p, kDotBlocks, kUpdDotNorm, s));
                SG_HIP(launch_reduce_partials(h->partial.p, kDotBlocks, kk + 1, d_h2, s));
                SG_HIP(launch_update_dot(V, n, kk, d_h2, h->w2.p, vnext, n, h->partial.p, kDotBlocks, kUpdScaled, s));
                SG_HIP(hipMemcpyAsync(hscal, h->dscal.p, sizeof(double) * 160, hipMemcpyDeviceToHost, s));
                SG_HIP(hipStreamSynchronize(s));
                double ss = 0.0;                      // the device's sum, in the same order
                for (int i = 0; i < kk; ++i) ss += hscal[80 + i] * hscal[80 + i];
                const double hn2 = hscal[80 + kk] - ss;
                const double hn = hn2 > 0.0 ? std::sqrt(hn2) : 0.0;
                for (int i = 0; i < kk; ++i) H[(size_t)i * m + j] = hscal[i] + hscal[80 + i];
                H[(size_t)(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
                    H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
                    H[(size_t)i * m + j] = t;
                }
                const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
                cs[j] = H[(size_t)j * m + j] / den;
                sn[j] = H[(size_t)(j + 1) * m + j] / den;
                H[(size_t)j * m + j] = den;
                H[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                inf.iterations++;
                kdim = j + 1;
                if (hn == 0.0 || std::fabs(g[j + 1]) / bnorm <= rtol || inf.iterations >= max_iter) break;
            }
            if (kdim == 0) break;
            for (int i = kdim - 1; i >= 0; --i) {
                double acc = g[i];
                for (int c = i + 1; c < kdim; ++c) acc -= H[(size_t)i * m + c] * y[c];
                y[i] = acc / H[(size_t)i * m + i];
            }
            SG_HIP(hipMemcpyAsync(h->dscal.p, y.data(), sizeof(double) * kdim, hipMemcpyHostToDevice, s));
            SG_HIP(launch_multi_axpy(Z, n, kdim, h->dscal.p, x, n, s));
        }
    }
    SG_HIP(mark(ev_total));
    SG_HIP(hipStreamSynchronize(s));
    auto sum_pairs = [](const std::vector<hipEvent_t>& v) {
        double t = 0.0;
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, v[i], v[i + 1]) == hipSuccess) t += ms;
        }
        return t;
    };
    inf.t_apply_ms = sum_pairs(ev_apply);
    inf.t_prec_ms = sum_pairs(ev_prec);
    inf.t_total_ms = sum_pairs(ev_total);
    inf.work_proxy = (double)n * inf.vcycles;
    if (info) *info = inf;
    if (result == SG_NOT_CONVERGED) g_last_error = "FGMRES did not reach the tolerance within max_iter";
    return result;
}

sg_status sg_update_coefficients(sg_handle h, const double* coef_qp) {
    if (!h || !coef_qp) return fail(SG_EINVAL, "null argument");
    try {
        h->quiesce();
        h->drop_graph();                       // the graph holds the set-up's buffers and tiles
        return set_coefficients(h, coef_qp);
    } catch (const std::bad_alloc&) {
        return fail(SG_ENOMEM, "host allocation failed during the coefficient update");
    }
}

sg_status sg_operator_apply_T(sg_handle h, const double* x, double* y, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !x || !y) return fail(SG_EINVAL, "null argument");
    if (overlap(x, y, h->N * sizeof(double))) return fail(SG_EINVAL, "x and y overlap");
    ApplyOp<double> op = make_op<double>(h, 0, true);
    op.tables = &h->tabT64;
    SG_TRY(op_apply<double>(h, op, x, y, nullptr, (hipStream_t)hip_stream));
    return SG_OK;
}

sg_status sg_slab_transfer(sg_handle h, int transpose, const double* x, double* y, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !x || !y) return fail(SG_EINVAL, "null argument");
    if (transpose != 0 && transpose != 1) return fail(SG_EINVAL, "transpose must be 0 or 1");
    if (overlap(x, y, h->N * sizeof(double))) return fail(SG_EINVAL, "x and y overlap");
    hipStream_t s = (hipStream_t)hip_stream;
    SG_TRY(zero_coef(h, s));
    const int NT = h->NT, r = NT - 1;
    std::vector<double> ct((size_t)NT * NT, 0.0);   // C_t[i][j] = v_i(0+) [j == r]
    for (int i = 0; i < NT; ++i) {
        if (transpose) ct[(size_t)r * NT + i] = h->radau0[i];
        else ct[(size_t)i * NT + r] = h->radau0[i];
    }
    const Tables<double> tb = tables_with(h, ct);
    return variant_apply(h, &tb, h->zcoef.p, false, x, y, GATHER_INTERIOR, s);
}

namespace {

// out[K] = lam^T (G_mu (x) B_t (x) K_{c|K}) u on level 0.  The scaled field of every mode stays on the
// device: it is uploaded again (and the stream synchronised, the staging array being the caller's
// stack) only when the caller's values differ from the last ones given for that mode.
sg_status form_cells(sg_handle h, int mu_index, const double* coef_qp, const double* lam, const double* u,
                     double* out, hipStream_t s) {
    const Level& l0 = h->lv[0];
    const int dim = h->d.dim, N1 = h->d.fe_degree + 1;
    const size_t per_mode = (size_t)l0.g.n_cells * h->NP;
    const bool mean = mu_index == h->cpl.mu0;
    if (h->form_fields.n < (size_t)h->n_mu * per_mode) {
        SG_TRY(h->form_fields.alloc((size_t)h->n_mu * per_mode, "form fields"));
        SG_TRY(h->fcoef.alloc((size_t)h->n_mu * per_mode, "form coefficient"));
        SG_HIP(launch_fill<double>(h->fcoef.p, 0.0, (long long)(h->n_mu * per_mode), s));
        h->form_raw.assign(h->n_mu, {});
        h->form_active = -1;
    }
    std::vector<double>& raw = h->form_raw[mu_index];
    double* field = h->form_fields.p + (size_t)mu_index * per_mode;
    if (raw.size() != per_mode || std::memcmp(raw.data(), coef_qp, per_mode * sizeof(double)) != 0) {
        // the field at the Gauss points, scaled like the create-time coefficients (weight, h^(d-2))
        std::vector<double> stage(per_mode);
        const double hs = std::pow(l0.h, dim - 2);
        for (size_t c = 0; c < (size_t)l0.g.n_cells; ++c)
            for (int q = 0; q < h->NP; ++q) {
                double wq = hs;
                for (int dd = 0, qq = q; dd < dim; ++dd, qq /= N1) wq *= h->tgw[qq % N1];
                stage[c * h->NP + q] = coef_qp[c * h->NP + q] * wq;
            }
        SG_HIP(hipMemcpyAsync(field, stage.data(), per_mode * sizeof(double), hipMemcpyHostToDevice, s));
        SG_HIP(hipStreamSynchronize(s));
        raw.assign(coef_qp, coef_qp + per_mode);
        if (h->form_active == mu_index) h->form_active = -1;    // fcoef holds the old values
    }
    const double* coef = field;                 // the mean-block operator reads one mode
    if (!mean) {
        // the full operator reads every mode: only mode mu of fcoef is non-zero
        if (h->form_active != mu_index) {
            if (h->form_active >= 0)
                SG_HIP(launch_fill<double>(h->fcoef.p + (size_t)h->form_active * per_mode, 0.0, (long long)per_mode, s));
            SG_HIP(hipMemcpyAsync(h->fcoef.p + (size_t)mu_index * per_mode, field, per_mode * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
            h->form_active = mu_index;
        }
        coef = h->fcoef.p;
    }
    const std::vector<double> no_mass((size_t)h->NT * h->NT, 0.0);
    const Tables<double> tb = tables_with(h, no_mass);
    SG_TRY(variant_apply(h, &tb, coef, !mean, u, nullptr, GATHER_SET, s, true));
    SG_HIP(launch_cell_dot(dim, h->d.fe_degree, l0.g, h->n_xi * h->NT, lam, h->sbuf.p, out, s));
    return SG_OK;
}

}  // namespace

sg_status sg_stiffness_form_cells(sg_handle h, int mu_index, const double* coef_qp, const double* lam,
                                  const double* u, double* out, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !coef_qp || !lam || !u || !out) return fail(SG_EINVAL, "null argument");
    if (mu_index < 0 || mu_index >= h->n_mu) return fail(SG_EINVAL, "mu_index out of range");
    return form_cells(h, mu_index, coef_qp, lam, u, out, (hipStream_t)hip_stream);
}

sg_status sg_stiffness_form_accumulate(sg_handle h, int mu_index, const double* coef_qp, const double* lam,
                                       const double* u, double scale, double* cells, double* total,
                                       void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !coef_qp || !lam || !u) return fail(SG_EINVAL, "null argument");
    if (!cells && !total) return fail(SG_EINVAL, "cells and total are both null");
    if (mu_index < 0 || mu_index >= h->n_mu) return fail(SG_EINVAL, "mu_index out of range");
    const hipStream_t s = (hipStream_t)hip_stream;
    const long long nc = h->lv[0].g.n_cells;
    if (h->form_cells.n < (size_t)nc) SG_TRY(h->form_cells.alloc((size_t)nc, "cell forms"));
    SG_TRY(form_cells(h, mu_index, coef_qp, lam, u, h->form_cells.p, s));
    SG_HIP(launch_form_accumulate(h->form_cells.p, nc, scale, cells, total, s));
    return SG_OK;
}

sg_status sg_qoi_mean_var(sg_handle h, const double* u, double w_mean, double w_var, double* qoi, double* grad,
                          void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !u || !qoi) return fail(SG_EINVAL, "null argument");
    if (h->d.n_samples > 0 || h->d.n_members > 0)
        return fail(SG_EUNSUPPORTED, "the chaos QoI needs a single stochastic Galerkin problem");
    if (grad && overlap(u, grad, h->N * sizeof(double))) return fail(SG_EINVAL, "u and grad overlap");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nx = h->n_xi, NT = h->NT, r = NT - 1;
    const long long nn = h->lv[0].g.n_nodes, ld = (long long)NT * nn;
    SG_TRY(zero_coef(h, s));
    // w = (I (x) e_r e_r^T (x) M_x) u: the mass-weighted end-of-slab trace, Dirichlet rows 0
    std::vector<double> err((size_t)NT * NT, 0.0);
    err[(size_t)r * NT + r] = 1.0;
    const Tables<double> tb = tables_with(h, err);
    double* w = h->w1.p;
    SG_TRY(variant_apply(h, &tb, h->zcoef.p, false, u, w, GATHER_INTERIOR, s));
    if (h->qpart.n < (size_t)kDotBlocks * nx) SG_TRY(h->qpart.alloc((size_t)kDotBlocks * nx, "QoI partials"));
    if (h->qout.n < (size_t)nx * nx) SG_TRY(h->qout.alloc((size_t)nx * nx, "QoI Gram matrix"));
    if (h->qC.n < (size_t)nx * nx) SG_TRY(h->qC.alloc((size_t)nx * nx, "QoI gradient weights"));
    // Gram matrix m[b][a] = u_a(T) . (M_x u_b(T))
    for (int b = 0; b < nx; ++b) {
        SG_HIP(launch_multidot(u + (long long)r * nn, ld, nx, w + ((long long)b * NT + r) * nn, nn, h->qpart.p,
                               kDotBlocks, s));
        SG_HIP(launch_reduce_partials(h->qpart.p, kDotBlocks, nx, h->qout.p + (size_t)b * nx, s));
    }
    std::vector<double> m((size_t)nx * nx);
    SG_HIP(hipMemcpyAsync(m.data(), h->qout.p, m.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    build_triple_table(h);
    const int ne = h->n_eps;
    std::vector<double> q(ne, 0.0);
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < nx; ++b) {
            const double mab = 0.5 * (m[(size_t)a * nx + b] + m[(size_t)b * nx + a]);
            const double* t = &h->trip[((size_t)a * nx + b) * ne];
            for (int e = 0; e < ne; ++e) q[e] += mab * t[e];
        }
    double var = 0.0;
    for (int e = 1; e < ne; ++e) var += q[e] * q[e];
    qoi[0] = q[0];
    qoi[1] = var;
    if (!grad) return SG_OK;
    // dJ/du_a(T) = sum_d C[a][d] w_d,  C = 2 w_mean I + 4 w_var sum_{eps != 0} q_eps E[Psi_a Psi_d Psi_eps]
    h->hstage.assign((size_t)nx * nx, 0.0);
    for (int a = 0; a < nx; ++a)
        for (int d = 0; d < nx; ++d) {
            const double* t = &h->trip[((size_t)a * nx + d) * ne];
            double c = (a == d) ? 2.0 * w_mean : 0.0;
            for (int e = 1; e < ne; ++e) c += 4.0 * w_var * q[e] * t[e];
            h->hstage[(size_t)a * nx + d] = c;
        }
    SG_HIP(hipMemcpyAsync(h->qC.p, h->hstage.data(), h->hstage.size() * sizeof(double), hipMemcpyHostToDevice, s));
    SG_HIP(launch_fill<double>(grad, 0.0, h->N, s));
    for (int a = 0; a < nx; ++a)
        for (int d0 = 0; d0 < nx; d0 += 64) {
            const int kk = std::min(64, nx - d0);
            SG_HIP(launch_multi_axpy(w + ((long long)d0 * NT + r) * nn, ld, kk, h->qC.p + (size_t)a * nx + d0,
                                     grad + ((long long)a * NT + r) * nn, nn, s));
        }
    SG_HIP(hipStreamSynchronize(s));
    return SG_OK;
}

sg_status sg_gauss_points(const sg_problem_desc* d, int level, int nq1, double* xyz) {
    if (!d || !xyz) return fail(SG_EINVAL, "null argument");
    if (d->dim != 2 && d->dim != 3) return fail(SG_EINVAL, "dim must be 2 or 3");
    if (d->fe_degree < 1 || d->fe_degree > 4 || d->n_cells_1d < 1) return fail(SG_EINVAL, "bad mesh");
    if (nq1 < 1 || nq1 > kMaxQ1) return fail(SG_EINVAL, "nq1 must be in 1..8");
    if (level < 0 || (d->n_cells_1d >> level) < 1 || (d->n_cells_1d % (1 << level)) != 0)
        return fail(SG_EINVAL, "level out of range");
    const int n = d->n_cells_1d >> level, dim = d->dim;
    const double h = (d->hi - d->lo) / n;
    std::vector<double> gw;
    const std::vector<double> gq = gauss_points(nq1, &gw);
    const int NP = ipow_h(nq1, dim);
    long long ncell = 1;
    for (int i = 0; i < dim; ++i) ncell *= n;
    for (long long c = 0; c < ncell; ++c) {
        int cc[3] = {0, 0, 0};
        long long r = c;
        for (int i = 0; i < dim; ++i) { cc[i] = r % n; r /= n; }
        for (int q = 0; q < NP; ++q)
            for (int i = 0, qq = q; i < dim; ++i, qq /= nq1) xyz[(c * NP + q) * dim + i] = d->lo + h * (cc[i] + gq[qq % nq1]);
    }
    return SG_OK;
}

sg_status sg_quadrature_points(const sg_problem_desc* d, int level, double* xyz) {
    if (!d) return fail(SG_EINVAL, "null argument");
    return sg_gauss_points(d, level, d->fe_degree + 1, xyz);
}

sg_status sg_index_set(sg_handle h, int* alpha) {
    if (!h || !alpha) return fail(SG_EINVAL, "null argument");
    if (h->d.n_samples > 0 || h->d.n_members > 0) return fail(SG_EINVAL, "needs a single stochastic Galerkin problem");
    const auto idx = total_degree_set(h->d.n_vars, h->d.chaos_degree);
    for (size_t a = 0; a < idx.size(); ++a)
        for (int m = 0; m < h->d.n_vars; ++m) alpha[a * h->d.n_vars + m] = idx[a][m];
    return SG_OK;
}

sg_status sg_chaos_projection(sg_handle h, int n_src, const int* src_alpha, const double* src_c, double* out) {
    if (!h || (n_src > 0 && (!src_alpha || !src_c)) || !out || n_src < 0) return fail(SG_EINVAL, "bad argument");
    if (h->d.n_samples > 0 || h->d.n_members > 0) return fail(SG_EINVAL, "needs a single stochastic Galerkin problem");
    const int M = h->d.n_vars;
    const auto idx = total_degree_set(M, h->d.chaos_degree);
    for (int k = 0; k < h->n_mu; ++k)
        for (size_t b = 0; b < idx.size(); ++b) {
            double tot = 0.0;
            for (int si = 0; si < n_src; ++si) {
                double v = src_c[si];
                for (int m = 0; m < M && v != 0.0; ++m)
                    v *= hermite_triple_1d(h->coef_mu[(size_t)k * M + m], src_alpha[(size_t)si * M + m], idx[b][m]);
                tot += v;
            }
            out[(size_t)k * idx.size() + b] = tot;
        }
    return SG_OK;
}

sg_status sg_time_rule(sg_handle h, int ntq, double* s, double* w) {
    if (!h || !s || !w) return fail(SG_EINVAL, "null argument");
    if (ntq < 1 || ntq > kMaxTimeQ) return fail(SG_EINVAL, "ntq must be in 1..8");
    std::vector<double> gw;
    const std::vector<double> gq = gauss_points(ntq, &gw);
    for (int k = 0; k < ntq; ++k) {
        s[k] = gq[k];
        w[k] = gw[k] * h->d.tau;
    }
    return SG_OK;
}

sg_status sg_time_load_weights(sg_handle h, int ntq, int n_g, const double* gvals, double* out) {
    if (!h || !gvals || !out) return fail(SG_EINVAL, "null argument");
    if (ntq < 1 || ntq > kMaxTimeQ || n_g < 0) return fail(SG_EINVAL, "ntq must be in 1..8");
    std::vector<double> gw;
    const std::vector<double> gq = gauss_points(ntq, &gw);
    const std::vector<double> tn = right_radau_points(h->d.time_degree);
    for (int g = 0; g < n_g; ++g)
        for (int i = 0; i < h->NT; ++i) {
            double acc = 0.0;
            for (int k = 0; k < ntq; ++k) acc += gw[k] * h->d.tau * gvals[(size_t)g * ntq + k] * lagrange_value(tn, i, gq[k]);
            out[(size_t)g * h->NT + i] = acc;
        }
    return SG_OK;
}

namespace {
QTables make_qtables(int k, int nq1) {
    QTables tb{};
    std::vector<double> gw;
    const std::vector<double> gq = gauss_points(nq1, &gw);
    const std::vector<double> gll = gll_points(k);
    for (int q = 0; q < nq1; ++q) {
        tb.w[q] = gw[q];
        for (int a = 0; a <= k; ++a) {
            tb.V[q][a] = lagrange_value(gll, a, gq[q]);
            tb.D[q][a] = lagrange_deriv(gll, a, gq[q]);
        }
    }
    return tb;
}
}  // namespace

sg_status sg_load_vectors(sg_handle h, int nq1, int n_fields, const double* fval, const double* fgrad, double* out,
                          void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !out || n_fields < 0) return fail(SG_EINVAL, "bad argument");
    if (nq1 < 1 || nq1 > kMaxQ1) return fail(SG_EINVAL, "nq1 must be in 1..8");
    if (n_fields == 0) return SG_OK;
    const hipStream_t s = (hipStream_t)hip_stream;
    const Level& l0 = h->lv[0];
    const QTables tb = make_qtables(h->d.fe_degree, nq1);
    const int cap = h->n_xi * h->NT;          // fields per pass through the broken-node buffer
    const long long nq = ipow_h(nq1, h->d.dim);
    for (int f0 = 0; f0 < n_fields; f0 += cap) {
        const int nf = std::min(cap, n_fields - f0);
        const long long off = (long long)f0 * l0.g.n_cells * nq;
        SG_HIP(launch_load_cells(h->d.dim, h->d.fe_degree, l0.g, nq1, tb, l0.h, fval ? fval + off : nullptr,
                                 fgrad ? fgrad + off * h->d.dim : nullptr, nf, h->sbuf.p, s));
        SG_HIP(launch_node_gather<double>(GATHER_INTERIOR, h->d.dim, h->d.fe_degree, l0.g, nf, h->sbuf.p, nullptr,
                                          nullptr, out + (long long)f0 * l0.g.n_nodes, 0.0, h->d.fe_degree,
                                          h->d.fe_degree, s));
    }
    return SG_OK;
}

sg_status sg_separable_vector(sg_handle h, int n_terms, const double* W, const double* V, double beta, double* y,
                              void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !y || n_terms < 0 || (n_terms > 0 && (!W || !V))) return fail(SG_EINVAL, "bad argument");
    const hipStream_t s = (hipStream_t)hip_stream;
    const size_t nw = (size_t)std::max(n_terms, 1) * h->n_xi * h->NT;
    SG_TRY(h->sepW.alloc(nw, "separable weights"));
    SG_HIP(hipStreamSynchronize(s));            // the previous call's kernel may still read sepW
    if (n_terms > 0) SG_HIP(hipMemcpy(h->sepW.p, W, sizeof(double) * n_terms * h->n_xi * h->NT, hipMemcpyHostToDevice));
    SG_HIP(launch_separable(n_terms, h->n_xi * h->NT, h->lv[0].g.n_nodes, h->sepW.p, V, beta, y, s));
    return SG_OK;
}

sg_status sg_separable_error(sg_handle h, const double* u, int nq1, const double* s_qp, const double* gs_qp, int ntq,
                             const double* theta, const double* c, double C2, double* out, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !u || !s_qp || !gs_qp || !theta || !c || !out) return fail(SG_EINVAL, "null argument");
    if (nq1 < 1 || nq1 > kMaxQ1 || ntq < 1 || ntq > kMaxTimeQ) return fail(SG_EINVAL, "nq1 and ntq must be in 1..8");
    if (h->d.n_samples > 0 || h->d.n_members > 0) return fail(SG_EINVAL, "needs a single stochastic Galerkin problem");
    if (!error_cells_supported(h->d.dim, h->d.fe_degree, h->NT))
        return fail(SG_EUNSUPPORTED, "error sums: 2D k <= 4 or 3D k <= 2, dG(r) with r <= 3");
    const size_t lds = (size_t)h->n_xi * h->NT * h->NP * sizeof(double);
    if (lds > 160 * 1024) return fail(SG_EUNSUPPORTED, "error sums: N_xi * N_t * (k+1)^d values exceed one LDS");
    const hipStream_t s = (hipStream_t)hip_stream;
    const Level& l0 = h->lv[0];
    const QTables tb = make_qtables(h->d.fe_degree, nq1);
    TimeTables tt{};
    tt.ntq = ntq;
    {
        std::vector<double> gw;
        const std::vector<double> gq = gauss_points(ntq, &gw);
        const std::vector<double> tn = right_radau_points(h->d.time_degree);
        for (int k = 0; k < ntq; ++k) {
            tt.w[k] = gw[k] * h->d.tau;
            tt.theta[k] = theta[k];
            for (int i = 0; i < h->NT; ++i) tt.v[i][k] = lagrange_value(tn, i, gq[k]);
        }
    }
    SG_TRY(h->errC.alloc((size_t)h->n_xi, "error sums"));
    SG_TRY(h->errPart.alloc((size_t)l0.g.n_cells * 8, "error sums"));
    SG_TRY(h->errOut.alloc(8, "error sums"));
    SG_HIP(hipStreamSynchronize(s));
    SG_HIP(hipMemcpy(h->errC.p, c, sizeof(double) * h->n_xi, hipMemcpyHostToDevice));
    SG_HIP(launch_error_cells(h->d.dim, h->d.fe_degree, h->NT, l0.g, nq1, tb, l0.h, tt, h->n_xi, u, h->errC.p, C2, s_qp,
                              gs_qp, h->errPart.p, s));
    SG_HIP(launch_reduce_partials(h->errPart.p, (int)l0.g.n_cells, 8, h->errOut.p, s));
    SG_HIP(hipMemcpyAsync(out, h->errOut.p, sizeof(double) * 8, hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    return SG_OK;
}

namespace {
TimeTables make_ttables(sg_handle h, int ntq, const double* theta) {
    TimeTables tt{};
    tt.ntq = ntq;
    std::vector<double> gw;
    const std::vector<double> gq = gauss_points(ntq, &gw);
    const std::vector<double> tn = right_radau_points(h->d.time_degree);
    for (int k = 0; k < ntq; ++k) {
        tt.w[k] = gw[k] * h->d.tau;
        tt.theta[k] = theta ? theta[k] : 0.0;
        for (int i = 0; i < h->NT; ++i) tt.v[i][k] = lagrange_value(tn, i, gq[k]);
    }
    return tt;
}
}  // namespace

sg_status sg_sample_psi(sg_handle h, int n_idx, const int* alpha, double* out) {
    if (!h || !alpha || !out || n_idx < 0) return fail(SG_EINVAL, "bad argument");
    if (h->d.n_samples < 1) return fail(SG_EINVAL, "not a sample-batch handle");
    const int M = h->d.n_vars;
    for (int sm = 0; sm < h->d.n_samples; ++sm)
        for (int j = 0; j < n_idx; ++j) {
            double v = 1.0;
            for (int m = 0; m < M; ++m) v *= hermite_normalized(alpha[(size_t)j * M + m], h->samples[(size_t)sm * M + m]);
            out[(size_t)sm * n_idx + j] = v;
        }
    return SG_OK;
}

sg_status sg_sample_qp_moments(sg_handle h, const double* u, int nq1, int ntq, double* acc, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !u || !acc) return fail(SG_EINVAL, "null argument");
    if (h->d.n_samples < 1) return fail(SG_EINVAL, "not a sample-batch handle");
    if (nq1 < 1 || nq1 > kMaxQ1 || ntq < 1 || ntq > kMaxTimeQ) return fail(SG_EINVAL, "nq1 and ntq must be in 1..8");
    if (!error_cells_supported(h->d.dim, h->d.fe_degree, h->NT))
        return fail(SG_EUNSUPPORTED, "sample moments: 2D k <= 4 or 3D k <= 2, dG(r) with r <= 3");
    if ((size_t)h->n_xi * h->NT * h->NP * sizeof(double) > 160 * 1024)
        return fail(SG_EUNSUPPORTED, "sample moments: n_samples * N_t * (k+1)^d values exceed one LDS");
    const QTables tb = make_qtables(h->d.fe_degree, nq1);
    const TimeTables tt = make_ttables(h, ntq, nullptr);
    SG_HIP(launch_sample_qp_moments(h->d.dim, h->d.fe_degree, h->NT, h->lv[0].g, nq1, tb, tt, h->n_xi, u, acc,
                                    (hipStream_t)hip_stream));
    return SG_OK;
}

sg_status sg_moment_errors(sg_handle h, const double* acc, long long n_tot, int nq1, const double* s_qp, int ntq,
                           const double* theta, const double* mean_targets, const double* var_targets, double* out,
                           void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !acc || !s_qp || !theta || !mean_targets || !var_targets || !out) return fail(SG_EINVAL, "null argument");
    if (n_tot < 2) return fail(SG_EINVAL, "the unbiased variance needs at least two samples");
    if (nq1 < 1 || nq1 > kMaxQ1 || ntq < 1 || ntq > kMaxTimeQ) return fail(SG_EINVAL, "nq1 and ntq must be in 1..8");
    const hipStream_t s = (hipStream_t)hip_stream;
    const Level& l0 = h->lv[0];
    const QTables tb = make_qtables(h->d.fe_degree, nq1);
    const TimeTables tt = make_ttables(h, ntq, theta);
    SG_TRY(h->momPart.alloc((size_t)l0.g.n_cells * 6, "moment errors"));
    SG_TRY(h->errOut.alloc(8, "moment errors"));
    SG_HIP(launch_moment_errors(h->d.dim, l0.g, nq1, tb, l0.h, tt, (double)n_tot, acc, s_qp, mean_targets[0],
                                mean_targets[1], var_targets[0], var_targets[1], h->momPart.p, s));
    SG_HIP(launch_reduce_partials(h->momPart.p, (int)l0.g.n_cells, 6, h->errOut.p, s));
    SG_HIP(hipMemcpyAsync(out, h->errOut.p, sizeof(double) * 6, hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
    return SG_OK;
}

sg_status sg_set_vcycle_segment(sg_handle h, int enable, int* first_level) {
    if (!h || enable < -1 || enable > 1) return fail(SG_EINVAL, "bad argument");
    if (first_level) *first_level = enable == -1 && !h->seg_on ? -1 : h->seg_level;
    if (enable == -1) return SG_OK;
    h->quiesce();
    h->drop_graph();                           // a captured V-cycle holds the other path
    h->seg_on = enable == 1;
    return SG_OK;
}

sg_status sg_set_vcycle_graph(sg_handle h, int enable) {
    if (!h || (enable != 0 && enable != 1)) return fail(SG_EINVAL, "bad argument");
    if (!enable) {
        h->quiesce();
        h->drop_graph();
    }
    h->graph_on = enable == 1;
    return SG_OK;
}

sg_status sg_autotune(sg_handle h, int reps, int* cpb_out, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h) return fail(SG_EINVAL, "null argument");
    if (reps < 1 || reps > 1000) return fail(SG_EINVAL, "reps must be in 1..1000");
    const hipStream_t s = (hipStream_t)hip_stream;
    const int L = std::min(h->d.n_levels, 16);
    SG_HIP(hipStreamSynchronize(s));
    h->drop_graph();                           // a captured V-cycle would keep the old tiles
    SG_TRY(autotune_apply<double>(h, 0, true, reps, s));
    for (int l = 0; l < L; ++l) SG_TRY(autotune_apply<double>(h, l, false, reps, s));
    if (h->mixed)
        for (int l = 0; l < L; ++l) SG_TRY(autotune_apply<float>(h, l, false, reps, s));
    SG_TRY(autotune_segment(h, reps, s));
    if (cpb_out)
        for (int p = 0; p < 2; ++p)
            for (int f = 0; f < 2; ++f)
                for (int l = 0; l < h->d.n_levels; ++l)
                    cpb_out[(p * 2 + f) * h->d.n_levels + l] = l < 16 ? h->tuned_cpb[p][f][l] : 0;
    return SG_OK;
}

sg_status sg_sample_statistics(sg_handle h, const double* u, double* mean, double* var, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !u || !mean) return fail(SG_EINVAL, "null argument");
    if (h->d.n_samples < 1) return fail(SG_EINVAL, "not a sample-batch handle");
    SG_HIP(launch_sample_stats(u, h->d.n_samples, h->NT, h->lv[0].g.n_nodes, mean, var, (hipStream_t)hip_stream));
    return SG_OK;
}

sg_status sg_chaos_moments(sg_handle h, const double* u, double* mean, double* var, void* hip_stream) {
    const WorkMark work_mark{h, (hipStream_t)hip_stream};
    if (!h || !u || !mean) return fail(SG_EINVAL, "null argument");
    if (h->d.n_samples > 0) return fail(SG_EINVAL, "a sample-batch handle has no chaos modes");
    SG_HIP(launch_chaos_moments(u, h->moff.p, (int)h->member_off.size() - 1, h->NT, h->lv[0].g.n_nodes, mean, var,
                                (hipStream_t)hip_stream));
    return SG_OK;
}

sg_status sg_node_coordinates(const sg_problem_desc* d, int level, double* xyz) {
    if (!d || !xyz) return fail(SG_EINVAL, "null argument");
    if (d->dim != 2 && d->dim != 3) return fail(SG_EINVAL, "dim must be 2 or 3");
    if (d->fe_degree < 1 || d->fe_degree > 4 || d->n_cells_1d < 1) return fail(SG_EINVAL, "bad mesh");
    if (level < 0 || (d->n_cells_1d >> level) < 1 || (d->n_cells_1d % (1 << level)) != 0)
        return fail(SG_EINVAL, "level out of range");
    const int n = d->n_cells_1d >> level, k = d->fe_degree, dim = d->dim;
    const int n1 = n * k + 1;
    const double h = (d->hi - d->lo) / n;
    const std::vector<double> gll = gll_points(k);
    std::vector<double> x1(n1);
    for (int i = 0; i < n1; ++i) {
        const int c = std::min(i / k, n - 1);
        x1[i] = d->lo + h * (c + gll[i - c * k]);
    }
    long long nn = 1;
    for (int i = 0; i < dim; ++i) nn *= n1;
    for (long long v = 0; v < nn; ++v) {
        long long r = v;
        for (int i = 0; i < dim; ++i) {
            xyz[v * dim + i] = x1[r % n1];
            r /= n1;
        }
    }
    return SG_OK;
}

const char* sg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
