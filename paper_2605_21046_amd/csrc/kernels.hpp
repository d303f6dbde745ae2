// Launchers of the gfx950 kernels.  Every launcher enqueues on the given stream and returns the
// launch status; argument validity is checked by the caller (sgheat.cpp) before any launch.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace sg {

// ---- slab operator ------------------------------------------------------------------------------
// Cell-local part of y = AA x (or of (I (x) A_0) x when `mean` is set): every cell writes its
// (k+1)^d nodal results per component to s_out in the broken layout
//     s_out[comp][b_z][b_y][b_x],  b_d = c_d (k+1) + a_d  (cell c, local node a),
// which k_node_gather (launch_node_gather) sums per node.
// coef: [n_mu][n_cells][(k+1)^d] values a_mu(x_q) * w_q * h^(d-2).
// Coupling CSR: row alpha * n_mu + mu lists (beta, [G_mu]_{alpha beta}).
template <typename T>
struct ApplyOp {
    int dim, k, nt;
    Grid g;
    int n_xi, n_mu;
    const T* coef;
    long long coef_mode_stride;   // n_cells * (k+1)^d
    const int* cptr;
    const int* cbeta;
    const int* cmu;               // mu index of every entry
    const T* cw;
    const Tables<T>* tables;      // host copy, passed by value to the kernel
    int n_ent;                    // number of coupling entries
    int cells_per_block;          // cells handled by one workgroup (0 = chosen from occupancy)
    bool mean;                    // mean block only: identity coupling with the mean coefficient
    bool affine;                  // coefficient modes are mu = 0 and mu = e_m only
    int chaos_m, chaos_p;         // M and p_xi of the total-degree index set
    int mu0;                      // position of mu = 0 in the coefficient list
    int mum[8];                   // position of mu = e_m in the coefficient list (-1 if absent)
    int merge;                    // 1: the cells of a workgroup sum their shared x faces before storing
                                  // (broken along x only between workgroups: segments of cpb cells)
    int* used_cpb;                // if set, receives the cells per workgroup of the launch
    int lz;                       // 3D, merged layout: cells per z chunk a workgroup marches through
                                  // (0 = chosen from the mesh size; the z faces inside a chunk are summed
                                  // in registers, so the broken layout is chunked along z as along x)
    int* used_lz;                 // if set, receives the z chunk length of the launch
    int level;                    // multigrid level of the operator
};
template <typename T>
hipError_t launch_apply(const ApplyOp<T>& op, const T* x, T* s_out, hipStream_t s);
// Length in node intervals of one broken x segment of an apply's output (k: per cell; cpb k: merged).
template <typename T>
inline int apply_segment(const ApplyOp<T>& op, int cpb) { return op.merge && cpb > 1 ? cpb * op.k : op.k; }
// The same along z (lz k; k for the per-cell layout).
template <typename T>
inline int apply_zsegment(const ApplyOp<T>& op, int lz) { return lz * op.k; }

// Sum of the broken copies of every node, then one of (sx, sz: length of a broken segment along x and
// along z in node intervals; k for the per-cell layout, cpb k (x) and lz k (z) for an apply whose
// workgroups merged their x faces and marched through z chunks)
//   GATHER_SET:      out = sum                 (Dirichlet rows: out = x)
//   GATHER_RESIDUAL: out = b - sum             (Dirichlet rows: out = b - x)
//   GATHER_VANKA:    out += omega sum / mult   (Dirichlet rows: out = b); mult = cells sharing the node
//   GATHER_INTERIOR: out = sum                 (Dirichlet rows: out = 0)
enum GatherOp { GATHER_SET = 0, GATHER_RESIDUAL = 1, GATHER_VANKA = 2, GATHER_INTERIOR = 3 };

// out[K] = sum over the ncomp components and the (k+1)^d local nodes a of cell K of
// lam[comp][node(K, a)] * s_in[comp][broken(K, a)]: the cell-wise bilinear form lam^T A_K u of a
// cell-local operator whose per-cell results s_in = A_K u are in the broken layout.
hipError_t launch_cell_dot(int dim, int k, Grid g, int ncomp, const double* lam, const double* s_in, double* out,
                           hipStream_t s);
// cells[K] += scale form[K] (cells may be null) and total[0] += scale sum_K form[K] (total may be null),
// the sum taken in one fixed order by one workgroup
hipError_t launch_form_accumulate(const double* form, long long n, double scale, double* cells, double* total,
                                  hipStream_t s);

// mean[i][node] and unbiased var[i][node] over N sample blocks of a slab vector u[N][nt][nn]
// mean[j][i][node] = u[off[j]][i][node], var = sum_{off[j] < a < off[j+1]} u[a][i][node]^2
hipError_t launch_chaos_moments(const double* u, const int* off, int n_members, int nt, long long nn, double* mean,
                                double* var, hipStream_t s);

hipError_t launch_sample_stats(const double* u, int N, int nt, long long nn, double* mean, double* var,
                               hipStream_t s);
template <typename T>
hipError_t launch_node_gather(GatherOp op, int dim, int k, Grid g, int ncomp, const T* s_in, const T* x, const T* b,
                              T* out, T omega, int sx, int sz, hipStream_t s);

// ---- Vanka -----------------------------------------------------------------------------------------
// Element stiffness of the mean coefficient: E[cell][a][b] = sum_q c0(cell,q) sum_d dphi_a dphi_b.
struct ElemTables {
    double S[kMaxN1 * kMaxN1];    // l_a(g_q)
    double Dn[kMaxN1 * kMaxN1];   // l_a'(g_q)
};
hipError_t launch_elem_stiffness(int dim, int k, Grid g, const double* coef0, const ElemTables& et,
                                 double* E, hipStream_t s);

// Form every patch matrix A_{0,K} = A_t (x) M_K + B_t (x) K_K (restrictions of the assembled
// matrices; Dirichlet local DoFs replaced by identity rows and columns), invert it by Gauss-Jordan
// elimination with partial pivoting in FP64, and store the inverse in FP64 and/or FP32.
struct PatchTime {
    double At[kMaxNT * kMaxNT];
    double Bt[kMaxNT];
};
// In-place inverse of a dense n x n FP64 matrix A (row-major) by Gauss-Jordan elimination with
// partial pivoting, then its transpose into AinvT (column-major inverse, for coalesced reads of the
// coarse solve).  Scratch: col[n], perm[n]; status is set to 1 if a pivot is zero.  2n + 2 launches.
hipError_t launch_dense_invert(double* A, int n, double* col, int* perm, int* status, double* AinvT, hipStream_t s);
// cells == nullptr: every cell's patch, inverse slot = cell index; else the n_list patches of the
// listed cells, inverse slot = position in the list.
hipError_t launch_patch_invert(int dim, int k, int nt, Grid g, const double* E, const double* Me,
                               const PatchTime& pt, double* inv64, float* inv32, int* status,
                               hipStream_t s, const int* cells = nullptr, int n_list = 0);

// Inverse slot of a cell: the cell itself, or with position classes (a level whose patch matrices
// depend only on where the cell sits: constant coefficient on a uniform mesh) one of 3^d slots,
// sum_d 3^d c_d with c_d = 0 for the first cell along d, 2 for the last and 1 between (n >= 2).
template <int DIM>
__host__ __device__ inline long long inverse_slot(long long cell, const int* cc, int n, int classes) {
    if (!classes) return cell;
    long long slot = 0, m = 1;
    for (int d = 0; d < DIM; ++d) {
        slot += m * (cc[d] == 0 ? 0 : (cc[d] == n - 1 ? 2 : 1));
        m *= 3;
    }
    return slot;
}

// Storage of one cell's patch inverse (n_p x n_p) for the patch products below: B[c][I] = A^{-1}[I][c]
// (c: the k index of the product, I: the patch row), in fragments so that the `spl` consecutive
// k-steps (4 columns each) one lane consumes are contiguous: element (c, I) is at
//     ((g * 4 + c % 4) * n_p + I) * spl + (c / 4) % spl,   g = c / (4 spl),
// with 4 ceil(n_p / 4) columns per cell (zero beyond n_p).  spl: the largest of 4, 2, 1 dividing the
// k-step count with spl values in at most 16 bytes (one vector load per lane and fragment).
constexpr int vanka_ksteps(int npp) { return (npp + 3) / 4; }
constexpr int vanka_spl(int npp, int elem) {
    return (vanka_ksteps(npp) % 4 == 0 && 4 * elem <= 16) ? 4 : ((vanka_ksteps(npp) % 2 == 0 && 2 * elem <= 16) ? 2 : 1);
}
__host__ __device__ constexpr long long vanka_inv_stride(int npp) { return 4LL * vanka_ksteps(npp) * npp; }
__host__ __device__ inline long long vanka_inv_offset(int npp, int spl, int c, int I) {
    const int st = c / 4, kk = c % 4;
    return ((long long)((st / spl) * 4 + kk) * npp + I) * spl + st % spl;
}

// Patch corrections c_K = A_{0,K}^{-1} R_K r of every cell (inverses in the fragment layout), written to
// s_out in the broken layout; launch_node_gather(GATHER_VANKA) then forms
// x <- x + omega sum_K R_K^T W_K c_K.  The residual patch of a cell (48 modes at a time) takes
// ceil(n_p / 4) * 4 * 49 * sizeof(T) bytes of LDS.
inline size_t vanka_lds_bytes(int npp, size_t elem) { return (size_t)((npp + 3) / 4 * 4) * 49 * elem; }
// classes: 1 when the level stores one inverse per position class (inverse_slot), 0 for one per cell.
template <typename T>
hipError_t launch_vanka_cells(int dim, int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out,
                              int classes, hipStream_t s);
// the same with one inverse per (mode, cell): invT [n_xi][n_cells][vanka_inv_stride(n_p)]
template <typename T>
hipError_t launch_vanka_cells_modes(int dim, int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out,
                                    hipStream_t s);

// The same corrections for a level whose mean coefficient is one constant, by fast diagonalisation of
// the Kronecker-structured patch matrices (kernels_vanka.hip): Sv [3][k+1][k+1] per-direction
// transforms of the first / inner / last cell, Tt [3^d][(k+1)^d][N_t][N_t] inverted time blocks per
// position class.  The modes go through LDS in passes of vanka_fdm_modes_per_pass.
constexpr int kFdmLdsBudget = 32 * 1024;   // LDS per workgroup aimed at (several workgroups per CU)
// LDS stride of one component: (k+1)^(d-1) x-lines of odd length (k+1) | 1
inline int vanka_fdm_component_stride(int dim, int k) {
    int nl = 1;
    for (int d = 1; d < dim; ++d) nl *= k + 1;
    return nl * ((k + 1) | 1);
}
inline int vanka_fdm_modes_per_pass(int dim, int k, int nt, int n_xi, size_t elem) {
    int np = 1;
    for (int d = 0; d < dim; ++d) np *= k + 1;
    const long long per_mode = (long long)nt * vanka_fdm_component_stride(dim, k) * (long long)elem;
    const long long tab = (long long)np * nt * nt * (long long)elem;
    long long mmax = (kFdmLdsBudget - tab) / per_mode;
    if (mmax < 1) mmax = 1;
    const long long passes = (n_xi + mmax - 1) / mmax;
    return (int)((n_xi + passes - 1) / passes);
}
inline size_t vanka_fdm_lds_bytes(int dim, int k, int nt, int mp, size_t elem) {
    int np = 1;
    for (int d = 0; d < dim; ++d) np *= k + 1;
    return ((size_t)np * nt * nt + (size_t)mp * nt * vanka_fdm_component_stride(dim, k)) * elem;
}
// sx receives the x segment length of the broken layout written, for the gather: k (one entry per cell
// and local node) or n k (one entry per node along x, the register form summing the shared x faces).
template <typename T>
hipError_t launch_vanka_fdm(int dim, int k, int nt, Grid g, int n_xi, const T* Sv, const T* Tt, const T* r,
                            T* s_out, int* sx, hipStream_t s);

// ---- the coarse segment of the V-cycle in one launch ----------------------------------------------------
// Levels l0 .. l0 + nlev - 1 (the last is the coarsest) of the block-Jacobi cycle with the mean block, one
// workgroup per stochastic mode (kernels_segment.hip).  Vectors are the levels' [n_xi][N_t][n_nodes]
// buffers (b of the first level is the segment's right-hand side, x of the first level its result);
// every pointer is a device pointer of the precision T of the launch (E, Me and the coarsest inverse FP64).
constexpr int kSegMaxLevels = 4;
struct SegLevelArgs {
    Grid g;
    const void* inv;           // Vanka patch inverses (fragment layout), T
    int classes;               // inverse per position class (inverse_slot) or per cell
    const double* E;           // element stiffness of the mean coefficient [n_cells][(k+1)^d][(k+1)^d]
    const double* Me;          // element mass [(k+1)^d][(k+1)^d]
    const int* r_idx;          // restriction to the next level: banded 1D tables (T weights)
    const void* r_w;
    int wr;
    const int* p_idx;          // prolongation from the next level
    const void* p_w;
    int wp;
    void* b;                   // level vectors (b of the first level is only read)
    void* x;
    void* r;
    int lds_b, lds_x, lds_r;   // byte offsets of the on-chip copies in LDS (-1: used in place), set at launch
    int lds_E, lds_Me, lds_inv;  // on-chip copies of E (one cell's, when the level has position classes),
                                 // Me and the class inverses; set at launch
};
struct SegArgs {
    int dim, k, nt, np, n_xi, nlev;
    SegLevelArgs lv[kSegMaxLevels];
    double At[kMaxNT * kMaxNT], Bt[kMaxNT];
    double omega;
    int pre, post;
    const double* coarse_invT;   // [nint][nint], column-major inverse of A_0 on the coarsest interior DoFs
    int nint;
    const int* coarse_dofs;      // interior DoFs of one mode on the coarsest level
    void* scratch;               // scratch_per_mode elements of T per mode
    long long scratch_per_mode;
    long long tmp_len;           // one transfer temporary (elements of T)
    int lds_G, lds_C, lds_t0, lds_t1, lds_bytes;   // LDS placement, set at launch
    int coarse_split;            // partial sums per coarsest row, set at launch
};
long long segment_scratch_per_mode(int nt, int np, long long cells0, long long tmp_len);

template <typename T>
hipError_t launch_vcycle_segment(const SegArgs& a, hipStream_t s);

// ---- the mean block as a Kronecker sum (constant mean coefficient) ----------------------------------
// y = A_0 x (b == nullptr; Dirichlet rows y = x) or y = b - A_0 x (Dirichlet rows b - x) on every mode of
// one level, A_0 = A_t (x) M + B_t (x) K_0 with M and K_0 formed from the assembled 1D mass and stiffness
// matrices in band storage, band[i][d] = M1[i][i - k + d] (zero beyond the mesh), the stiffness band
// already multiplied by the constant mean coefficient (kernels_stencil.hip).  Vectors [n_xi][N_t][n1^d].
struct StencilArgs {
    int dim, k, nt, n1, n_xi;
    const void* Mb;          // [n1][2k+1], T
    const void* Kb;          // [n1][2k+1], T
    double At[kMaxNT * kMaxNT], Bt[kMaxNT];
    const void* x;
    const void* b;           // nullptr: y = A_0 x
    void* y;
    int ty, zc;              // rows per workgroup and z planes per workgroup (set at launch)
    int mode;                // set inside the kernel
};
size_t stencil_lds_bytes(const StencilArgs& a, int elem);
// Chooses the rows per workgroup; false when no tile fits (the element route applies then).
bool stencil_fits(StencilArgs& a, int elem);
template <typename T>
hipError_t launch_mean_stencil(const StencilArgs& a, hipStream_t s);

// ---- transfers ---------------------------------------------------------------------------------------
// One 1D pass along `dir`: out[c][.., o, ..] (+)= sum_w tw[o*width + w] in[c][.., tidx[o*width + w], ..]
template <typename T>
hipError_t launch_transfer_1d(int dim, int ncomp, const int* in_dims, const int* out_dims, int dir,
                              const int* tidx, const T* tw, int width, const T* in, T* out,
                              bool accumulate, hipStream_t s);

// ---- coarsest level ------------------------------------------------------------------------------
// x = b, then on interior DoFs x[alpha][dof_r] = sum_l AinvT[l][r] b[alpha][dof_l] in FP64.
template <typename T>
hipError_t launch_coarse_solve(const double* AinvT, long long inv_stride, int nint, const int* dofs, int n_xi,
                               long long mode_len, const T* b, T* x, hipStream_t s);

// ---- vector kernels (FP64 unless noted) -----------------------------------------------------------
hipError_t launch_multidot(const double* V, long long ldv, int k, const double* w, long long n,
                           double* partial, int nblk, hipStream_t s);
// wout = w - sum_j h[j] V[j] (j < k) with, by mode: partial sums of V[j]^T wout and of |wout|^2
// (partial[blk][k + 1]); of |wout|^2 only (partial[blk]); or none, wout divided by
// sqrt(h[k] - sum_j h[j]^2) (the norm by Pythagoras when h[k] = |w|^2 and V is orthonormal)
constexpr int kUpdDotNorm = 0, kUpdNorm = 1, kUpdScaled = 2;
hipError_t launch_update_dot(const double* V, long long ldv, int k, const double* h, const double* w,
                             double* wout, long long n, double* partial, int nblk, int mode,
                             hipStream_t s);
hipError_t launch_reduce_partials(const double* partial, int nblk, int k, double* out, hipStream_t s);
hipError_t launch_multi_axpy(const double* V, long long ldv, int k, const double* y, double* x,
                             long long n, hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* out,
                        long long n, hipStream_t s);     // out = a x + b y
template <typename S, typename D>
hipError_t launch_convert(const S* in, D* out, long long n, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* out, T v, long long n, hipStream_t s);

constexpr int kDotBlocks = 1024;   // fixed partial-sum count: reductions are deterministic

}  // namespace sg
