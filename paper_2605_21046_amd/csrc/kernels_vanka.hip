// Vanka patch smoother (Remark solver-matrix-free-sg: local dense patch problems on space-time
// patches).  Patch of cell K = every local node of the closed cell x all N_t time DoFs; the patch
// matrix is the restriction of the assembled mean block A_0 = A_t (x) M_x + B_t (x) K_{a_0}, with
// Dirichlet local DoFs replaced by identity rows and columns.
//
//   k_elem_stiffness : element stiffness matrices of the mean coefficient (one thread per entry)
//   k_patch_invert   : forms A_{0,K} from the element matrices of every cell sharing the node pair,
//                      inverts it by Gauss-Jordan elimination with partial pivoting, FP64, with the
//                      matrix distributed over a TG x TG thread grid (R x R entries per thread)
//   k_vanka_cells    : c_K = A_{0,K}^{-1} R_K r for every cell, into the broken node array; the
//                      node gather then forms x <- x + omega sum_K R_K^T W_K c_K
#include "kernels.hpp"

#include <cstdlib>
#include <cstring>


namespace sg {

namespace {

__device__ __forceinline__ int digit(int v, int n1, int d) {
    for (int i = 0; i < d; ++i) v /= n1;
    return v % n1;
}

// ------------------------------------------------------------------------------------------------
__global__ void k_elem_stiffness(int dim, int k, Grid g, const double* __restrict__ coef0, ElemTables et,
                                 double* __restrict__ E) {
    const int N1 = k + 1;
    const int NP = dim == 2 ? N1 * N1 : N1 * N1 * N1;
    const long long total = g.n_cells * NP * NP;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int bb = idx % NP;
        const int aa = (idx / NP) % NP;
        const long long cell = idx / ((long long)NP * NP);
        double s = 0.0;
        for (int q = 0; q < NP; ++q) {
            double gsum = 0.0;
            for (int e = 0; e < dim; ++e) {
                double va = 1.0, vb = 1.0;
                for (int d = 0; d < dim; ++d) {
                    const int qd = digit(q, N1, d), ad = digit(aa, N1, d), bd = digit(bb, N1, d);
                    va *= (d == e) ? et.Dn[qd * N1 + ad] : et.S[qd * N1 + ad];
                    vb *= (d == e) ? et.Dn[qd * N1 + bd] : et.S[qd * N1 + bd];
                }
                gsum += va * vb;
            }
            s += coef0[cell * NP + q] * gsum;
        }
        E[idx] = s;
    }
}

// ------------------------------------------------------------------------------------------------
// Assembled value of (mass, stiffness) between local nodes a and b of cell cc: sum over every cell
// whose closure contains both nodes.
__device__ void assembled_pair(int dim, int k, const Grid& g, const int* cc, int a, int b,
                               const double* __restrict__ E, const double* __restrict__ Me,
                               double* m_out, double* k_out) {
    const int N1 = k + 1;
    const int NP = dim == 2 ? N1 * N1 : N1 * N1 * N1;
    int opt[3][2], nopt[3];
    for (int d = 0; d < 3; ++d) {
        opt[d][0] = 0;
        nopt[d] = 1;
        if (d >= dim) continue;
        const int ad = digit(a, N1, d), bd = digit(b, N1, d);
        if (ad == 0 && bd == 0 && cc[d] > 0) { opt[d][1] = -1; nopt[d] = 2; }
        if (ad == k && bd == k && cc[d] < g.n - 1) { opt[d][1] = +1; nopt[d] = 2; }
    }
    double ms = 0.0, ks = 0.0;
    for (int i0 = 0; i0 < nopt[0]; ++i0)
        for (int i1 = 0; i1 < nopt[1]; ++i1)
            for (int i2 = 0; i2 < nopt[2]; ++i2) {
                const int sh[3] = {opt[0][i0], opt[1][i1], opt[2][i2]};
                long long cell = 0, mul = 1;
                int la = 0, lb = 0, lmul = 1;
                for (int d = 0; d < dim; ++d) {
                    cell += (long long)(cc[d] + sh[d]) * mul;
                    mul *= g.n;
                    int ad = digit(a, N1, d), bd = digit(b, N1, d);
                    if (sh[d] == -1) { ad = k; bd = k; }
                    if (sh[d] == +1) { ad = 0; bd = 0; }
                    la += ad * lmul;
                    lb += bd * lmul;
                    lmul *= N1;
                }
                ms += Me[la * NP + lb];
                ks += E[(cell * NP + la) * NP + lb];
            }
    *m_out = ms;
    *k_out = ks;
}

template <int TG, int R>
__global__ void __launch_bounds__(TG * TG)
    k_patch_invert(int dim, int k, int nt, Grid g, const double* __restrict__ E, const double* __restrict__ Me,
                   PatchTime pt, double* __restrict__ inv64, float* __restrict__ inv32, int* status,
                   const int* __restrict__ cells) {
    constexpr int NPAD = TG * R;
    __shared__ double prow[NPAD], pcol[NPAD];
    __shared__ double cval[TG];
    __shared__ int crow[TG];
    __shared__ int perm[NPAD];
    __shared__ int sigma_inv[NPAD];
    __shared__ int piv_row;
    __shared__ double piv_val;

    const int N1 = k + 1;
    const int NP = dim == 2 ? N1 * N1 : N1 * N1 * N1;
    const int npp = nt * NP;
    // the patch of cell `cell`, stored in inverse slot `slot` (a cell list inverts representatives only)
    const long long slot = blockIdx.x;
    const long long cell = cells ? cells[slot] : slot;
    int cc[3] = {0, 0, 0};
    {
        long long r = cell;
        for (int d = 0; d < dim; ++d) { cc[d] = r % g.n; r /= g.n; }
    }
    const int tx = threadIdx.x % TG, ty = threadIdx.x / TG;

    // local DoF l = i * NP + p; Dirichlet if node p of this cell is on the domain boundary
    auto dirichlet = [&](int p) {
        for (int d = 0; d < dim; ++d) {
            const int id = cc[d] * k + digit(p, N1, d);
            if (id == 0 || id == g.n1 - 1) return true;
        }
        return false;
    };

    double Am[R][R];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int I = ty + TG * r, J = tx + TG * c;
            double v = (I == J) ? 1.0 : 0.0;
            if (I < npp && J < npp) {
                const int i = I / NP, p = I % NP, j = J / NP, q = J % NP;
                if (dirichlet(p) || dirichlet(q)) {
                    v = (I == J) ? 1.0 : 0.0;
                } else {
                    double m, s;
                    assembled_pair(dim, k, g, cc, p, q, E, Me, &m, &s);
                    v = pt.At[i * nt + j] * m + (i == j ? pt.Bt[i] * s : 0.0);
                }
            }
            Am[r][c] = v;
        }

    for (int kk = 0; kk < NPAD; ++kk) {
        const int kr = kk / TG, kt = kk % TG;
        // 1. pivot search in column kk among rows >= kk
        if (tx == kt) {
            double best = -1.0;
            int brow = NPAD;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int I = ty + TG * r;
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < R; ++c) if (c == kr) v = Am[r][c];
                v = fabs(v);
                if (I >= kk && (v > best || (v == best && I < brow))) { best = v; brow = I; }
            }
            cval[ty] = best;
            crow[ty] = brow;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double best = -1.0;
            int brow = NPAD;
            for (int t = 0; t < TG; ++t)
                if (cval[t] > best || (cval[t] == best && crow[t] < brow)) { best = cval[t]; brow = crow[t]; }
            piv_row = brow;
            perm[kk] = brow;
            if (!(best > 0.0)) atomicOr(status, 1);
        }
        __syncthreads();
        const int p = piv_row;
        // 2. swap rows kk and p through LDS
        if (p != kk) {
            if (ty == p % TG) {
#pragma unroll
                for (int c = 0; c < R; ++c)
#pragma unroll
                    for (int r = 0; r < R; ++r) if (r == p / TG) prow[tx + TG * c] = Am[r][c];
            }
            if (ty == kt) {
#pragma unroll
                for (int c = 0; c < R; ++c)
#pragma unroll
                    for (int r = 0; r < R; ++r) if (r == kr) pcol[tx + TG * c] = Am[r][c];
            }
            __syncthreads();
            if (ty == kt) {
#pragma unroll
                for (int c = 0; c < R; ++c)
#pragma unroll
                    for (int r = 0; r < R; ++r) if (r == kr) Am[r][c] = prow[tx + TG * c];
            }
            if (ty == p % TG) {
#pragma unroll
                for (int c = 0; c < R; ++c)
#pragma unroll
                    for (int r = 0; r < R; ++r) if (r == p / TG) Am[r][c] = pcol[tx + TG * c];
            }
            __syncthreads();
        }
        // 3. broadcast pivot row and pivot column
        if (ty == kt) {
#pragma unroll
            for (int c = 0; c < R; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) if (r == kr) prow[tx + TG * c] = Am[r][c];
        }
        if (tx == kt) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < R; ++c) if (c == kr) pcol[ty + TG * r] = Am[r][c];
        }
        __syncthreads();
        if (threadIdx.x == 0) piv_val = prow[kk];
        __syncthreads();
        const double piv = piv_val;
        const double ipiv = 1.0 / piv;
        // 4. in-place Gauss-Jordan update
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int I = ty + TG * r;
            const double f = pcol[I];
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int J = tx + TG * c;
                double v = Am[r][c];
                if (I == kk) v = (J == kk) ? ipiv : v * ipiv;
                else if (J == kk) v = -f * ipiv;
                else v = v - f * prow[J] * ipiv;
                Am[r][c] = v;
            }
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges: result column j = computed column sigma[j]
    if (threadIdx.x == 0) {
        for (int j = 0; j < NPAD; ++j) sigma_inv[j] = j;   // holds sigma first
        for (int kk = NPAD - 1; kk >= 0; --kk) {
            const int p = perm[kk];
            const int tmp = sigma_inv[kk];
            sigma_inv[kk] = sigma_inv[p];
            sigma_inv[p] = tmp;
        }
        // invert sigma in place via prow as scratch
        for (int j = 0; j < NPAD; ++j) pcol[j] = (double)sigma_inv[j];
        for (int j = 0; j < NPAD; ++j) sigma_inv[(int)pcol[j]] = j;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int I = ty + TG * r, J = tx + TG * c;
            const int Jd = sigma_inv[J];
            if (I < npp && J < npp && Jd < npp) {
                // B[Jd][I] = A^{-1}[I][Jd] in the fragment layout of each precision
                const long long base = slot * vanka_inv_stride(npp);
                if (inv64) inv64[base + vanka_inv_offset(npp, vanka_spl(npp, 8), Jd, I)] = Am[r][c];
                if (inv32) inv32[base + vanka_inv_offset(npp, vanka_spl(npp, 4), Jd, I)] = (float)Am[r][c];
            }
        }
}

// ------------------------------------------------------------------------------------------------
// Vanka patch products on the matrix cores.  For one cell, C = A_K^{-1} R with A_K^{-1} of size
// n_p x n_p and R = [n_p][N_xi] (one column per chaos mode) is a small dense GEMM.  It runs
// transposed, C^T = R^T A_K^{-T}, as 16x16x4 MFMA tiles (FP64 MFMA for FP64, FP32 MFMA for the mixed
// V-cycle): one workgroup per cell, wave w owns the 16 patch rows 16w..16w+15 (the N dimension) and
// the chaos modes are the M dimension, so every lane ends up holding results of one patch row and
// stores them straight to the broken node array (summed per node by k_node_gather).
// 16x16x4 lane layout: lane l supplies A[m l%16][k l/16] and B[k l/16][n l%16] and receives
// D[out_row(l/16, v)][l%16], v = 0..3, with out_row = l/16 + 4v for the FP64 instruction and
// 4(l/16) + v for the FP32 one (both checked on gfx950 with known operands).
//  * B = A_K^{-T} streams from HBM: the inverse is stored transposed ([col][row]), so a fragment is
//    four 128-byte runs and every entry is read once.  The first PF fragments (all of them for
//    n_p <= 64) are requested at entry, together with the residual values, so one memory latency
//    covers both; later fragments are refilled PF k-steps ahead.
//  * A = R^T comes from LDS: the residual patch gathered from the node vector.
template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int kk, int v) { return kk + 4 * v; }
};
template <>
struct Mfma16<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int kk, int v) { return 4 * kk + v; }
};

// Vector of N values of T for one load (N = 1: T itself) and its element j (compile-time j).
template <typename T, int N>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(N)));
};
template <typename T>
struct VecOf<T, 1> {
    typedef T type;
};
template <typename T, int N>
__device__ __forceinline__ T vec_elem(const typename VecOf<T, N>::type& v, int j) {
    if constexpr (N == 1) {
        return v;
    } else {
        return v[j];
    }
}

constexpr int kVankaTiles = 3;                       // 16-mode tiles per pass (35 modes: one pass)
constexpr int kVankaModesPerPass = kVankaTiles * 16;
constexpr int kVankaLdr = kVankaModesPerPass + 1;    // LDS row stride, odd: rows in different banks
static_assert(kVankaLdr == 49, "vanka_lds_bytes assumes 49");

constexpr int vanka_threads(int dim, int k, int nt) { return 64 * ((nt * ipow(k + 1, dim) + 15) / 16); }

// Offsets inside r, the broken array and one cell's inverse are 32-bit (the launcher checks the
// sizes); only the per-cell base of the inverse is 64-bit.
template <int DIM, int K, int NT, typename T>
__global__ void __launch_bounds__(vanka_threads(DIM, K, NT))
    k_vanka_cells(Grid g, int n_xi, int n_cells, const T* __restrict__ invT, const T* __restrict__ r,
                  T* __restrict__ s_out, int classes) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NPP = NT * NP;
    constexpr int KS = (NPP + 3) / 4;     // k-steps
    constexpr int KP = KS * 4;            // rows of the LDS tile (zero beyond n_p)
    constexpr int LR = (KP + 63) / 64 * 64;
    // k-steps of B in flight: 128 bytes per lane (16 FP64 or 32 FP32 steps), or 64 for patches of more
    // than 128 rows (whose three accumulator tiles and gather registers leave no room for more within
    // the 3-waves-per-SIMD budget); all of them when the patch has fewer steps
    constexpr int PF0 = (NPP > 128 ? 64 : 128) / (int)sizeof(T);
    constexpr int PF = KS < PF0 ? KS : PF0;
    constexpr int NG = vanka_threads(DIM, K, NT) / LR;   // gather groups
    constexpr int LDR = kVankaLdr;
    constexpr int GB = (LDR + NG - 1) / NG;               // gathered values per thread and pass
    using M = Mfma16<T>;
    using v4 = typename M::v4;
    extern __shared__ unsigned char smem_raw[];
    T* const rk = reinterpret_cast<T*>(smem_raw);   // [KP][LDR]

    const int lane = threadIdx.x & 63;
    const int kk = lane >> 4;
    const int I = (threadIdx.x >> 6) * 16 + (lane & 15);  // patch row of this lane (B column, output)

    // cells in the XCD-local tiled row order
    const int pos = xcd_position(blockIdx.x, n_cells);
    const int cell = tiled_row<DIM>(pos / g.n, g.n) * g.n + pos % g.n;
    int cc[3] = {0, 0, 0};
    {
        int rr = cell;
        for (int d = 0; d < DIM; ++d) { cc[d] = rr % g.n; rr /= g.n; }
    }

    // B fragments: rows I, columns 4 step + kk of the inverse, SPL consecutive k-steps per vector load
    // (the fragment layout keeps them contiguous; columns beyond n_p are stored as zeros).  Every load
    // is unconditional: lanes with I >= n_p read row n_p - 1 instead, they own output columns that
    // are never stored.  (Loads under a branch would make the compiler wait for each refill at once.)
    constexpr int SPL = vanka_spl(NPP, sizeof(T));
    constexpr int NGR = KS / SPL;                          // fragment loads per lane and pass
    constexpr int PFV = (PF / SPL) > 0 ? PF / SPL : 1;     // loads in flight
    using VT = typename VecOf<T, SPL>::type;
    const VT* const bc = reinterpret_cast<const VT*>(invT + inverse_slot<DIM>(cell, cc, g.n, classes) *
                                                               vanka_inv_stride(NPP)) +
                         kk * NPP + min(I, NPP - 1);
    auto load_b = [&](int grp) -> VT {   // grp is a compile-time constant at every call
        return bc[grp * 4 * NPP];
    };
    VT ring[PFV];
#pragma unroll
    for (int u = 0; u < PFV; ++u) ring[u] = load_b(u);

    // gather role: patch row lrow (node fastest: neighbouring lanes read neighbouring nodes), modes
    // agrp, agrp + NG, ... of the pass; Dirichlet rows, rows beyond n_p and modes beyond N_xi are 0.
    // Loads are unconditional from clamped addresses; the mask is applied when writing LDS.
    const int nn = (int)g.n_nodes;
    const int rstride = NT * nn;                     // one chaos mode in r
    const int lrow = threadIdx.x % LR;
    const int agrp = threadIdx.x / LR;
    const bool gthread = agrp < NG && lrow < KP;
    int src = 0;
    bool live = lrow < NPP;
    {
        const int l = min(lrow, NPP - 1);
        const int p = l % NP;
        int m = 1;
        for (int d = 0; d < DIM; ++d) {
            const int id = cc[d] * K + (p / ipow(N1, d)) % N1;
            live &= (id != 0) & (id != g.n1 - 1);
            src += id * m;
            m *= g.n1;
        }
        src += (l / NP) * nn;
    }
    // store role: row I of the patch in the broken layout [comp][b_z][b_y][b_x]
    const int nb1 = g.n * N1;
    int nbn = 1;
    for (int d = 0; d < DIM; ++d) nbn *= nb1;
    const int sstride = NT * nbn;                    // one chaos mode in the broken array
    int dst = 0;
    {
        const int p = min(I, NPP - 1) % NP;
        int bm = 1;
        for (int d = 0; d < DIM; ++d) {
            dst += (cc[d] * N1 + (p / ipow(N1, d)) % N1) * bm;
            bm *= nb1;
        }
        dst += (min(I, NPP - 1) / NP) * nbn;
    }

    const int n_pass = (n_xi + kVankaModesPerPass - 1) / kVankaModesPerPass;
#pragma unroll 1
    for (int pass = 0; pass < n_pass; ++pass) {
        const int m0 = pass * kVankaModesPerPass;         // first mode of this pass
        if (pass > 0) {
            __syncthreads();                              // every wave is done with the previous pass
#pragma unroll
            for (int u = 0; u < PFV; ++u) ring[u] = load_b(u);
        }
        if (gthread) {
            T v[GB];
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const int al = min(m0 + agrp + u * NG, n_xi - 1);
                v[u] = r[src + al * rstride];
            }
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const int a = agrp + u * NG;
                if (a < LDR) rk[lrow * LDR + a] = (live && m0 + a < n_xi) ? v[u] : T(0);
            }
        }
        __syncthreads();

        // C^T tile: all three mode tiles every step (modes beyond N_xi have zero rows in A), so the
        // accumulators stay in the matrix-core registers and the MFMAs of consecutive steps overlap
        v4 acc[kVankaTiles];
#pragma unroll
        for (int q = 0; q < kVankaTiles; ++q) acc[q] = v4{T(0), T(0), T(0), T(0)};
        const T* const abase = rk + kk * LDR + (lane & 15);
#pragma unroll
        for (int step = 0; step < KS; ++step) {
            const int grp = step / SPL;
            const T bv = vec_elem<T, SPL>(ring[grp % PFV], step % SPL);
            if (step % SPL == SPL - 1 && grp + PFV < NGR) ring[grp % PFV] = load_b(grp + PFV);
            const T* arow = abase + step * 4 * LDR;
#pragma unroll
            for (int q = 0; q < kVankaTiles; ++q) acc[q] = M::run(arow[q * 16], bv, acc[q]);
        }
        // results of patch row I, modes m0 + 16q + out_row: straight into the broken array
        if (I < NPP) {
#pragma unroll
            for (int q = 0; q < kVankaTiles; ++q) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int al = m0 + q * 16 + M::out_row(kk, v);
                    if (al < n_xi) s_out[dst + al * sstride] = acc[q][v];
                }
            }
        }
    }
}

template <int DIM, int K, int NT, typename T>
hipError_t run_vanka(Grid g, int n_xi, const T* invT, const T* r, T* s_out, int classes, hipStream_t s) {
    constexpr int NPP = NT * ipow(K + 1, DIM);
    constexpr int KP = (NPP + 3) / 4 * 4;
    constexpr int waves = (NPP + 15) / 16;
    if constexpr (waves > 16) {
        return hipErrorInvalidValue;      // n_p > 256 is rejected when the handle is created
    } else {
        long long nbn = 1;
        for (int d = 0; d < DIM; ++d) nbn *= (long long)g.n * (K + 1);
        if ((long long)n_xi * NT * g.n_nodes >= (1LL << 31) || (long long)n_xi * NT * nbn >= (1LL << 31) ||
            g.n_cells >= (1LL << 31))
            return hipErrorInvalidValue;  // 32-bit offsets
        const size_t lds = (size_t)KP * kVankaLdr * sizeof(T);
        auto kern = k_vanka_cells<DIM, K, NT, T>;
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        const int n_cells = (int)g.n_cells;
        hipLaunchKernelGGL(kern, dim3(n_cells), dim3(waves * 64), lds, s, g, n_xi, n_cells, invT, r, s_out, classes);
        return hipGetLastError();
    }
}

template <int DIM, int K, typename T>
hipError_t vanka_nt(int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out, int classes, hipStream_t s) {
    switch (nt) {
        case 1: return run_vanka<DIM, K, 1, T>(g, n_xi, invT, r, s_out, classes, s);
        case 2: return run_vanka<DIM, K, 2, T>(g, n_xi, invT, r, s_out, classes, s);
        case 3: return run_vanka<DIM, K, 3, T>(g, n_xi, invT, r, s_out, classes, s);
        case 4: return run_vanka<DIM, K, 4, T>(g, n_xi, invT, r, s_out, classes, s);
    }
    return hipErrorInvalidValue;
}

template <int DIM, typename T>
hipError_t vanka_k(int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out, int classes, hipStream_t s) {
    switch (k) {
        case 1: return vanka_nt<DIM, 1, T>(nt, g, n_xi, invT, r, s_out, classes, s);
        case 2: return vanka_nt<DIM, 2, T>(nt, g, n_xi, invT, r, s_out, classes, s);
        case 3: return vanka_nt<DIM, 3, T>(nt, g, n_xi, invT, r, s_out, classes, s);
        case 4: return vanka_nt<DIM, 4, T>(nt, g, n_xi, invT, r, s_out, classes, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// ---- dense Gauss-Jordan inverse (coarsest level) -------------------------------------------------
// Step k, part 1 (one workgroup): pivot p = argmax_{i >= k} |A[i][k]|, swap rows k and p, scale row k
// by 1/A[k][k] (A[k][k] <- 1/A[k][k]), and stash column k (before the update) in col.
__global__ void __launch_bounds__(1024) k_gj_pivot(double* __restrict__ A, int n, int k, double* __restrict__ col,
                                                   int* __restrict__ perm, int* __restrict__ status) {
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    double best = -1.0;
    int arg = k;
    for (int i = k + threadIdx.x; i < n; i += 1024) {
        const double v = fabs(A[(long long)i * n + k]);
        if (v > best) { best = v; arg = i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = arg;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = bv[threadIdx.x + w];
            const int oi = bi[threadIdx.x + w];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = bi[0];
    if (!(bv[0] > 0.0)) {
        if (threadIdx.x == 0) *status = 1;
        return;                       // uniform: every thread returns
    }
    if (p != k)
        for (int j = threadIdx.x; j < n; j += 1024) {
            const double t = A[(long long)k * n + j];
            A[(long long)k * n + j] = A[(long long)p * n + j];
            A[(long long)p * n + j] = t;
        }
    __syncthreads();
    const double ipiv = 1.0 / A[(long long)k * n + k];
    for (int i = threadIdx.x; i < n; i += 1024) col[i] = A[(long long)i * n + k];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 1024)
        A[(long long)k * n + j] = (j == k) ? ipiv : A[(long long)k * n + j] * ipiv;
    if (threadIdx.x == 0) perm[k] = p;
}

// Step k, part 2: every row i != k: A[i][j] -= col[i] A[k][j] (j != k), A[i][k] = -col[i] / pivot.
__global__ void __launch_bounds__(256) k_gj_eliminate(double* __restrict__ A, int n, int k,
                                                      const double* __restrict__ col, const int* __restrict__ status) {
    if (*status) return;
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y;
    if (i == k || j >= n) return;
    const double f = col[i];
    if (f == 0.0) return;
    const double akj = A[(long long)k * n + j];   // row k is final (scaled) after part 1
    if (j == k) A[(long long)i * n + k] = -f * akj;
    else A[(long long)i * n + j] -= f * akj;
}

// Undo the row interchanges on the inverse (column swaps in reverse order; one thread per row) and
// write the transpose.
__global__ void __launch_bounds__(256) k_gj_finish(double* __restrict__ A, int n, const int* __restrict__ perm,
                                                   const int* __restrict__ status, double* __restrict__ AinvT) {
    if (*status) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double* row = A + (long long)i * n;
    for (int k = n - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k) {
            const double t = row[k];
            row[k] = row[p];
            row[p] = t;
        }
    }
    for (int j = 0; j < n; ++j) AinvT[(long long)j * n + i] = row[j];
}

hipError_t launch_dense_invert(double* A, int n, double* col, int* perm, int* status, double* AinvT, hipStream_t s) {
    if (n < 1 || n > 65535) return hipErrorInvalidValue;
    const dim3 eg((n + 255) / 256, n);
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, A, n, k, col, perm, status);
        hipLaunchKernelGGL(k_gj_eliminate, eg, dim3(256), 0, s, A, n, k, col, status);
    }
    hipLaunchKernelGGL(k_gj_finish, dim3((n + 255) / 256), dim3(256), 0, s, A, n, perm, status, AinvT);
    return hipGetLastError();
}

hipError_t launch_elem_stiffness(int dim, int k, Grid g, const double* coef0, const ElemTables& et, double* E,
                                 hipStream_t s) {
    const int np = dim == 2 ? (k + 1) * (k + 1) : (k + 1) * (k + 1) * (k + 1);
    const long long total = g.n_cells * np * np;
    const int threads = 256;
    long long blocks = (total + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_elem_stiffness, dim3((unsigned)blocks), dim3(threads), 0, s, dim, k, g, coef0, et, E);
    return hipGetLastError();
}

hipError_t launch_patch_invert(int dim, int k, int nt, Grid g, const double* E, const double* Me,
                               const PatchTime& pt, double* inv64, float* inv32, int* status, hipStream_t s,
                               const int* cells, int n_list) {
    const int np = dim == 2 ? (k + 1) * (k + 1) : (k + 1) * (k + 1) * (k + 1);
    const int npp = nt * np;
    const unsigned blocks = cells ? (unsigned)n_list : (unsigned)g.n_cells;
#define SG_PI(TG, R)                                                                                        \
    if (npp <= TG * R) {                                                                                    \
        hipLaunchKernelGGL((k_patch_invert<TG, R>), dim3(blocks), dim3(TG * TG), 0, s, dim, k, nt, g, E, Me, pt, \
                           inv64, inv32, status, cells);                                                    \
        return hipGetLastError();                                                                           \
    }
    SG_PI(8, 1)
    SG_PI(8, 2)
    SG_PI(8, 3)
    SG_PI(16, 2)
    SG_PI(16, 3)
    SG_PI(16, 4)
    SG_PI(32, 3)
    SG_PI(32, 4)
    SG_PI(32, 5)
    SG_PI(32, 6)
    SG_PI(32, 7)
    SG_PI(32, 8)
#undef SG_PI
    return hipErrorInvalidValue;
}

// Per-mode diagonal blocks: c_{K,alpha} = A_{alpha,K}^{-1} R_K r_alpha with one inverse per (mode, cell),
// one workgroup per (cell, mode), one thread per patch row: a dense matrix-vector product reading the
// transposed inverse column by column (consecutive rows in consecutive lanes).
template <int DIM, int K, int NT, typename T>
__global__ void __launch_bounds__(256)
    k_vanka_cells_modes(Grid g, const T* __restrict__ invT, const T* __restrict__ r, T* __restrict__ s_out) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NPP = NT * NP;
    __shared__ T rp[NPP];
    const long long cell = blockIdx.x;
    const int al = blockIdx.y;
    const int t = threadIdx.x;
    const long long nn = g.n_nodes;
    int cc[3] = {0, 0, 0};
    {
        long long rr = cell;
        for (int d = 0; d < DIM; ++d) { cc[d] = (int)(rr % g.n); rr /= g.n; }
    }
    const int nb1 = g.n * N1;
    long long nbn = 1;
    for (int d = 0; d < DIM; ++d) nbn *= nb1;
    long long src = 0, dst = 0;
    if (t < NPP) {
        const int p = t % NP, ti = t / NP;
        bool live = true;
        long long m = 1, bm = 1;
        for (int d = 0; d < DIM; ++d) {
            const int a = (p / ipow(N1, d)) % N1;
            const int id = cc[d] * K + a;
            live &= (id != 0) & (id != g.n1 - 1);
            src += id * m;
            dst += (long long)(cc[d] * N1 + a) * bm;
            m *= g.n1;
            bm *= nb1;
        }
        src += ((long long)al * NT + ti) * nn;
        dst += ((long long)al * NT + ti) * nbn;
        rp[t] = live ? r[src] : T(0);
    }
    __syncthreads();
    if (t < NPP) {
        constexpr int SPL = vanka_spl(NPP, sizeof(T));
        const T* c = invT + ((long long)al * g.n_cells + cell) * vanka_inv_stride(NPP);
        T acc = T(0);
#pragma unroll 8
        for (int j = 0; j < NPP; ++j) acc += c[vanka_inv_offset(NPP, SPL, j, t)] * rp[j];
        s_out[dst] = acc;
    }
}

template <int DIM, typename T>
hipError_t vanka_modes_k(int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out, hipStream_t s) {
    const dim3 grid((unsigned)g.n_cells, (unsigned)n_xi);
#define SG_VM(K_, T_)                                                                                         \
    if (k == K_ && nt == T_) {                                                                                \
        constexpr int npp = T_ * ipow(K_ + 1, DIM);                                                           \
        if constexpr (npp <= 256) {                                                                           \
            hipLaunchKernelGGL((k_vanka_cells_modes<DIM, K_, T_, T>), grid, dim3((npp + 63) / 64 * 64), 0, s, \
                               g, invT, r, s_out);                                                            \
            return hipGetLastError();                                                                         \
        } else {                                                                                              \
            return hipErrorInvalidValue;                                                                      \
        }                                                                                                     \
    }
#define SG_VM_K(K_) SG_VM(K_, 1) SG_VM(K_, 2) SG_VM(K_, 3) SG_VM(K_, 4)
    SG_VM_K(1) SG_VM_K(2) SG_VM_K(3) SG_VM_K(4)
#undef SG_VM_K
#undef SG_VM
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_vanka_cells_modes(int dim, int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out,
                                    hipStream_t s) {
    if (dim == 2) return vanka_modes_k<2, T>(k, nt, g, n_xi, invT, r, s_out, s);
    if (dim == 3) return vanka_modes_k<3, T>(k, nt, g, n_xi, invT, r, s_out, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_vanka_cells_modes<double>(int, int, int, Grid, int, const double*, const double*, double*,
                                                     hipStream_t);
template hipError_t launch_vanka_cells_modes<float>(int, int, int, Grid, int, const float*, const float*, float*,
                                                    hipStream_t);

template <typename T>
hipError_t launch_vanka_cells(int dim, int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out,
                              int classes, hipStream_t s) {
    if (classes && g.n < 2) return hipErrorInvalidValue;
    if (dim == 2) return vanka_k<2, T>(k, nt, g, n_xi, invT, r, s_out, classes, s);
    if (dim == 3) return vanka_k<3, T>(k, nt, g, n_xi, invT, r, s_out, classes, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_vanka_cells<double>(int, int, int, Grid, int, const double*, const double*, double*,
                                               int, hipStream_t);
template hipError_t launch_vanka_cells<float>(int, int, int, Grid, int, const float*, const float*, float*, int,
                                              hipStream_t);

// ------------------------------------------------------------------------------------------------
// Vanka patch corrections by fast diagonalisation, for levels whose mean coefficient is one constant
// c.  The assembled mean block is then A_t (x) M + B_t (x) K with M = (x)_d M1 and K = sum_d of the
// Kronecker products with one factor c K1 (M1, K1 the assembled 1D matrices), and the restriction of
// a Kronecker product to the nodes of a cell is the Kronecker product of the restrictions.  On the
// interior nodes of the cell along each direction, the 1D pencil has c K1r S = M1r S Lambda with
// S^T M1r S = I, so with S3 = (x)_d S_d the patch matrix becomes block diagonal:
//     A_{0,K}^{-1} = (I (x) S3) diag_e (A_t + lambda_e B_t)^{-1} (I (x) S3^T),
// lambda_e the sum of the 1D eigenvalues of eigen index e.  S_d is stored (k+1) x (k+1) with zero
// rows for Dirichlet nodes and zero columns for unused eigen indices, so the product is zero on the
// Dirichlet DoFs, as the identity rows of the dense patch give for the masked residual there.
//   Sv: [3 variants][k+1 nodes j][k+1 eigen i]; variant 0 / 1 / 2 = first / inner / last cell
//       along a direction (the 1D restriction is the same in every direction of the uniform mesh).
//   Tt: [3^d classes][(k+1)^d eigen e][N_t][N_t], (A_t + lambda_e B_t)^{-1} (zero for unused e);
//       class = sum_d 3^d variant_d.
// One workgroup per cell.  The residual patch of up to `mp` modes is gathered into LDS (x-lines of odd
// length, so the line sweeps below hit different banks), transformed along every direction
// but the last in place, then the last direction, the time blocks and the inverse transform of the
// last direction run in one sweep per (mode, line), and the remaining inverse transforms follow; the
// result goes to the broken node array like k_vanka_cells' results.
namespace {

constexpr int kFdmThreads = 256;
constexpr int kFdmBatch = 8;      // global loads a thread has in flight in the gather

// Every thread keeps one node p of the cell (gather and store) and one line q (the sweeps) for the
// whole launch and walks the components: the index arithmetic is done once, not per element.
template <int DIM, int K, int NT, typename T>
__global__ void __launch_bounds__(kFdmThreads)
    k_vanka_fdm(Grid g, int n_xi, int mp, const T* __restrict__ Sv, const T* __restrict__ Tt,
                const T* __restrict__ r, T* __restrict__ s_out) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NL = NP / N1;               // lines of one component along one direction
    constexpr int LS = N1 | 1;                // LDS stride of an x-line (odd: the x sweeps hit different banks)
    constexpr int PC = NL * LS;               // LDS stride of one component
    constexpr int NTT = NT * NT;
    constexpr int GP = kFdmThreads / NP;      // components per round of the gather and the store
    constexpr int GL = kFdmThreads / NL;      // components (modes in the last sweep) per round of a sweep
    static_assert(GP >= 1 && GL >= 1, "one cell's nodes must fit the workgroup");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* const tb = reinterpret_cast<T*>(smem_raw);   // [NP][NT][NT] of this cell's class
    T* const X = tb + NP * NTT;                     // [mp * NT][PC], node p at (p / N1) LS + p % N1

    const int n_cells = (int)g.n_cells;
    const int pos = xcd_position(blockIdx.x, n_cells);
    const int cell = tiled_row<DIM>(pos / g.n, g.n) * g.n + pos % g.n;
    int cc[3] = {0, 0, 0};
    {
        int rr = cell;
        for (int d = 0; d < DIM; ++d) { cc[d] = rr % g.n; rr /= g.n; }
    }
    int cls = 0, node0 = 0, brk0 = 0;
    const int nb1 = g.n * N1;
    int nbn = 1;
    const T* Sd[3];
    for (int d = 0, m3 = 1, mn = 1; d < DIM; ++d) {
        const int v = cc[d] == 0 ? 0 : (cc[d] == g.n - 1 ? 2 : 1);
        cls += m3 * v;
        Sd[d] = Sv + v * N1 * N1;
        node0 += cc[d] * K * mn;
        brk0 += cc[d] * N1 * nbn;
        m3 *= 3;
        mn *= g.n1;
        nbn *= nb1;
    }
    const int nn = (int)g.n_nodes;
    const T* const tc = Tt + (long long)cls * NP * NTT;
    for (int i = threadIdx.x; i < NP * NTT; i += kFdmThreads) tb[i] = tc[i];

    // node role: node tp of the cell for components tg, tg + GP, ...
    const int tp = threadIdx.x % NP, tg = threadIdx.x / NP;
    int noff = 0, boff = 0;
    bool live = true;
    for (int d = 0, pp = tp, mn = 1, bm = 1; d < DIM; ++d, pp /= N1) {
        const int id = cc[d] * K + pp % N1;
        live &= (id != 0) & (id != g.n1 - 1);
        noff += (pp % N1) * mn;
        boff += (pp % N1) * bm;
        mn *= g.n1;
        bm *= nb1;
    }
    const int lpos = (tp / N1) * LS + tp % N1;
    // line role: line tq of components tl, tl + GL, ... (LDS offset of its first node per direction)
    const int tq = threadIdx.x % NL, tl = threadIdx.x / NL;
    int lbase[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int st = ipow(N1, d);
        const int pb = d == DIM - 1 ? tq : tq % st + (tq / st) * st * N1;
        lbase[d] = (pb / N1) * LS + pb % N1;
    }
    __syncthreads();

    for (int m0 = 0; m0 < n_xi; m0 += mp) {
        const int nm = min(mp, n_xi - m0);
        const int ncomp = nm * NT;
        const T* const rp = r + node0 + noff + m0 * NT * nn;
        // gather: neighbouring threads read neighbouring nodes, kFdmBatch loads in flight per thread
        // (clamped to the last component where past the end); Dirichlet values are zeroed
        if (tg < GP) {
            for (int cb = tg; cb < ncomp; cb += GP * kFdmBatch) {
                T v[kFdmBatch];
#pragma unroll
                for (int u = 0; u < kFdmBatch; ++u) v[u] = rp[min(cb + u * GP, ncomp - 1) * nn];
#pragma unroll
                for (int u = 0; u < kFdmBatch; ++u) {
                    const int c = cb + u * GP;
                    if (c < ncomp) X[c * PC + lpos] = live ? v[u] : T(0);
                }
            }
        }
        __syncthreads();
        // forward transforms along every direction but the last: u_i = sum_j S[j][i] v_j
#pragma unroll
        for (int d = 0; d < DIM - 1; ++d) {
            const int ls = d == 0 ? 1 : (ipow(N1, d) / N1) * LS;   // LDS stride of direction d
            T S[N1 * N1];
#pragma unroll
            for (int i = 0; i < N1 * N1; ++i) S[i] = Sd[d][i];
            if (tl < GL) {
                for (int c = tl; c < ncomp; c += GL) {
                    T* const line = X + c * PC + lbase[d];
                    T v[N1];
#pragma unroll
                    for (int j = 0; j < N1; ++j) v[j] = line[j * ls];
#pragma unroll
                    for (int i = 0; i < N1; ++i) {
                        T u = T(0);
#pragma unroll
                        for (int j = 0; j < N1; ++j) u += S[j * N1 + i] * v[j];
                        line[i * ls] = u;
                    }
                }
            }
            __syncthreads();
        }
        // last direction: forward transform, the time block of every eigen index, inverse transform
        {
            constexpr int st = NL;
            constexpr int ls = DIM == 1 ? 1 : (NL / N1) * LS;
            T S[N1 * N1];
#pragma unroll
            for (int i = 0; i < N1 * N1; ++i) S[i] = Sd[DIM - 1][i];
            if (tl < GL) {
                for (int ml = tl; ml < nm; ml += GL) {
                    T u[NT][N1];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const T* const line = X + (ml * NT + t) * PC + lbase[DIM - 1];
                        T v[N1];
#pragma unroll
                        for (int j = 0; j < N1; ++j) v[j] = line[j * ls];
#pragma unroll
                        for (int i = 0; i < N1; ++i) {
                            T a = T(0);
#pragma unroll
                            for (int j = 0; j < N1; ++j) a += S[j * N1 + i] * v[j];
                            u[t][i] = a;
                        }
                    }
                    T w[NT][N1];
#pragma unroll
                    for (int i = 0; i < N1; ++i) {
                        const T* const te = tb + (tq + i * st) * NTT;
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            T a = T(0);
#pragma unroll
                            for (int t2 = 0; t2 < NT; ++t2) a += te[t * NT + t2] * u[t2][i];
                            w[t][i] = a;
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        T* const line = X + (ml * NT + t) * PC + lbase[DIM - 1];
#pragma unroll
                        for (int j = 0; j < N1; ++j) {
                            T a = T(0);
#pragma unroll
                            for (int i = 0; i < N1; ++i) a += S[j * N1 + i] * w[t][i];
                            line[j * ls] = a;
                        }
                    }
                }
            }
            __syncthreads();
        }
        // inverse transforms along the other directions: o_j = sum_i S[j][i] w_i
#pragma unroll
        for (int d = DIM - 2; d >= 0; --d) {
            const int ls = d == 0 ? 1 : (ipow(N1, d) / N1) * LS;
            T S[N1 * N1];
#pragma unroll
            for (int i = 0; i < N1 * N1; ++i) S[i] = Sd[d][i];
            if (tl < GL) {
                for (int c = tl; c < ncomp; c += GL) {
                    T* const line = X + c * PC + lbase[d];
                    T w[N1];
#pragma unroll
                    for (int i = 0; i < N1; ++i) w[i] = line[i * ls];
#pragma unroll
                    for (int j = 0; j < N1; ++j) {
                        T a = T(0);
#pragma unroll
                        for (int i = 0; i < N1; ++i) a += S[j * N1 + i] * w[i];
                        line[j * ls] = a;
                    }
                }
            }
            __syncthreads();
        }
        // store into the broken layout [comp][b_z][b_y][b_x]
        if (tg < GP) {
            T* const sp = s_out + brk0 + boff + m0 * NT * nbn;
#pragma unroll 4
            for (int c = tg; c < ncomp; c += GP) sp[c * nbn] = X[c * PC + lpos];
        }
        __syncthreads();                          // the next pass reuses X
    }
}

// The same corrections with one thread per (cell, mode) holding the mode's whole patch residual, all
// N_t (k+1)^d values, in registers: no LDS and no barrier.  Neighbouring lanes take neighbouring cells
// along x of one mode, so the loads of one local node and the stores of one broken entry cover
// contiguous stretches.  Same tables and the same operations in the same order as k_vanka_fdm, so
// the results are bitwise those of the LDS form.  For Q1 and Q2 patches of at most kFdmRegValues values
// (larger ones spill registers).
constexpr int kFdmRegValues = 54;
// waves per SIMD the register form is compiled for (the compiler would otherwise keep every table
// value live: 256 VGPRs for the 3D Q2 dG(1) patch)
template <int NV, typename T>
constexpr int fdm_reg_waves() { return NV * (int)sizeof(T) > 300 ? 2 : (NV * (int)sizeof(T) > 160 ? 3 : 4); }

template <int DIM, int K, int NT, typename T, bool MERGE>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(fdm_reg_waves<NT * ipow(K + 1, DIM), T>())))
    k_vanka_fdm_reg(Grid g, int n_xi, const T* __restrict__ Sv, const T* __restrict__ Tt, const T* __restrict__ r,
                    T* __restrict__ s_out) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NTT = NT * NT;
    const int n_cells = (int)g.n_cells;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (long long)n_xi * n_cells) return;    // no barrier follows
    const int mode = (int)(gid / n_cells);
    const int cell = (int)(gid - (long long)mode * n_cells);
    int cc[3] = {0, 0, 0};
    {
        int rr = cell;
        for (int d = 0; d < DIM; ++d) { cc[d] = rr % g.n; rr /= g.n; }
    }
    int cls = 0, node0 = 0, brk0 = 0, vv[3] = {0, 0, 0};
    const int nb1 = g.n * N1;
    int nbn = 1;
    for (int d = 0, m3 = 1, mn = 1; d < DIM; ++d) {
        vv[d] = cc[d] == 0 ? 0 : (cc[d] == g.n - 1 ? 2 : 1);
        cls += m3 * vv[d];
        node0 += cc[d] * K * mn;
        // MERGE: one x entry per node (b_x = node x index), the cells' shared x faces summed
        const int ext = (MERGE && d == 0) ? g.n1 : nb1;
        brk0 += cc[d] * (MERGE && d == 0 ? K : N1) * nbn;
        m3 *= 3;
        mn *= g.n1;
        nbn *= ext;
    }
    const int nn = (int)g.n_nodes;
    // the residual patch, Dirichlet values zeroed
    T u[NT][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        int node = node0;
        bool live = true;
#pragma unroll
        for (int d = 0, pp = p, mn = 1; d < DIM; ++d, pp /= N1) {
            const int id = cc[d] * K + pp % N1;
            live &= (id != 0) & (id != g.n1 - 1);
            node += (pp % N1) * mn;
            mn *= g.n1;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const T v = r[(mode * NT + t) * nn + node];
            u[t][p] = live ? v : T(0);
        }
    }
    // transforms along direction d (node stride st = (k+1)^d): fwd u_i = sum_j S[j][i] v_j, else
    // o_j = sum_i S[j][i] w_i
    auto sweep = [&](int d, bool fwd, T (&a)[NP]) {
        const int st = ipow(N1, d);
        const T* const S = Sv + vv[d] * N1 * N1;
#pragma unroll
        for (int q = 0; q < NP / N1; ++q) {
            const int pb = q % st + (q / st) * st * N1;
            T v[N1];
#pragma unroll
            for (int j = 0; j < N1; ++j) v[j] = a[pb + j * st];
#pragma unroll
            for (int i = 0; i < N1; ++i) {
                T o = T(0);
#pragma unroll
                for (int j = 0; j < N1; ++j) o += (fwd ? S[j * N1 + i] : S[i * N1 + j]) * v[j];
                a[pb + i * st] = o;
            }
        }
    };
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int t = 0; t < NT; ++t) sweep(d, true, u[t]);
    // the time block of every eigen index
    const T* const tc = Tt + (long long)cls * NP * NTT;
#pragma unroll
    for (int e = 0; e < NP; ++e) {
        T w[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            T a = T(0);
#pragma unroll
            for (int t2 = 0; t2 < NT; ++t2) a += tc[e * NTT + t * NT + t2] * u[t2][e];
            w[t] = a;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) u[t][e] = w[t];
        // keep the table loads of the next eigen index after this one's use (the scheduler would
        // otherwise issue all of them at once and hold every block in registers)
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int d = DIM - 1; d >= 0; --d)
#pragma unroll
        for (int t = 0; t < NT; ++t) sweep(d, false, u[t]);
    // store into the broken layout [comp][b_z][b_y][b_x], one x-line at a time.  MERGE: the next lane
    // holds the next cell along x of the same row (rows never straddle a wave); its left x face is added
    // into this cell's right face, in the gather's order (left cell's copy first).  Every cell but the
    // first of a row stores the merged face of its left neighbour at its own left face, the same value to
    // the same address (no branch around a store)
    const bool has_right = cc[0] < g.n - 1;
    const int bx = MERGE ? g.n1 : nb1;           // entries along x per (b_y, b_z)
#pragma unroll
    for (int q = 0; q < NP / N1; ++q) {
        int b = brk0;
        for (int d = 1, qq = q, bm = bx; d < DIM; ++d, qq /= N1) {
            b += (qq % N1) * bm;
            bm *= nb1;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            T* const dst = s_out + (mode * NT + t) * nbn + b;
            if constexpr (MERGE) {
                const T left_of_next = __shfl_down(u[t][q * N1], 1);
                const T merged = u[t][q * N1 + K] + (has_right ? left_of_next : T(0));
                const T merged_prev = __shfl_up(merged, 1);
                dst[0] = cc[0] == 0 ? u[t][q * N1] : merged_prev;
#pragma unroll
                for (int x = 1; x < K; ++x) dst[x] = u[t][q * N1 + x];
                dst[K] = merged;
            } else {
#pragma unroll
                for (int x = 0; x < N1; ++x) dst[x] = u[t][q * N1 + x];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The register form where the patch fits it, unless SGHEAT_VANKA_FDM=lds (a measurement switch).
inline bool fdm_lds_forced() {
    const char* e = std::getenv("SGHEAT_VANKA_FDM");
    return e && std::strcmp(e, "lds") == 0;
}

template <int DIM, int K, int NT, typename T>
hipError_t run_vanka_fdm(Grid g, int n_xi, const T* Sv, const T* Tt, const T* r, T* s_out, int* sx, hipStream_t s) {
    *sx = K;
    constexpr int NP = ipow(K + 1, DIM);
    long long nbn = 1;
    for (int d = 0; d < DIM; ++d) nbn *= (long long)g.n * (K + 1);
    if ((long long)n_xi * NT * g.n_nodes >= (1LL << 31) || (long long)n_xi * NT * nbn >= (1LL << 31) ||
        g.n_cells >= (1LL << 31) || n_xi < 1)
        return hipErrorInvalidValue;      // 32-bit offsets
    if constexpr (NT * NP <= kFdmRegValues && K <= 2) {
        if (!fdm_lds_forced()) {
            const long long threads = (long long)n_xi * g.n_cells;
            const dim3 grid((unsigned)((threads + 255) / 256));
            // whole rows inside one wave (n a power of two up to 64): the x faces are summed in registers
            if (g.n <= 64 && (64 % g.n) == 0) {
                *sx = g.n * K;
                hipLaunchKernelGGL((k_vanka_fdm_reg<DIM, K, NT, T, true>), grid, dim3(256), 0, s, g, n_xi, Sv, Tt, r,
                                   s_out);
            } else {
                hipLaunchKernelGGL((k_vanka_fdm_reg<DIM, K, NT, T, false>), grid, dim3(256), 0, s, g, n_xi, Sv, Tt, r,
                                   s_out);
            }
            return hipGetLastError();
        }
    }
    const int mp = vanka_fdm_modes_per_pass(DIM, K, NT, n_xi, sizeof(T));
    const size_t lds = vanka_fdm_lds_bytes(DIM, K, NT, mp, sizeof(T));
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    auto kern = k_vanka_fdm<DIM, K, NT, T>;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)g.n_cells), dim3(kFdmThreads), lds, s, g, n_xi, mp, Sv, Tt, r, s_out);
    return hipGetLastError();
}

template <int DIM, int K, typename T>
hipError_t vanka_fdm_nt(int nt, Grid g, int n_xi, const T* Sv, const T* Tt, const T* r, T* s_out, int* sx,
                        hipStream_t s) {
    switch (nt) {
        case 1: return run_vanka_fdm<DIM, K, 1, T>(g, n_xi, Sv, Tt, r, s_out, sx, s);
        case 2: return run_vanka_fdm<DIM, K, 2, T>(g, n_xi, Sv, Tt, r, s_out, sx, s);
        case 3: return run_vanka_fdm<DIM, K, 3, T>(g, n_xi, Sv, Tt, r, s_out, sx, s);
        case 4: return run_vanka_fdm<DIM, K, 4, T>(g, n_xi, Sv, Tt, r, s_out, sx, s);
    }
    return hipErrorInvalidValue;
}

template <int DIM, typename T>
hipError_t vanka_fdm_k(int k, int nt, Grid g, int n_xi, const T* Sv, const T* Tt, const T* r, T* s_out, int* sx,
                       hipStream_t s) {
    switch (k) {
        case 1: return vanka_fdm_nt<DIM, 1, T>(nt, g, n_xi, Sv, Tt, r, s_out, sx, s);
        case 2: return vanka_fdm_nt<DIM, 2, T>(nt, g, n_xi, Sv, Tt, r, s_out, sx, s);
        case 3: return vanka_fdm_nt<DIM, 3, T>(nt, g, n_xi, Sv, Tt, r, s_out, sx, s);
        case 4: return vanka_fdm_nt<DIM, 4, T>(nt, g, n_xi, Sv, Tt, r, s_out, sx, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

template <typename T>
hipError_t launch_vanka_fdm(int dim, int k, int nt, Grid g, int n_xi, const T* Sv, const T* Tt, const T* r,
                            T* s_out, int* sx, hipStream_t s) {
    if (dim == 2) return vanka_fdm_k<2, T>(k, nt, g, n_xi, Sv, Tt, r, s_out, sx, s);
    if (dim == 3) return vanka_fdm_k<3, T>(k, nt, g, n_xi, Sv, Tt, r, s_out, sx, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_vanka_fdm<double>(int, int, int, Grid, int, const double*, const double*, const double*,
                                             double*, int*, hipStream_t);
template hipError_t launch_vanka_fdm<float>(int, int, int, Grid, int, const float*, const float*, const float*,
                                            float*, int*, hipStream_t);

}  // namespace sg
