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
                   PatchTime pt, double* __restrict__ inv64, float* __restrict__ inv32, int* status) {
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
    const long long cell = blockIdx.x;
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
                const long long o = (cell * npp + Jd) * npp + I;   // stored transposed: [cell][col][row]
                if (inv64) inv64[o] = Am[r][c];
                if (inv32) inv32[o] = (float)Am[r][c];
            }
        }
}

// ------------------------------------------------------------------------------------------------
// One workgroup per cell, one wave per chunk of 64 patch rows.  Lane l owns row l of its chunk and
// keeps SW chaos modes in registers (all of them when N_xi <= SW, else strips in turn); the patch
// inverse is stored transposed so that, for a fixed column m, the 64 lanes read 64 consecutive
// entries, and every entry is read once; the residual patch rk[m][mode] is an LDS broadcast.  The
// correction of the cell goes to the broken node array (summed per node by k_node_gather).
template <int DIM, int K, int NT, typename T, int SW>
__global__ void __launch_bounds__(256)
    k_vanka_cells(Grid g, int n_xi, int nblocks, const T* __restrict__ invT, const T* __restrict__ r,
                  T* __restrict__ s_out) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NPP = NT * NP;
    extern __shared__ unsigned char smem_raw[];
    const int nstrip = (n_xi + SW - 1) / SW;
    const int ldr = nstrip * SW;
    T* rk = reinterpret_cast<T*>(smem_raw);   // [NPP][ldr]

    // contiguous cell ranges per XCD (blocks are dispatched round-robin over the 8 XCDs)
    const int b = blockIdx.x;
    const long long cell = (long long)((b % 8) * (nblocks / 8) + min(b % 8, nblocks % 8) + b / 8);
    int cc[3] = {0, 0, 0};
    {
        long long rr = cell;
        for (int d = 0; d < DIM; ++d) { cc[d] = (int)(rr % g.n); rr /= g.n; }
    }
    const long long nn = g.n_nodes;

    // gather r_K: rk[l][alpha], l = i*NP + p; Dirichlet rows and padding modes are zero
    for (int idx = threadIdx.x; idx < NPP * ldr; idx += blockDim.x) {
        const int p = idx % NP;
        const int i = (idx / NP) % NT;
        const int al = idx / NPP;
        T v = T(0);
        if (al < n_xi) {
            long long node = 0, m = 1;
            bool bnd = false;
            for (int d = 0; d < DIM; ++d) {
                const int id = cc[d] * K + (p / ipow(N1, d)) % N1;
                bnd |= (id == 0) | (id == g.n1 - 1);
                node += id * m;
                m *= g.n1;
            }
            if (!bnd) v = r[((long long)al * NT + i) * nn + node];
        }
        rk[(i * NP + p) * ldr + al] = v;
    }
    __syncthreads();

    const int l = threadIdx.x;            // patch row of this lane
    if (l >= NPP) return;
    const T* A = invT + cell * NPP * NPP + l;
    const long long nb1 = (long long)g.n * N1;
    long long nbn = 1;
    for (int d = 0; d < DIM; ++d) nbn *= nb1;
    const int p = l % NP, i = l / NP;
    long long off = 0, mul = 1;
    for (int d = 0; d < DIM; ++d) {
        off += ((long long)cc[d] * N1 + (p / ipow(N1, d)) % N1) * mul;
        mul *= nb1;
    }
    constexpr int U = 8;                  // columns of the inverse in flight per lane
    for (int strip = 0; strip < nstrip; ++strip) {
        T acc[SW];
#pragma unroll
        for (int u = 0; u < SW; ++u) acc[u] = T(0);
        const T* rs = rk + strip * SW;
        T nxt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = (u < NPP) ? A[(long long)u * NPP] : T(0);
        for (int m0 = 0; m0 < NPP; m0 += U) {
            T cur[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u] = nxt[u];
            // prefetch the next U columns while this chunk is multiplied
#pragma unroll
            for (int u = 0; u < U; ++u) nxt[u] = (m0 + U + u < NPP) ? A[(long long)(m0 + U + u) * NPP] : T(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (m0 + u >= NPP) break;
                const T* rr = rs + (m0 + u) * ldr;
#pragma unroll
                for (int k2 = 0; k2 < SW; ++k2) acc[k2] += cur[u] * rr[k2];
            }
        }
        // cell-local correction into the broken layout [comp][b_z][b_y][b_x]
#pragma unroll
        for (int u = 0; u < SW; ++u) {
            const int al = strip * SW + u;
            if (al < n_xi) s_out[((long long)al * NT + i) * nbn + off] = acc[u];
        }
    }
}

template <int DIM, int K, int NT, typename T>
hipError_t run_vanka(Grid g, int n_xi, const T* invT, const T* r, T* s_out, hipStream_t s) {
    constexpr int NPP = NT * ipow(K + 1, DIM);
    constexpr int SW = 36;
    const int nstrip = (n_xi + SW - 1) / SW;
    const size_t lds = (size_t)NPP * nstrip * SW * sizeof(T);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    auto kern = k_vanka_cells<DIM, K, NT, T, SW>;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int blocks = (int)g.n_cells;
    const int threads = ((NPP + 63) / 64) * 64;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, s, g, n_xi, blocks, invT, r, s_out);
    return hipGetLastError();
}

template <int DIM, int K, typename T>
hipError_t vanka_nt(int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out, hipStream_t s) {
    switch (nt) {
        case 1: return run_vanka<DIM, K, 1, T>(g, n_xi, invT, r, s_out, s);
        case 2: return run_vanka<DIM, K, 2, T>(g, n_xi, invT, r, s_out, s);
        case 3: return run_vanka<DIM, K, 3, T>(g, n_xi, invT, r, s_out, s);
        case 4: return run_vanka<DIM, K, 4, T>(g, n_xi, invT, r, s_out, s);
    }
    return hipErrorInvalidValue;
}

template <int DIM, typename T>
hipError_t vanka_k(int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out, hipStream_t s) {
    switch (k) {
        case 1: return vanka_nt<DIM, 1, T>(nt, g, n_xi, invT, r, s_out, s);
        case 2: return vanka_nt<DIM, 2, T>(nt, g, n_xi, invT, r, s_out, s);
        case 3: return vanka_nt<DIM, 3, T>(nt, g, n_xi, invT, r, s_out, s);
        case 4: return vanka_nt<DIM, 4, T>(nt, g, n_xi, invT, r, s_out, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

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
                               const PatchTime& pt, double* inv64, float* inv32, int* status, hipStream_t s) {
    const int np = dim == 2 ? (k + 1) * (k + 1) : (k + 1) * (k + 1) * (k + 1);
    const int npp = nt * np;
    const unsigned blocks = (unsigned)g.n_cells;
#define SG_PI(TG, R)                                                                                        \
    if (npp <= TG * R) {                                                                                    \
        hipLaunchKernelGGL((k_patch_invert<TG, R>), dim3(blocks), dim3(TG * TG), 0, s, dim, k, nt, g, E, Me, pt, \
                           inv64, inv32, status);                                                           \
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

template <typename T>
hipError_t launch_vanka_cells(int dim, int k, int nt, Grid g, int n_xi, const T* invT, const T* r, T* s_out,
                              hipStream_t s) {
    if (dim == 2) return vanka_k<2, T>(k, nt, g, n_xi, invT, r, s_out, s);
    if (dim == 3) return vanka_k<3, T>(k, nt, g, n_xi, invT, r, s_out, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_vanka_cells<double>(int, int, int, Grid, int, const double*, const double*, double*,
                                               hipStream_t);
template hipError_t launch_vanka_cells<float>(int, int, int, Grid, int, const float*, const float*, float*,
                                              hipStream_t);

}  // namespace sg
