// Vanka patch smoother (Remark solver-matrix-free-sg: local dense patch problems on space-time
// patches).  Patch of cell K = every local node of the closed cell x all N_t time DoFs; the patch
// matrix is the restriction of the assembled mean block A_0 = A_t (x) M_x + B_t (x) K_{a_0}, with
// Dirichlet local DoFs replaced by identity rows and columns.
//
//   k_elem_stiffness : element stiffness matrices of the mean coefficient (one thread per entry)
//   k_patch_invert   : forms A_{0,K} from the element matrices of every cell sharing the node pair,
//                      inverts it by Gauss-Jordan elimination with partial pivoting, FP64, with the
//                      matrix distributed over a TG x TG thread grid (R x R entries per thread)
//   k_vanka_apply    : x <- x + omega sum_K R_K^T W_K A_{0,K}^{-1} R_K r for one colour of cells
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
                const long long o = (cell * npp + I) * npp + Jd;
                if (inv64) inv64[o] = Am[r][c];
                if (inv32) inv32[o] = (float)Am[r][c];
            }
        }
}

// ------------------------------------------------------------------------------------------------
template <int DIM, int K, int NT, typename T>
__global__ void __launch_bounds__(256)
    k_vanka_apply(Grid g, int n_xi, int par0, int par1, int par2, int cnt0, int cnt1, int cells_in_colour,
                  const T* __restrict__ inv, const T* __restrict__ r, const T* __restrict__ b, T* __restrict__ x,
                  T omega) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NPP = NT * NP;
    extern __shared__ unsigned char smem_raw[];
    const int ldr = (n_xi + 3) & ~3;
    T* rk = reinterpret_cast<T*>(smem_raw);   // [NPP][ldr]
    T* ck = rk + NPP * ldr;                   // [NPP][ldr]

    const int ci = blockIdx.x;
    if (ci >= cells_in_colour) return;
    const int par[3] = {par0, par1, par2};
    int cc[3] = {0, 0, 0};
    {
        int rr = ci;
        cc[0] = 2 * (rr % cnt0) + par0;
        rr /= cnt0;
        if (DIM >= 2) { cc[1] = 2 * (rr % cnt1) + par1; rr /= cnt1; }
        if (DIM == 3) cc[2] = 2 * rr + par2;
    }
    long long cell = 0, mul = 1;
    for (int d = 0; d < DIM; ++d) { cell += cc[d] * mul; mul *= g.n; }
    const long long nn = g.n_nodes;

    auto node_of = [&](int p, bool* bnd, bool* first, int* mult) {
        long long node = 0, m = 1;
        *bnd = false;
        *first = true;
        *mult = 1;
        for (int d = 0; d < DIM; ++d) {
            const int ad = (p / ipow(N1, d)) % N1;
            const int id = cc[d] * K + ad;
            *bnd |= (id == 0) | (id == g.n1 - 1);
            const bool shared = (ad == 0 && cc[d] > 0) || (ad == K && cc[d] < g.n - 1);
            if (shared) { *mult *= 2; if (par[d]) *first = false; }
            node += id * m;
            m *= g.n1;
        }
        return node;
    };

    // gather r_K: rk[l][alpha], l = i*NP + p
    for (int idx = threadIdx.x; idx < NPP * n_xi; idx += blockDim.x) {
        const int p = idx % NP;
        const int i = (idx / NP) % NT;
        const int al = idx / NPP;
        bool bnd, first;
        int mult;
        const long long node = node_of(p, &bnd, &first, &mult);
        rk[(i * NP + p) * ldr + al] = bnd ? T(0) : r[((long long)al * NT + i) * nn + node];
    }
    for (int idx = threadIdx.x; idx < NPP * (ldr - n_xi); idx += blockDim.x) {
        const int l = idx / (ldr - n_xi), al = n_xi + idx % (ldr - n_xi);
        rk[l * ldr + al] = T(0);
    }
    __syncthreads();

    // ck = inv_K rk, a 4-wide strip of modes per task
    const T* A = inv + cell * NPP * NPP;
    const int nab = ldr / 4;
    for (int task = threadIdx.x; task < NPP * nab; task += blockDim.x) {
        const int l = task / nab;
        const int a0 = (task % nab) * 4;
        T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
        const T* arow = A + (long long)l * NPP;
        for (int m = 0; m < NPP; ++m) {
            const T av = arow[m];
            const T* rr = rk + m * ldr + a0;
            acc0 += av * rr[0];
            acc1 += av * rr[1];
            acc2 += av * rr[2];
            acc3 += av * rr[3];
        }
        T* cw = ck + l * ldr + a0;
        cw[0] = acc0;
        cw[1] = acc1;
        cw[2] = acc2;
        cw[3] = acc3;
    }
    __syncthreads();

    // weighted scatter-add (coloured: no other cell of this colour touches these nodes)
    for (int idx = threadIdx.x; idx < NPP * n_xi; idx += blockDim.x) {
        const int p = idx % NP;
        const int i = (idx / NP) % NT;
        const int al = idx / NPP;
        bool bnd, first;
        int mult;
        const long long node = node_of(p, &bnd, &first, &mult);
        const long long gi = ((long long)al * NT + i) * nn + node;
        if (bnd) {
            if (first) x[gi] = b[gi];
        } else {
            x[gi] += omega * ck[(i * NP + p) * ldr + al] / T(mult);
        }
    }
}

template <int DIM, int K, int NT, typename T>
hipError_t run_vanka(Grid g, int n_xi, const T* inv, const T* r, const T* b, T* x, T omega, hipStream_t s) {
    constexpr int NPP = NT * ipow(K + 1, DIM);
    const int ldr = (n_xi + 3) & ~3;
    const size_t lds = 2 * (size_t)NPP * ldr * sizeof(T);
    for (int colour = 0; colour < (1 << DIM); ++colour) {
        int par[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
        int cells = 1;
        for (int d = 0; d < DIM; ++d) {
            par[d] = (colour >> d) & 1;
            cnt[d] = (g.n - par[d] + 1) / 2;
            cells *= cnt[d];
        }
        if (cells == 0) continue;
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void*)k_vanka_apply<DIM, K, NT, T>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_vanka_apply<DIM, K, NT, T>), dim3(cells), dim3(256), lds, s, g, n_xi, par[0], par[1],
                           par[2], cnt[0], cnt[1], cells, inv, r, b, x, omega);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int DIM, int K, typename T>
hipError_t vanka_nt(int nt, Grid g, int n_xi, const T* inv, const T* r, const T* b, T* x, T omega, hipStream_t s) {
    switch (nt) {
        case 1: return run_vanka<DIM, K, 1, T>(g, n_xi, inv, r, b, x, omega, s);
        case 2: return run_vanka<DIM, K, 2, T>(g, n_xi, inv, r, b, x, omega, s);
        case 3: return run_vanka<DIM, K, 3, T>(g, n_xi, inv, r, b, x, omega, s);
        case 4: return run_vanka<DIM, K, 4, T>(g, n_xi, inv, r, b, x, omega, s);
    }
    return hipErrorInvalidValue;
}

template <int DIM, typename T>
hipError_t vanka_k(int k, int nt, Grid g, int n_xi, const T* inv, const T* r, const T* b, T* x, T omega,
                   hipStream_t s) {
    switch (k) {
        case 1: return vanka_nt<DIM, 1, T>(nt, g, n_xi, inv, r, b, x, omega, s);
        case 2: return vanka_nt<DIM, 2, T>(nt, g, n_xi, inv, r, b, x, omega, s);
        case 3: return vanka_nt<DIM, 3, T>(nt, g, n_xi, inv, r, b, x, omega, s);
        case 4: return vanka_nt<DIM, 4, T>(nt, g, n_xi, inv, r, b, x, omega, s);
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
hipError_t launch_vanka_apply(int dim, int k, int nt, Grid g, int n_xi, const T* inv, const T* r, const T* b,
                              T* x, T omega, hipStream_t s) {
    if (dim == 2) return vanka_k<2, T>(k, nt, g, n_xi, inv, r, b, x, omega, s);
    if (dim == 3) return vanka_k<3, T>(k, nt, g, n_xi, inv, r, b, x, omega, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_vanka_apply<double>(int, int, int, Grid, int, const double*, const double*,
                                               const double*, double*, double, hipStream_t);
template hipError_t launch_vanka_apply<float>(int, int, int, Grid, int, const float*, const float*, const float*,
                                              float*, float, hipStream_t);

}  // namespace sg
