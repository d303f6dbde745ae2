// Matrix-free application of the stochastic-Galerkin space-time slab operator
//     AA = I_xi (x) A_t (x) M_x + sum_mu G_mu (x) B_t (x) K_mu      (eq. local_rhs_tensor)
// on a uniform Cartesian Q_k mesh, by sum factorisation (Remark solver-matrix-free-sg: only the
// action of AA is formed).
//
// Work decomposition (gfx950, wave64):
//   * one workgroup = `cpb` cells of one colour x all N_xi * N_t components; one thread owns one
//     (cell, component) pair and keeps its (k+1)^d point values in registers;
//   * per thread: gather the cell's nodal values (Dirichlet columns dropped), interpolate to the
//     Gauss points (d 1D sweeps with the GLL-basis table), take reference derivatives by Gauss
//     collocation (d sweeps), and integrate back with the transposed sweeps;
//   * the two couplings that cross components go through LDS:
//       - time: the mass term needs sum_j A_t[i][j] u_j at each point,
//       - chaos: the stiffness flux of mode alpha is sum_mu a_mu(x_q) sum_beta [G_mu]_{alpha beta}
//         grad u_beta, read from the neighbours listed in the coupling CSR;
//   * continuous-FE scatter without atomics: cells are split into 2^d colours by coordinate
//     parity, one launch per colour; cells of one colour share no node.  A node's first writer
//     (lowest colour) stores, later colours read-modify-write, so the result is deterministic.
#pragma once

#include "kernels.hpp"

namespace sg {

namespace {

template <typename T>
struct ApplyArgs {
    const T* x;
    T* y;
    const T* b;
    const T* coef;
    long long coef_mode_stride;
    const int* cptr;
    const int* cbeta;
    const int* cmu;
    const T* cw;
    int n_xi, n_mu;
    Grid g;
    int par[3];
    int cnt[3];
    int cells_in_colour;
    int cpb;
};

// out[.., o, ..] (+)= sum_i M(o, i) in[.., i, ..] along direction DIR of an N1^DIM point block;
// M(o, i) = TR ? M[i*N1 + o] : M[o*N1 + i].
template <int DIM, int N1, int DIR, bool ACC, bool TR, typename T>
__device__ __forceinline__ void sweep(const T (&in)[ipow(N1, DIM)], T (&out)[ipow(N1, DIM)],
                                      const T* __restrict__ M) {
    constexpr int NP = ipow(N1, DIM);
    constexpr int st = ipow(N1, DIR);
#pragma unroll
    for (int base = 0; base < NP; ++base) {
        if ((base / st) % N1 != 0) continue;
#pragma unroll
        for (int o = 0; o < N1; ++o) {
            T acc = ACC ? out[base + o * st] : T(0);
#pragma unroll
            for (int i = 0; i < N1; ++i) acc += (TR ? M[i * N1 + o] : M[o * N1 + i]) * in[base + i * st];
            out[base + o * st] = acc;
        }
    }
}

// Keeps the scheduler from hoisting every unrolled load of a long loop ahead of its uses, which
// would otherwise blow the register budget and spill.
#define SG_FENCE() __builtin_amdgcn_sched_barrier(0)

__device__ __forceinline__ long long colour_cell(const int* par, const int* cnt, int n, int dim, int ci,
                                                 int* cc) {
    int r = ci;
    long long cell = 0, mul = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            cc[d] = 2 * (r % cnt[d]) + par[d];
            r /= cnt[d];
            cell += (long long)cc[d] * mul;
            mul *= n;
        } else {
            cc[d] = 0;
        }
    }
    return cell;
}

// Coloured scatter of one (cell, component) block: the lowest colour touching a node stores, the
// others read-modify-write; Dirichlet rows get the identity (y = x, or b - x for a residual).
template <int DIM, int K, typename T, bool RESID>
__device__ __forceinline__ void scatter(const ApplyArgs<T>& a, const T (&Y)[ipow(K + 1, DIM)], T bt,
                                        const int* cc, long long cbase) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    const int n = a.g.n, n1 = a.g.n1;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        long long node = 0, mul = 1;
        bool bnd = false, first = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int ad = (p / ipow(N1, d)) % N1;
            const int id = cc[d] * K + ad;
            bnd |= (id == 0) | (id == n1 - 1);
            const bool shared = (ad == 0 && cc[d] > 0) || (ad == K && cc[d] < n - 1);
            if (shared && a.par[d]) first = false;
            node += id * mul;
            mul *= n1;
        }
        const long long gi = cbase + node;
        if (bnd) {
            if (first) a.y[gi] = RESID ? a.b[gi] - a.x[gi] : a.x[gi];
        } else {
            const T v = Y[p] * bt;
            if (RESID) a.y[gi] = first ? a.b[gi] - v : a.y[gi] - v;
            else a.y[gi] = first ? v : a.y[gi] + v;
        }
        if (p % 9 == 8) SG_FENCE();
    }
}

// Points u_q of one (cell, component) at the Gauss points are in U; W accumulates the integrand.
// Slice s of direction DIR = the N1^(DIM-1) points with q_DIR = s.
template <int DIM, int N1, int DIR>
__device__ __forceinline__ constexpr int slice_point(int s, int j) {
    // j enumerates the other directions (x fastest), s is the index along DIR
    constexpr int st = ipow(N1, DIR);
    return (j / st) * st * N1 + s * st + (j % st);
}

// MODE 0: y = AA x;  MODE 1: y = b - AA x;  MODE 2: y = b - (I (x) A_0) x with the mean coefficient
// only (no chaos coupling, so the stiffness flux never leaves the thread).
template <int DIM, int K, int NT, typename T, int MODE>
__device__ __forceinline__ void apply_body(const ApplyArgs<T>& a, const Tables<T>& tb, T (&U)[ipow(K + 1, DIM)],
                                           T (&W)[ipow(K + 1, DIM)], T* slot_rows, const T* slot_coef,
                                           int comp, int alpha, int ti, bool active, const int* cc,
                                           long long cbase) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NS = NP / N1;   // points per slice
    T* const my_row = slot_rows + comp * NP;

    // time coupling of the mass term: W[q] = w_q h^d sum_j (A_t[i][j] / B_t[i]) u_j(q)
#pragma unroll
    for (int q = 0; q < NP; ++q) my_row[q] = U[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) W[q] = T(0);
#pragma unroll 1
    for (int j = 0; j < NT; ++j) {
        const T as = tb.As[ti * NT + j];
        const T* row = slot_rows + (alpha * NT + j) * NP;
#pragma unroll
        for (int q = 0; q < NP; ++q) W[q] += as * row[q];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        T wq = tb.vol;
#pragma unroll
        for (int d = 0; d < DIM; ++d) wq *= tb.w[(q / ipow(N1, d)) % N1];
        W[q] *= wq;
    }
    __syncthreads();

    if constexpr (MODE == 2) {
        // mean block: flux = a_0(x_q) * d u / d x_dir, all in registers
#pragma unroll
        for (int dir = 0; dir < DIM; ++dir) {
            const int st = ipow(N1, dir);
#pragma unroll
            for (int s = 0; s < N1; ++s) {
                T F[NS];
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int q = (j / st) * st * N1 + s * st + (j % st);
                    const int base = q - s * st;
                    T g = T(0);
#pragma unroll
                    for (int i = 0; i < N1; ++i) g += tb.D[s * N1 + i] * U[base + i * st];
                    F[j] = slot_coef[q] * g;
                }
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int q = (j / st) * st * N1 + s * st + (j % st);
                    const int base = q - s * st;
#pragma unroll
                    for (int o = 0; o < N1; ++o) W[base + o * st] += tb.D[s * N1 + o] * F[j];
                }
            }
        }
    } else {
    const int e0 = a.cptr[alpha * a.n_mu];
        const int e1 = a.cptr[(alpha + 1) * a.n_mu];
        // stiffness term, one reference direction at a time
    #pragma unroll
        for (int dir = 0; dir < DIM; ++dir) {
            const int st = ipow(N1, dir);
            // reference derivative along dir by Gauss collocation, written straight to LDS
    #pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int qd = (q / st) % N1;
                const int base = q - qd * st;
                T g = T(0);
    #pragma unroll
                for (int i = 0; i < N1; ++i) g += tb.D[qd * N1 + i] * U[base + i * st];
                my_row[q] = g;
            }
            __syncthreads();
            // flux of mode alpha on one slice at a time, then W += D^T flux along dir
    #pragma unroll
            for (int s = 0; s < N1; ++s) {
                T F[NS];
    #pragma unroll
                for (int j = 0; j < NS; ++j) F[j] = T(0);
    #pragma unroll 1
                for (int e = e0; e < e1; ++e) {
                    const int beta = a.cbeta[e];
                    const T w = a.cw[e];
                    const T* cp = slot_coef + a.cmu[e] * NP;
                    const T* gp = slot_rows + (beta * NT + ti) * NP;
    #pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const int q = (j / st) * st * N1 + s * st + (j % st);
                        F[j] += (w * cp[q]) * gp[q];
                    }
                }
    #pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int q = (j / st) * st * N1 + s * st + (j % st);
                    const int base = q - s * st;
    #pragma unroll
                    for (int o = 0; o < N1; ++o) W[base + o * st] += tb.D[s * N1 + o] * F[j];
                }
            }
            __syncthreads();
        }
    
    }

    // integrate back to the nodes and scatter
    if constexpr (DIM == 2) {
        sweep<DIM, N1, 0, false, true>(W, U, tb.S);
        sweep<DIM, N1, 1, false, true>(U, W, tb.S);
        if (active) scatter<DIM, K, T, MODE != 0>(a, W, tb.Bt[ti], cc, cbase);
    } else {
        sweep<DIM, N1, 0, false, true>(W, U, tb.S);
        sweep<DIM, N1, 1, false, true>(U, W, tb.S);
        sweep<DIM, N1, 2, false, true>(W, U, tb.S);
        if (active) scatter<DIM, K, T, MODE != 0>(a, U, tb.Bt[ti], cc, cbase);
    }
}

template <int DIM, int K, int NT, typename T, int MODE>
__global__ void __launch_bounds__(ipow(K + 1, DIM) > 27 ? 256 : 512) k_apply(ApplyArgs<T> a, Tables<T> tb) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    extern __shared__ unsigned char smem_raw[];
    const int cpb = a.cpb;
    const int NC = a.n_xi * NT;
    T* exch = reinterpret_cast<T*>(smem_raw);               // [cpb][NC][NP]
    T* cl = exch + (size_t)NC * NP * cpb;                    // [cpb][n_mu][NP]

    const int t = threadIdx.x;
    const int slot = t % cpb;
    const int comp = t / cpb;
    const int alpha = comp / NT;
    const int ti = comp % NT;
    const int ci = blockIdx.x * cpb + slot;
    const bool active = ci < a.cells_in_colour;
    const int n = a.g.n, n1 = a.g.n1;
    const long long nn = a.g.n_nodes;

    int cc[3];
    colour_cell(a.par, a.cnt, n, DIM, active ? ci : 0, cc);

    // stage the coefficient values of this block's cells
    for (int idx = t; idx < a.n_mu * NP * cpb; idx += blockDim.x) {
        const int q = idx % NP;
        const int mu = (idx / NP) % a.n_mu;
        const int s = idx / (NP * a.n_mu);
        const int c2 = blockIdx.x * cpb + s;
        T v = T(0);
        if (c2 < a.cells_in_colour) {
            int cq[3];
            const long long cell = colour_cell(a.par, a.cnt, n, DIM, c2, cq);
            v = a.coef[mu * a.coef_mode_stride + cell * NP + q];
        }
        cl[idx] = v;
    }

    T A[NP], B[NP];
    const long long cbase = ((long long)alpha * NT + ti) * nn;

    // gather (Dirichlet columns dropped)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        long long node = 0, mul = 1;
        bool bnd = false;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int ad = (p / ipow(N1, d)) % N1;
            const int id = cc[d] * K + ad;
            bnd |= (id == 0) | (id == n1 - 1);
            node += id * mul;
            mul *= n1;
        }
        A[p] = (active && !bnd) ? a.x[cbase + node] : T(0);
        if (p % 9 == 8) SG_FENCE();
    }

    T* const slot_rows = exch + (size_t)slot * NC * NP;
    const T* const slot_coef = cl + (size_t)slot * a.n_mu * NP;
    // values at the Gauss points, then the rest of the cell work
    if constexpr (DIM == 2) {
        sweep<DIM, N1, 0, false, false>(A, B, tb.S);
        sweep<DIM, N1, 1, false, false>(B, A, tb.S);
        apply_body<DIM, K, NT, T, MODE>(a, tb, A, B, slot_rows, slot_coef, comp, alpha, ti, active, cc, cbase);
    } else {
        sweep<DIM, N1, 0, false, false>(A, B, tb.S);
        sweep<DIM, N1, 1, false, false>(B, A, tb.S);
        sweep<DIM, N1, 2, false, false>(A, B, tb.S);
        apply_body<DIM, K, NT, T, MODE>(a, tb, B, A, slot_rows, slot_coef, comp, alpha, ti, active, cc, cbase);
    }
}

template <int DIM, int K, int NT, typename T>
hipError_t run_apply(const ApplyOp<T>& op, const T* x, T* y, const T* b, hipStream_t s) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    const int cpb = op.cells_per_block;
    ApplyArgs<T> a{};
    a.x = x;
    a.y = y;
    a.b = b;
    a.coef = op.coef;
    a.coef_mode_stride = op.coef_mode_stride;
    a.cptr = op.cptr;
    a.cbeta = op.cbeta;
    a.cmu = op.cmu;
    a.cw = op.cw;
    a.n_xi = op.n_xi;
    a.n_mu = op.n_mu;
    a.g = op.g;
    a.cpb = cpb;
    const int threads = op.n_xi * NT * cpb;
    const size_t lds = (size_t)(op.n_xi * NT + op.n_mu) * NP * cpb * sizeof(T);
    for (int colour = 0; colour < (1 << DIM); ++colour) {
        int cells = 1;
        for (int d = 0; d < 3; ++d) {
            if (d < DIM) {
                a.par[d] = (colour >> d) & 1;
                a.cnt[d] = (op.g.n - a.par[d] + 1) / 2;
            } else {
                a.par[d] = 0;
                a.cnt[d] = 1;
            }
            cells *= a.cnt[d];
        }
        a.cells_in_colour = cells;
        if (cells == 0) continue;
        const int blocks = (cells + cpb - 1) / cpb;
        const int mode = b ? (op.mean ? 2 : 1) : 0;
        auto kern = mode == 0 ? k_apply<DIM, K, NT, T, 0> : (mode == 1 ? k_apply<DIM, K, NT, T, 1> : k_apply<DIM, K, NT, T, 2>);
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, s, a, *op.tables);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int DIM, int K, typename T>
hipError_t dispatch_nt(const ApplyOp<T>& op, const T* x, T* y, const T* b, hipStream_t s) {
    switch (op.nt) {
        case 1: return run_apply<DIM, K, 1, T>(op, x, y, b, s);
        case 2: return run_apply<DIM, K, 2, T>(op, x, y, b, s);
        case 3: return run_apply<DIM, K, 3, T>(op, x, y, b, s);
        case 4: return run_apply<DIM, K, 4, T>(op, x, y, b, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// All (k, N_t) instances of one dimension and precision; instantiated in apply_<d>d_<type>.hip.
template <int DIM, typename T>
hipError_t apply_dim(const ApplyOp<T>& op, const T* x, T* y, const T* b, hipStream_t s) {
    switch (op.k) {
        case 1: return dispatch_nt<DIM, 1, T>(op, x, y, b, s);
        case 2: return dispatch_nt<DIM, 2, T>(op, x, y, b, s);
        case 3: return dispatch_nt<DIM, 3, T>(op, x, y, b, s);
        case 4: return dispatch_nt<DIM, 4, T>(op, x, y, b, s);
    }
    return hipErrorInvalidValue;
}


}  // namespace sg
