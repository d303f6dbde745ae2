// Forcing assembly, separable slab vectors and space-time error sums for prescribed solutions.
//
// k_load_cells:  per (cell, field) workgroup, per local node: the quadrature sum
//                sum_q w_q |K| (f_q psi_a(x_q) + g_q . grad psi_a(x_q)) into the broken-node layout
//                (k_node_gather then sums the cells of every node).
// k_separable:   y = beta y + sum_t W[t][comp] V[t][node].
// k_error_cells: per cell, the space-time quadrature of the error of a slab vector against the
//                separable field c_alpha theta(t) s(x), plus the mean and variance errors.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "forcing.hpp"

namespace sg {

namespace {

template <int N>
__device__ inline double wave_sum(double v) {
    for (int off = N / 2; off > 0; off >>= 1) v += __shfl_down(v, off, N);
    return v;
}

template <int DIM, int K>
__global__ void __launch_bounds__(128)
    k_load_cells(Grid g, int nq1, QTables tb, double h, const double* __restrict__ f, const double* __restrict__ gq,
                 double* __restrict__ S) {
    constexpr int N1 = K + 1;
    constexpr int NP = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    const int a = threadIdx.x;
    if (a >= NP) return;
    const long long cell = blockIdx.x;
    const int field = blockIdx.y;
    const int nq = DIM == 2 ? nq1 * nq1 : nq1 * nq1 * nq1;
    const int n = g.n;
    int cc[3] = {0, 0, 0}, aa[3] = {0, 0, 0};
    long long r = cell;
    int ra = a;
    for (int d = 0; d < DIM; ++d) {
        cc[d] = (int)(r % n);
        r /= n;
        aa[d] = ra % N1;
        ra /= N1;
    }
    double vol = 1.0;
    for (int d = 0; d < DIM; ++d) vol *= h;
    const long long base = ((long long)field * g.n_cells + cell) * nq;
    double acc = 0.0;
    for (int q = 0; q < nq; ++q) {
        int qq[3] = {0, 0, 0};
        int rq = q;
        double w = vol;
        for (int d = 0; d < DIM; ++d) {
            qq[d] = rq % nq1;
            rq /= nq1;
            w *= tb.w[qq[d]];
        }
        double psi = 1.0;
        for (int d = 0; d < DIM; ++d) psi *= tb.V[qq[d]][aa[d]];
        double val = f ? f[base + q] * psi : 0.0;
        if (gq) {
            for (int e = 0; e < DIM; ++e) {
                double de = 1.0 / h;
                for (int d = 0; d < DIM; ++d) de *= (d == e ? tb.D[qq[d]][aa[d]] : tb.V[qq[d]][aa[d]]);
                val += gq[(base + q) * DIM + e] * de;
            }
        }
        acc += w * val;
    }
    const long long nb1 = (long long)n * N1;
    long long off = 0, mul = 1;
    for (int d = 0; d < DIM; ++d) {
        off += (long long)(cc[d] * N1 + aa[d]) * mul;
        mul *= nb1;
    }
    S[(long long)field * mul + off] = acc;
}

__global__ void __launch_bounds__(256)
    k_separable(int n_terms, int ncomp, long long nn, const double* __restrict__ W, const double* __restrict__ V,
                double beta, double* __restrict__ y) {
    const int comp = blockIdx.y;
    for (long long node = blockIdx.x * 256LL + threadIdx.x; node < nn; node += (long long)gridDim.x * 256) {
        double s = 0.0;
        for (int t = 0; t < n_terms; ++t) s += W[(long long)t * ncomp + comp] * V[(long long)t * nn + node];
        const long long gi = (long long)comp * nn + node;
        y[gi] = (beta == 0.0 ? 0.0 : beta * y[gi]) + s;
    }
}

// One wave per cell; the cell's slab values (every mode and time DoF) are staged in LDS.
template <int DIM, int K, int NT>
__global__ void __launch_bounds__(64)
    k_error_cells(Grid g, int nq1, QTables tb, double h, TimeTables tt, int n_xi, const double* __restrict__ u,
                  const double* __restrict__ c, double C2, const double* __restrict__ s_qp,
                  const double* __restrict__ gs_qp, double* __restrict__ part) {
    constexpr int N1 = K + 1;
    constexpr int NP = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    extern __shared__ double lds[];                 // [n_xi * NT][NP]
    const int t = threadIdx.x;
    const long long cell = blockIdx.x;
    const int n = g.n, n1 = g.n1;
    const long long nn = g.n_nodes;
    int cc[3] = {0, 0, 0};
    {
        long long r = cell;
        for (int d = 0; d < DIM; ++d) {
            cc[d] = (int)(r % n);
            r /= n;
        }
    }
    const int ncomp = n_xi * NT;
    for (int idx = t; idx < ncomp * NP; idx += 64) {
        const int comp = idx / NP, a = idx % NP;
        int ra = a;
        long long node = 0, mul = 1;
        for (int d = 0; d < DIM; ++d) {
            node += (long long)(cc[d] * K + ra % N1) * mul;
            ra /= N1;
            mul *= n1;
        }
        lds[idx] = u[(long long)comp * nn + node];
    }
    __syncthreads();

    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int nq = DIM == 2 ? nq1 * nq1 : nq1 * nq1 * nq1;
    double vol = 1.0;
    for (int d = 0; d < DIM; ++d) vol *= h;
    for (int q = t; q < nq; q += 64) {
        int qq[3] = {0, 0, 0};
        int rq = q;
        double wq = vol;
        for (int d = 0; d < DIM; ++d) {
            qq[d] = rq % nq1;
            rq /= nq1;
            wq *= tb.w[qq[d]];
        }
        double psi[NP], dpsi[NP][DIM];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            int aa[3] = {0, 0, 0};
            int ra = a;
            for (int d = 0; d < DIM; ++d) {
                aa[d] = ra % N1;
                ra /= N1;
            }
            double p = 1.0;
            for (int d = 0; d < DIM; ++d) p *= tb.V[qq[d]][aa[d]];
            psi[a] = p;
            for (int e = 0; e < DIM; ++e) {
                double de = 1.0 / h;
                for (int d = 0; d < DIM; ++d) de *= (d == e ? tb.D[qq[d]][aa[d]] : tb.V[qq[d]][aa[d]]);
                dpsi[a][e] = de;
            }
        }
        const long long qi = cell * nq + q;
        const double s = s_qp[qi];
        double gs[DIM];
        for (int e = 0; e < DIM; ++e) gs[e] = gs_qp[qi * DIM + e];
        double sq[kMaxTimeQ], sg[kMaxTimeQ][DIM];
#pragma unroll
        for (int k = 0; k < kMaxTimeQ; ++k) {
            sq[k] = 0.0;
            for (int e = 0; e < DIM; ++e) sg[k][e] = 0.0;
        }
        for (int al = 0; al < n_xi; ++al) {
            double val[NT], gr[NT][DIM];
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const double* row = lds + (al * NT + i) * NP;
                double v = 0.0, gg[DIM];
                for (int e = 0; e < DIM; ++e) gg[e] = 0.0;
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    v += row[a] * psi[a];
                    for (int e = 0; e < DIM; ++e) gg[e] += row[a] * dpsi[a][e];
                }
                val[i] = v;
                for (int e = 0; e < DIM; ++e) gr[i][e] = gg[e];
            }
            const double ca = c[al];
#pragma unroll
            for (int k = 0; k < kMaxTimeQ; ++k) {
                if (k >= tt.ntq) break;
                double uh = 0.0, gh[DIM];
                for (int e = 0; e < DIM; ++e) gh[e] = 0.0;
#pragma unroll
                for (int i = 0; i < NT; ++i) {
                    uh += tt.v[i][k] * val[i];
                    for (int e = 0; e < DIM; ++e) gh[e] += tt.v[i][k] * gr[i][e];
                }
                const double th = tt.theta[k];
                const double w = tt.w[k] * wq;
                const double e0 = ca * th * s - uh;
                double ge2 = 0.0;
                for (int e = 0; e < DIM; ++e) {
                    const double d = ca * th * gs[e] - gh[e];
                    ge2 += d * d;
                }
                acc[0] += w * e0 * e0;
                acc[1] += w * ge2;
                if (al == 0) {
                    acc[2] += w * e0 * e0;
                    acc[3] += w * ge2;
                } else {
                    sq[k] += uh * uh;
                    for (int e = 0; e < DIM; ++e) sg[k][e] += uh * gh[e];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kMaxTimeQ; ++k) {
            if (k >= tt.ntq) break;
            const double th = tt.theta[k];
            const double w = tt.w[k] * wq;
            const double V = C2 * th * th * s * s - sq[k];
            double gv2 = 0.0, gs2 = 0.0;
            for (int e = 0; e < DIM; ++e) {
                const double d = 2.0 * C2 * th * th * s * gs[e] - 2.0 * sg[k][e];
                gv2 += d * d;
                gs2 += gs[e] * gs[e];
            }
            acc[4] += w * V * V;
            acc[5] += w * gv2;
            acc[6] += w * th * th * s * s;
            acc[7] += w * th * th * gs2;
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const double v = wave_sum<64>(acc[j]);
        if (t == 0) part[cell * 8 + j] = v;
    }
}

// Sample moments at the space-time quadrature points: acc[cell][q][tq][0..1] += (sum_s u_s, sum_s u_s^2)
// over the samples of a sample-batch slab vector.  One wave per cell, the cell's values in LDS.
template <int DIM, int K, int NT>
__global__ void __launch_bounds__(64)
    k_sample_qp_moments(Grid g, int nq1, QTables tb, TimeTables tt, int n_s, const double* __restrict__ u,
                        double* __restrict__ acc) {
    constexpr int N1 = K + 1;
    constexpr int NP = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    extern __shared__ double lds[];                 // [n_s * NT][NP]
    const int t = threadIdx.x;
    const long long cell = blockIdx.x;
    const int n = g.n, n1 = g.n1;
    const long long nn = g.n_nodes;
    int cc[3] = {0, 0, 0};
    {
        long long r = cell;
        for (int d = 0; d < DIM; ++d) {
            cc[d] = (int)(r % n);
            r /= n;
        }
    }
    const int ncomp = n_s * NT;
    for (int idx = t; idx < ncomp * NP; idx += 64) {
        const int comp = idx / NP, a = idx % NP;
        int ra = a;
        long long node = 0, mul = 1;
        for (int d = 0; d < DIM; ++d) {
            node += (long long)(cc[d] * K + ra % N1) * mul;
            ra /= N1;
            mul *= n1;
        }
        lds[idx] = u[(long long)comp * nn + node];
    }
    __syncthreads();
    const int nq = DIM == 2 ? nq1 * nq1 : nq1 * nq1 * nq1;
    for (int q = t; q < nq; q += 64) {
        int qq[3] = {0, 0, 0};
        int rq = q;
        for (int d = 0; d < DIM; ++d) {
            qq[d] = rq % nq1;
            rq /= nq1;
        }
        double psi[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            int ra = a;
            double p = 1.0;
            for (int d = 0; d < DIM; ++d) {
                p *= tb.V[qq[d]][ra % N1];
                ra /= N1;
            }
            psi[a] = p;
        }
        double s1[kMaxTimeQ], s2[kMaxTimeQ];
#pragma unroll
        for (int k = 0; k < kMaxTimeQ; ++k) s1[k] = s2[k] = 0.0;
        for (int sm = 0; sm < n_s; ++sm) {
            double val[NT];
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const double* row = lds + (sm * NT + i) * NP;
                double v = 0.0;
#pragma unroll
                for (int a = 0; a < NP; ++a) v += row[a] * psi[a];
                val[i] = v;
            }
#pragma unroll
            for (int k = 0; k < kMaxTimeQ; ++k) {
                if (k >= tt.ntq) break;
                double x = 0.0;
#pragma unroll
                for (int i = 0; i < NT; ++i) x += tt.v[i][k] * val[i];
                s1[k] += x;
                s2[k] += x * x;
            }
        }
        double* out = acc + (cell * nq + q) * (long long)tt.ntq * 2;
#pragma unroll
        for (int k = 0; k < kMaxTimeQ; ++k) {
            if (k >= tt.ntq) break;
            out[2 * k] += s1[k];
            out[2 * k + 1] += s2[k];
        }
    }
}

// Errors of the sample mean and unbiased sample variance (from acc over n_tot samples) against
// m_j theta s and v_j theta^2 s^2 (j = 0, 1); part[cell][6] = the four squared errors, |theta s|^2 and
// |theta^2 s^2|^2, integrated over the cell and the slab.
template <int DIM>
__global__ void __launch_bounds__(64)
    k_moment_errors(Grid g, int nq1, QTables tb, double h, TimeTables tt, double n_tot, const double* __restrict__ acc,
                    const double* __restrict__ s_qp, double m0, double m1, double v0, double v1,
                    double* __restrict__ part) {
    const int t = threadIdx.x;
    const long long cell = blockIdx.x;
    const int nq = DIM == 2 ? nq1 * nq1 : nq1 * nq1 * nq1;
    double vol = 1.0;
    for (int d = 0; d < DIM; ++d) vol *= h;
    double e[6] = {0, 0, 0, 0, 0, 0};
    for (int q = t; q < nq; q += 64) {
        int rq = q;
        double wq = vol;
        for (int d = 0; d < DIM; ++d) {
            wq *= tb.w[rq % nq1];
            rq /= nq1;
        }
        const double s = s_qp[cell * nq + q];
        const double* a = acc + (cell * nq + q) * (long long)tt.ntq * 2;
        for (int k = 0; k < tt.ntq; ++k) {
            const double w = tt.w[k] * wq;
            const double M = a[2 * k] / n_tot;
            const double V = (a[2 * k + 1] - n_tot * M * M) / (n_tot - 1.0);
            const double ph = tt.theta[k] * s;
            const double p2 = ph * ph;
            const double d0 = M - m0 * ph, d1 = M - m1 * ph, d2 = V - v0 * p2, d3 = V - v1 * p2;
            e[0] += w * d0 * d0;
            e[1] += w * d1 * d1;
            e[2] += w * d2 * d2;
            e[3] += w * d3 * d3;
            e[4] += w * p2;
            e[5] += w * p2 * p2;
        }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double v = wave_sum<64>(e[j]);
        if (t == 0) part[cell * 6 + j] = v;
    }
}

}  // namespace

hipError_t launch_load_cells(int dim, int k, Grid g, int nq1, const QTables& tb, double h, const double* f,
                             const double* gq, int nf, double* S, hipStream_t s) {
    const dim3 grid((unsigned)g.n_cells, (unsigned)nf);
#define SG_LC(D_, K_) hipLaunchKernelGGL((k_load_cells<D_, K_>), grid, dim3(128), 0, s, g, nq1, tb, h, f, gq, S)
    if (dim == 2) {
        switch (k) {
            case 1: SG_LC(2, 1); break;
            case 2: SG_LC(2, 2); break;
            case 3: SG_LC(2, 3); break;
            default: SG_LC(2, 4); break;
        }
    } else {
        switch (k) {
            case 1: SG_LC(3, 1); break;
            case 2: SG_LC(3, 2); break;
            case 3: SG_LC(3, 3); break;
            default: SG_LC(3, 4); break;
        }
    }
#undef SG_LC
    return hipGetLastError();
}

hipError_t launch_separable(int n_terms, int ncomp, long long nn, const double* W, const double* V, double beta,
                            double* y, hipStream_t s) {
    const unsigned bx = (unsigned)std::min<long long>((nn + 255) / 256, 4096);
    hipLaunchKernelGGL(k_separable, dim3(bx, (unsigned)ncomp), dim3(256), 0, s, n_terms, ncomp, nn, W, V, beta, y);
    return hipGetLastError();
}

bool error_cells_supported(int dim, int k, int nt) {
    return nt >= 1 && nt <= 4 && ((dim == 2 && k >= 1 && k <= 4) || (dim == 3 && k >= 1 && k <= 2));
}

hipError_t launch_error_cells(int dim, int k, int nt, Grid g, int nq1, const QTables& tb, double h,
                              const TimeTables& tt, int n_xi, const double* u, const double* c, double C2,
                              const double* s_qp, const double* gs_qp, double* part, hipStream_t s) {
    const int np = dim == 2 ? (k + 1) * (k + 1) : (k + 1) * (k + 1) * (k + 1);
    const size_t lds = (size_t)n_xi * nt * np * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    hipError_t err = hipErrorInvalidValue;
#define SG_EC(D_, K_, T_)                                                                                     \
    do {                                                                                                      \
        auto kern = k_error_cells<D_, K_, T_>;                                                                \
        if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kern, dim3((unsigned)g.n_cells), dim3(64), lds, s, g, nq1, tb, h, tt, n_xi, u, c, C2,  \
                           s_qp, gs_qp, part);                                                                 \
        err = hipGetLastError();                                                                              \
    } while (0)
#define SG_EC_T(D_, K_)                   \
    switch (nt) {                         \
        case 1: SG_EC(D_, K_, 1); break;  \
        case 2: SG_EC(D_, K_, 2); break;  \
        case 3: SG_EC(D_, K_, 3); break;  \
        default: SG_EC(D_, K_, 4); break; \
    }
    if (dim == 2) {
        switch (k) {
            case 1: SG_EC_T(2, 1); break;
            case 2: SG_EC_T(2, 2); break;
            case 3: SG_EC_T(2, 3); break;
            default: SG_EC_T(2, 4); break;
        }
    } else {
        switch (k) {
            case 1: SG_EC_T(3, 1); break;
            default: SG_EC_T(3, 2); break;
        }
    }
#undef SG_EC_T
#undef SG_EC
    return err;
}

hipError_t launch_sample_qp_moments(int dim, int k, int nt, Grid g, int nq1, const QTables& tb, const TimeTables& tt,
                                    int n_s, const double* u, double* acc, hipStream_t s) {
    const int np = dim == 2 ? (k + 1) * (k + 1) : (k + 1) * (k + 1) * (k + 1);
    const size_t lds = (size_t)n_s * nt * np * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    hipError_t err = hipErrorInvalidValue;
#define SG_SM(D_, K_, T_)                                                                                     \
    do {                                                                                                      \
        auto kern = k_sample_qp_moments<D_, K_, T_>;                                                          \
        if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kern, dim3((unsigned)g.n_cells), dim3(64), lds, s, g, nq1, tb, tt, n_s, u, acc);   \
        err = hipGetLastError();                                                                              \
    } while (0)
#define SG_SM_T(D_, K_)                   \
    switch (nt) {                         \
        case 1: SG_SM(D_, K_, 1); break;  \
        case 2: SG_SM(D_, K_, 2); break;  \
        case 3: SG_SM(D_, K_, 3); break;  \
        default: SG_SM(D_, K_, 4); break; \
    }
    if (dim == 2) {
        switch (k) {
            case 1: SG_SM_T(2, 1); break;
            case 2: SG_SM_T(2, 2); break;
            case 3: SG_SM_T(2, 3); break;
            default: SG_SM_T(2, 4); break;
        }
    } else {
        switch (k) {
            case 1: SG_SM_T(3, 1); break;
            default: SG_SM_T(3, 2); break;
        }
    }
#undef SG_SM_T
#undef SG_SM
    return err;
}

hipError_t launch_moment_errors(int dim, Grid g, int nq1, const QTables& tb, double h, const TimeTables& tt, double n_tot,
                                const double* acc, const double* s_qp, double m0, double m1, double v0, double v1,
                                double* part, hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL(k_moment_errors<2>, dim3((unsigned)g.n_cells), dim3(64), 0, s, g, nq1, tb, h, tt, n_tot, acc,
                           s_qp, m0, m1, v0, v1, part);
    else
        hipLaunchKernelGGL(k_moment_errors<3>, dim3((unsigned)g.n_cells), dim3(64), 0, s, g, nq1, tb, h, tt, n_tot, acc,
                           s_qp, m0, m1, v0, v1, part);
    return hipGetLastError();
}

}  // namespace sg
