// Gram-Schmidt passes of FGMRES with the reorthogonalisation of each basis vector delayed into the next
// step (DCGS2).  Each step reads the basis twice (one fused dot pass, one fused update pass) where
// classical Gram-Schmidt with reorthogonalisation reads it three times.
#include <hip/hip_runtime.h>

#include "krylov.hpp"

namespace sg {

namespace {

constexpr int kKT = 256;              // threads per block
constexpr int kKW = kKT / 64;         // waves per block
constexpr int kKG = 16;               // basis vectors per register group of the dot pass

// Sum over the 64 lanes of a wave (fixed tree; lane 0 holds the result).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(kKT)
    k_dcgs_dots(const double* __restrict__ V, long long ldv, int j, const double* __restrict__ u,
                const double* __restrict__ w, long long n, double* __restrict__ partial) {
    __shared__ double red[(2 * kKG + 2) * kKW];
    const int nv = 2 * j + 2;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long stride = (long long)gridDim.x * kKT;
    const long long i0 = blockIdx.x * (long long)kKT + threadIdx.x;
    // groups of kKG basis vectors (u and w are read once per group); u.u and u.w with the first group
    for (int g0 = 0; g0 == 0 || g0 < j; g0 += kKG) {
        double aa[kKG], bb[kKG];
#pragma unroll
        for (int l = 0; l < kKG; ++l) aa[l] = bb[l] = 0.0;
        double cc = 0.0, dd = 0.0;
        for (long long i = i0; i < n; i += stride) {
            const double ui = u[i], wi = w[i];
            double v[kKG];
#pragma unroll
            for (int l = 0; l < kKG; ++l) v[l] = g0 + l < j ? V[(long long)(g0 + l) * ldv + i] : 0.0;
#pragma unroll
            for (int l = 0; l < kKG; ++l) {
                aa[l] += v[l] * ui;
                bb[l] += v[l] * wi;
            }
            cc += ui * ui;
            dd += ui * wi;
        }
#pragma unroll
        for (int l = 0; l < kKG; ++l) {
            if (g0 + l < j) {
                const double sa = wave_sum(aa[l]);
                const double sb = wave_sum(bb[l]);
                if (lane == 0) {
                    red[(2 * l) * kKW + wv] = sa;
                    red[(2 * l + 1) * kKW + wv] = sb;
                }
            }
        }
        if (g0 == 0) {
            const double sc = wave_sum(cc);
            const double sd = wave_sum(dd);
            if (lane == 0) {
                red[(2 * kKG) * kKW + wv] = sc;
                red[(2 * kKG + 1) * kKW + wv] = sd;
            }
        }
        __syncthreads();
        const int q = threadIdx.x;
        if (q < 2 * kKG + 2) {
            int dest = -1;
            if (q < 2 * kKG) {
                const int l = g0 + q / 2;
                if (l < j) dest = (q % 2 == 0) ? l : j + l;
            } else if (g0 == 0) {
                dest = 2 * j + (q - 2 * kKG);
            }
            if (dest >= 0) {
                double s = 0.0;
#pragma unroll
                for (int x = 0; x < kKW; ++x) s += red[q * kKW + x];
                partial[(long long)blockIdx.x * nv + dest] = s;
            }
        }
        __syncthreads();
    }
}

template <int KMAX>
__global__ void __launch_bounds__(kKT)
    k_dcgs_update(const double* __restrict__ V, long long ldv, int j, const double* __restrict__ r, double* u,
                  const double* __restrict__ w, double* __restrict__ unext, long long n, double* __restrict__ partial) {
    __shared__ double cf[2 * KMAX];
    __shared__ double red[kKW];
    for (int q = threadIdx.x; q < 2 * j; q += kKT) cf[q] = r[q];
    double ss = 0.0, ab = 0.0;
    for (int l = 0; l < j; ++l) {
        ss += r[l] * r[l];
        ab += r[l] * r[j + l];
    }
    const double nu2 = r[2 * j] - ss;
    const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
    const double e = nu > 0.0 ? (r[2 * j + 1] - ab) / nu : 0.0;
    const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
    __syncthreads();
    double nrm = 0.0;
    const long long stride = (long long)gridDim.x * kKT;
    for (long long i = blockIdx.x * (long long)kKT + threadIdx.x; i < n; i += stride) {
        double v[KMAX];
#pragma unroll
        for (int l = 0; l < KMAX; ++l) v[l] = l < j ? V[(long long)l * ldv + i] : 0.0;
        double s = u[i], t = w[i];
#pragma unroll
        for (int l = 0; l < KMAX; ++l) {
            if (l < j) {
                s -= cf[l] * v[l];
                t -= cf[j + l] * v[l];
            }
        }
        const double vi = s * inv;
        u[i] = vi;
        const double wn = t - e * vi;
        unext[i] = wn;
        nrm += wn * wn;
    }
    const double sw = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sw;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int x = 0; x < kKW; ++x) s += red[x];
        partial[blockIdx.x] = s;
    }
}

}  // namespace

hipError_t launch_dcgs_dots(const double* V, long long ldv, int j, const double* u, const double* w, long long n,
                            double* partial, int nblk, hipStream_t s) {
    if (j < 0 || j > kDcgsMaxBasis || nblk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dcgs_dots, dim3(nblk), dim3(kKT), 0, s, V, ldv, j, u, w, n, partial);
    return hipGetLastError();
}

hipError_t launch_dcgs_update(const double* V, long long ldv, int j, const double* r, double* u, const double* w,
                              double* unext, long long n, double* partial, int nblk, hipStream_t s) {
    if (j < 0 || j > kDcgsMaxBasis || nblk < 1) return hipErrorInvalidValue;
#define SG_DU(KM)                                                                                                   \
    if (j <= KM) {                                                                                                  \
        hipLaunchKernelGGL((k_dcgs_update<KM>), dim3(nblk), dim3(kKT), 0, s, V, ldv, j, r, u, w, unext, n, partial); \
        return hipGetLastError();                                                                                   \
    }
    SG_DU(8)
    SG_DU(16)
    SG_DU(32)
    SG_DU(64)
#undef SG_DU
    return hipErrorInvalidValue;
}

}  // namespace sg
