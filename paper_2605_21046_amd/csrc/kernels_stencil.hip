// The mean-block operator of a level with a constant mean coefficient, as a Kronecker sum.
//
// The preconditioner's diagonal block (Remark solver-matrix-free-sg) is A_0 = A_t (x) M + B_t (x) K_0 on
// every stochastic mode.  On the uniform Cartesian Q_k mesh with the mean coefficient equal to one
// constant c, the Galerkin matrices factor exactly into assembled 1D matrices (M1: mass, K1: stiffness,
// both (2k+1)-banded):
//     M = M1 (x) M1 (x) M1,     K_0 = c (K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1)
// (in 2D the two-factor forms), so A_0 x is a separable stencil over the node grid: no cells, no
// cell-local copies of shared nodes and no gather pass.  The arithmetic is that of the element route
// up to rounding order (the 1D matrices are the same Gauss-quadrature integrals, assembled).
//
// 3D: a workgroup takes one mode (all N_t time components), TY node rows along y (plus k halo rows on
// each side) over the full x range, and a chunk of z planes.  Each thread keeps, for its (y, x)
// positions, the 2k+1 input planes around the current z in registers and forms the z products there;
// the y and x products go through LDS.  Per output plane:
//     P = (M1)_z u, Q = (K1)_z u                    (registers -> LDS)
//     A = (M1)_y P, B = (K1)_y P + (M1)_y Q          (LDS)
//     M u = (M1)_x A, K u = (K1)_x A + (M1)_x B      (LDS -> registers)
//     y_i = sum_j A_t[i][j] (M u_j) + B_t[i] c (K u_i)
// 2D: the same without the z direction (one pass over a block of rows).
//
// Dirichlet columns are dropped: inputs outside the mesh or on its boundary enter as zero.  Every load
// is unconditional (from a clamped, valid address; masked where the value is used), so no load waits
// on an earlier one: on this architecture loads and stores share one counter, and a load under a
// branch would make the next use wait for the previous plane's stores too.  The Dirichlet rows
// (y = x, or b - x for the residual form) are written by a separate pass over the boundary nodes.
#include <algorithm>
#include <cstdlib>

#include "kernels.hpp"

namespace sg {

namespace {

// 3D: 1024 (y, x) positions and output nodes per workgroup, one per thread in workgroups of 1024 threads
// where the z window of a position is small (FP64 with N_t (2k+1) <= 10: 16 waves per CU at about 113
// VGPRs), two per thread in workgroups of 512 otherwise (a larger window at 1024 threads spills, and
// the FP32 kernels keep two 512-thread workgroups per CU).
constexpr int kStSlots = 1024;
template <typename T, int K, int NT>
constexpr int st_threads() { return (sizeof(T) == 8 && NT * (2 * K + 1) <= 10) ? 1024 : 512; }
constexpr int kStThreads2d = 512;

template <typename T, int K, int NT>
__device__ __forceinline__ void st_x_pass(const T* Mb, const T* Kb, const T* A, const T* B, int rows_out, int n1,
                                          int yo, int xx, T* mu, T* ku) {
    constexpr int W = 2 * K + 1;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        T m = T(0), kk = T(0);
        const T* ar = A + (t * rows_out + yo) * n1;
        const T* br = B + (t * rows_out + yo) * n1;
#pragma unroll
        for (int d = 0; d < W; ++d) {
            const int xi = min(max(xx - K + d, 0), n1 - 1);     // band entries beyond the mesh are zero
            const T mb = Mb[xx * W + d], kb = Kb[xx * W + d];
            const T av = ar[xi], bv = br[xi];
            m += mb * av;
            kk += kb * av + mb * bv;
        }
        mu[t] = m;
        ku[t] = kk;
    }
}

// y = A_0 x (or b - A_0 x) at an interior node from M u and K u of all time components; bv: b there
template <typename T, int NT, bool RES>
__device__ __forceinline__ void st_store(const StencilArgs& a, long long nn, long long node, const T* mu,
                                         const T* ku, const T* bv) {
    T* y = static_cast<T*>(a.y);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        T v = (T)a.Bt[t] * ku[t];
#pragma unroll
        for (int j = 0; j < NT; ++j) v += (T)a.At[t * NT + j] * mu[j];
        y[((long long)a.mode * NT + t) * nn + node] = RES ? bv[t] - v : v;
    }
}

template <typename T, int K, int NT, bool RES>
__global__ void __launch_bounds__((st_threads<T, K, NT>())) k_mean_stencil_3d(StencilArgs a) {
    constexpr int W = 2 * K + 1;
    constexpr int kStThreads = st_threads<T, K, NT>();
    constexpr int kStPos = kStSlots / kStThreads;     // (y, x) positions per thread in the z march
    constexpr int kStOut = kStSlots / kStThreads;     // output nodes per thread and plane
    extern __shared__ __align__(16) unsigned char st_lds[];
    const int n1 = a.n1, TY = a.ty, ZC = a.zc;
    const int rows = TY + 2 * K;
    const long long nn = (long long)n1 * n1 * n1;
    const int nyt = (n1 + TY - 1) / TY, nzc = (n1 + ZC - 1) / ZC;
    int blk = blockIdx.x;
    const int yt = blk % nyt;
    blk /= nyt;
    const int zc = blk % nzc;
    a.mode = blk / nzc;
    const int y0 = yt * TY, z0 = zc * ZC, z1 = min(n1, z0 + ZC);
    T* Mb = reinterpret_cast<T*>(st_lds);           // [n1][W]
    T* Kb = Mb + n1 * W;                             // [n1][W], scaled by c
    T* P = Kb + n1 * W;                              // [NT][rows][n1]
    T* Q = P + NT * rows * n1;                       // [NT][rows][n1]
    T* A = Q + NT * rows * n1;                       // [NT][TY][n1]
    T* B = A + NT * TY * n1;                         // [NT][TY][n1]
    for (int i = threadIdx.x; i < n1 * W; i += kStThreads) {
        Mb[i] = static_cast<const T*>(a.Mb)[i];
        Kb[i] = static_cast<const T*>(a.Kb)[i];
    }
    const T* x = static_cast<const T*>(a.x) + (long long)a.mode * NT * nn;
    const T* b = RES ? static_cast<const T*>(a.b) + (long long)a.mode * NT * nn : nullptr;
    const int npos = rows * n1;
    // positions of this thread: (yy, xx) with global y = y0 - K + yy; pin: an interior node of the mesh
    // (the others enter as zero); paddr: the clamped node of its loads
    int pyy[kStPos], pxx[kStPos];
    bool pin[kStPos];
    long long paddr[kStPos];
#pragma unroll
    for (int i = 0; i < kStPos; ++i) {
        const int p = threadIdx.x + i * kStThreads;
        pyy[i] = p / n1;
        pxx[i] = p - pyy[i] * n1;
        const int gy = y0 - K + pyy[i];
        pin[i] = p < npos && gy > 0 && gy < n1 - 1 && pxx[i] > 0 && pxx[i] < n1 - 1;
        paddr[i] = (long long)min(max(gy, 0), n1 - 1) * n1 + min(pxx[i], n1 - 1);
    }
    auto zaddr = [&](int z) -> long long { return (long long)min(max(z, 0), n1 - 1) * n1 * n1; };
    auto zin = [&](int z) -> bool { return z > 0 && z < n1 - 1; };
    T win[kStPos][NT][W];
#pragma unroll
    for (int d = 0; d < W; ++d) {
        const long long za = zaddr(z0 - K + d);
#pragma unroll
        for (int i = 0; i < kStPos; ++i)
#pragma unroll
            for (int t = 0; t < NT; ++t) win[i][t][d] = x[t * nn + za + paddr[i]];
    }
#pragma unroll
    for (int d = 0; d < W; ++d) {
        const bool zi = zin(z0 - K + d);
#pragma unroll
        for (int i = 0; i < kStPos; ++i)
#pragma unroll
            for (int t = 0; t < NT; ++t) win[i][t][d] = (pin[i] && zi) ? win[i][t][d] : T(0);
    }
    // this thread's output nodes of a plane: (yo, xx) = it / n1, it % n1 with it = tid + u * threads;
    // oon: an interior node of the mesh (the boundary rows are written by their own pass)
    int oyo[kStOut], oxx[kStOut];
    bool oon[kStOut];
#pragma unroll
    for (int u = 0; u < kStOut; ++u) {
        const int it = threadIdx.x + u * kStThreads;
        oyo[u] = min(it / n1, TY - 1);
        oxx[u] = it - (it / n1) * n1;
        const int gy = y0 + oyo[u];
        oon[u] = it < TY * n1 && gy > 0 && gy < n1 - 1 && oxx[u] > 0 && oxx[u] < n1 - 1;
    }
    __syncthreads();
    T nxt[kStPos][NT];
    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;
        // z products of plane z in registers, to LDS
#pragma unroll
        for (int i = 0; i < kStPos; ++i) {
            const int p = threadIdx.x + i * kStThreads;
            if (p < npos) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    T pv = T(0), qv = T(0);
#pragma unroll
                    for (int d = 0; d < W; ++d) {
                        pv += Mb[z * W + d] * win[i][t][d];
                        qv += Kb[z * W + d] * win[i][t][d];
                    }
                    P[(t * rows + pyy[i]) * n1 + pxx[i]] = pv;
                    Q[(t * rows + pyy[i]) * n1 + pxx[i]] = qv;
                }
            }
        }
        // loads in flight across the y products: plane z + K + 1 (consumed at the end of the iteration)
        // and b at this plane's output nodes
        {
            const long long za = zaddr(z + 1 + K);
#pragma unroll
            for (int i = 0; i < kStPos; ++i)
#pragma unroll
                for (int t = 0; t < NT; ++t) nxt[i][t] = x[t * nn + za + paddr[i]];
        }
        T obv[kStOut][NT];
#pragma unroll
        for (int u = 0; u < kStOut; ++u) {
            const long long node = ((long long)z * n1 + y0 + oyo[u]) * n1 + oxx[u];
#pragma unroll
            for (int t = 0; t < NT; ++t) obv[u][t] = RES ? b[t * nn + node] : T(0);
        }
        __syncthreads();
        // y products of the TY output rows
        for (int it = threadIdx.x; it < NT * TY * n1; it += kStThreads) {
            const int t = it / (TY * n1);
            const int rem = it - t * TY * n1;
            const int yo = rem / n1, xx = rem - yo * n1;
            const int gy = min(y0 + yo, n1 - 1);
            T av = T(0), bv = T(0);
#pragma unroll
            for (int d = 0; d < W; ++d) {
                const T pv = P[(t * rows + yo + d) * n1 + xx], qv = Q[(t * rows + yo + d) * n1 + xx];
                av += Mb[gy * W + d] * pv;
                bv += Kb[gy * W + d] * pv + Mb[gy * W + d] * qv;
            }
            A[(t * TY + yo) * n1 + xx] = av;
            B[(t * TY + yo) * n1 + xx] = bv;
        }
        __syncthreads();
        // the window moves to plane z + 1 before this plane's stores (its loads are complete by now; a
        // wait placed after the stores would wait for them as well)
        if (more) {
            const bool zn = zin(z + 1 + K);
#pragma unroll
            for (int i = 0; i < kStPos; ++i)
#pragma unroll
                for (int t = 0; t < NT; ++t) {
#pragma unroll
                    for (int d = 0; d + 1 < W; ++d) win[i][t][d] = win[i][t][d + 1];
                    win[i][t][W - 1] = (pin[i] && zn) ? nxt[i][t] : T(0);
                }
        }
        // x products, time coupling, store (interior nodes)
        const bool zi = zin(z);
#pragma unroll
        for (int u = 0; u < kStOut; ++u) {
            if (!(oon[u] && zi)) continue;
            T mu[NT], ku[NT];
            st_x_pass<T, K, NT>(Mb, Kb, A, B, TY, n1, oyo[u], oxx[u], mu, ku);
            st_store<T, NT, RES>(a, nn, ((long long)z * n1 + y0 + oyo[u]) * n1 + oxx[u], mu, ku, obv[u]);
        }
    }
}

template <typename T, int K, int NT, bool RES>
__global__ void __launch_bounds__(kStThreads2d) k_mean_stencil_2d(StencilArgs a) {
    constexpr int kStThreads = kStThreads2d;
    constexpr int W = 2 * K + 1;
    extern __shared__ __align__(16) unsigned char st_lds[];
    const int n1 = a.n1, TY = a.ty;
    const int rows = TY + 2 * K;
    const long long nn = (long long)n1 * n1;
    const int nyt = (n1 + TY - 1) / TY;
    const int yt = blockIdx.x % nyt;
    a.mode = blockIdx.x / nyt;
    const int y0 = yt * TY;
    T* Mb = reinterpret_cast<T*>(st_lds);           // [n1][W]
    T* Kb = Mb + n1 * W;                             // [n1][W], scaled by c
    T* U = Kb + n1 * W;                              // [NT][rows][n1]
    T* A = U + NT * rows * n1;                       // [NT][TY][n1]
    T* B = A + NT * TY * n1;                         // [NT][TY][n1]
    for (int i = threadIdx.x; i < n1 * W; i += kStThreads) {
        Mb[i] = static_cast<const T*>(a.Mb)[i];
        Kb[i] = static_cast<const T*>(a.Kb)[i];
    }
    const T* x = static_cast<const T*>(a.x) + (long long)a.mode * NT * nn;
    const T* b = RES ? static_cast<const T*>(a.b) + (long long)a.mode * NT * nn : nullptr;
    for (int it = threadIdx.x; it < NT * rows * n1; it += kStThreads) {
        const int t = it / (rows * n1);
        const int rem = it - t * rows * n1;
        const int yy = rem / n1, xx = rem - yy * n1;
        const int gy = y0 - K + yy;
        const bool in = gy > 0 && gy < n1 - 1 && xx > 0 && xx < n1 - 1;
        const T v = x[t * nn + (long long)min(max(gy, 0), n1 - 1) * n1 + xx];
        U[it] = in ? v : T(0);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < NT * TY * n1; it += kStThreads) {
        const int t = it / (TY * n1);
        const int rem = it - t * TY * n1;
        const int yo = rem / n1, xx = rem - yo * n1;
        const int gy = min(y0 + yo, n1 - 1);
        T av = T(0), bv = T(0);
#pragma unroll
        for (int d = 0; d < W; ++d) {
            const T uv = U[(t * rows + yo + d) * n1 + xx];
            av += Mb[gy * W + d] * uv;
            bv += Kb[gy * W + d] * uv;
        }
        A[(t * TY + yo) * n1 + xx] = av;
        B[(t * TY + yo) * n1 + xx] = bv;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < TY * n1; it += kStThreads) {
        const int yo = it / n1, xx = it - yo * n1;
        const int gy = y0 + yo;
        if (!(gy > 0 && gy < n1 - 1 && xx > 0 && xx < n1 - 1)) continue;
        const long long node = (long long)gy * n1 + xx;
        T mu[NT], ku[NT], bv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) bv[t] = RES ? b[t * nn + node] : T(0);
        st_x_pass<T, K, NT>(Mb, Kb, A, B, TY, n1, yo, xx, mu, ku);
        st_store<T, NT, RES>(a, nn, node, mu, ku, bv);
    }
}

// Dirichlet rows: y = x (or b - x) on every boundary node of every component; one thread per node of
// the boundary of one component (blockIdx.y), the nodes enumerated face by face without repeats.
template <typename T, bool RES>
__global__ void __launch_bounds__(256) k_mean_stencil_boundary(StencilArgs a, long long nb) {
    const int n1 = a.n1;
    const long long nn = a.dim == 3 ? (long long)n1 * n1 * n1 : (long long)n1 * n1;
    const long long comp = blockIdx.y;
    const T* x = static_cast<const T*>(a.x) + comp * nn;
    const T* b = RES ? static_cast<const T*>(a.b) + comp * nn : nullptr;
    T* y = static_cast<T*>(a.y) + comp * nn;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < nb; i += (long long)gridDim.x * 256) {
        long long node;
        if (a.dim == 2) {
            // rows y = 0 and y = n1 - 1 (full), then columns x = 0 and x = n1 - 1 of the inner rows
            const long long full = 2LL * n1;
            if (i < full) {
                node = (i < n1 ? 0 : (long long)(n1 - 1) * n1) + i % n1;
            } else {
                const long long j = i - full;
                node = (1 + j / 2) * n1 + (j % 2 ? n1 - 1 : 0);
            }
        } else {
            // planes z = 0 and z = n1 - 1 (full), then on the inner planes the rows y = 0, n1 - 1 (full)
            // and the columns x = 0, n1 - 1 of the inner rows
            const long long plane = (long long)n1 * n1;
            const long long per_inner = 2LL * n1 + 2LL * (n1 - 2);
            if (i < 2 * plane) {
                node = (i < plane ? 0 : (long long)(n1 - 1) * plane) + i % plane;
            } else {
                const long long j = i - 2 * plane;
                const long long r = j % per_inner;
                long long yx;
                if (r < 2LL * n1) {
                    yx = (r < n1 ? 0 : (long long)(n1 - 1) * n1) + r % n1;
                } else {
                    const long long q = r - 2LL * n1;
                    yx = (1 + q / 2) * n1 + (q % 2 ? n1 - 1 : 0);
                }
                node = (1 + j / per_inner) * plane + yx;
            }
        }
        y[node] = RES ? b[node] - x[node] : x[node];
    }
}

long long boundary_nodes(int dim, int n1) {
    if (dim == 2) return 2LL * n1 + 2LL * (n1 - 2);
    return 2LL * n1 * n1 + (long long)(n1 - 2) * (2LL * n1 + 2LL * (n1 - 2));
}

template <typename T, int K, int NT, bool RES>
hipError_t launch_knt(const StencilArgs& a, hipStream_t s) {
    const size_t lds = stencil_lds_bytes(a, sizeof(T));
    const int nyt = (a.n1 + a.ty - 1) / a.ty;
    if (a.dim == 3) {
        const int nzc = (a.n1 + a.zc - 1) / a.zc;
        const long long blocks = (long long)a.n_xi * nyt * nzc;
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void*)k_mean_stencil_3d<T, K, NT, RES>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_mean_stencil_3d<T, K, NT, RES>), dim3((unsigned)blocks), dim3(st_threads<T, K, NT>()), lds, s,
                           a);
    } else {
        const long long blocks = (long long)a.n_xi * nyt;
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void*)k_mean_stencil_2d<T, K, NT, RES>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_mean_stencil_2d<T, K, NT, RES>), dim3((unsigned)blocks), dim3(kStThreads2d), lds, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nb = boundary_nodes(a.dim, a.n1);
    const long long gx = std::min<long long>((nb + 255) / 256, 1024);
    hipLaunchKernelGGL((k_mean_stencil_boundary<T, RES>), dim3((unsigned)gx, (unsigned)(a.n_xi * a.nt)), dim3(256), 0,
                       s, a, nb);
    return hipGetLastError();
}

template <typename T, int K, int NT>
hipError_t launch_kn(const StencilArgs& a, hipStream_t s) {
    return a.b ? launch_knt<T, K, NT, true>(a, s) : launch_knt<T, K, NT, false>(a, s);
}

template <typename T, int K>
hipError_t launch_k(const StencilArgs& a, hipStream_t s) {
    switch (a.nt) {
    case 1: return launch_kn<T, K, 1>(a, s);
    case 2: return launch_kn<T, K, 2>(a, s);
    case 3: return launch_kn<T, K, 3>(a, s);
    case 4: return launch_kn<T, K, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t stencil_lds_bytes(const StencilArgs& a, int elem) {
    const int W = 2 * a.k + 1, rows = a.ty + 2 * a.k;
    long long n = 2LL * a.n1 * W;
    if (a.dim == 3) n += 2LL * a.nt * rows * a.n1 + 2LL * a.nt * a.ty * a.n1;
    else n += (long long)a.nt * rows * a.n1 + 2LL * a.nt * a.ty * a.n1;
    return (size_t)n * elem;
}

bool stencil_fits(StencilArgs& a, int elem) {
    // rows per workgroup: as many as the positions of the z march (3D) and 160 KB of LDS allow, up to 10
    // in 3D (c2 FP64: 236 us with 8 rows, 194 with 10, 211 with 11) and 8 in 2D.
    // z planes per workgroup: about 16 (SGHEAT_STENCIL_ZC overrides; a measurement switch), split evenly:
    // each workgroup loads 2k window planes before its first output plane, so longer chunks read less
    // (chunks of 8: c3 FP64 678 us, 15: 608 us, 19: 630 us, the last with a worse final round of
    // workgroups; c2 FP64 251 / 241 / 237 us at 8 / 13 / 22)
    const int k = a.k;
    int zt = 16;
    if (const char* e = std::getenv("SGHEAT_STENCIL_ZC")) zt = std::max(1, std::atoi(e));
    const int nzc = (a.n1 + zt - 1) / zt;
    const int tymax = a.dim == 3 ? 10 : 8;
    for (int ty = tymax; ty >= 1; --ty) {
        a.ty = ty;
        a.zc = (a.n1 + nzc - 1) / nzc;
        if (a.dim == 3 && (long long)(ty + 2 * k) * a.n1 > kStSlots) continue;
        if (a.dim == 3 && (long long)ty * a.n1 > kStSlots) continue;
        if (stencil_lds_bytes(a, elem) > 160 * 1024) continue;
        return true;
    }
    return false;
}

template <typename T>
hipError_t launch_mean_stencil(const StencilArgs& args, hipStream_t s) {
    StencilArgs a = args;
    if (a.n1 < 3 || a.n_xi < 1 || a.nt < 1 || a.nt > kMaxNT || (long long)a.n_xi * a.nt > 65535 ||
        !stencil_fits(a, sizeof(T)))
        return hipErrorInvalidValue;
    switch (a.k) {
    case 1: return launch_k<T, 1>(a, s);
    case 2: return launch_k<T, 2>(a, s);
    case 3: return launch_k<T, 3>(a, s);
    case 4: return launch_k<T, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_mean_stencil<double>(const StencilArgs&, hipStream_t);
template hipError_t launch_mean_stencil<float>(const StencilArgs&, hipStream_t);

}  // namespace sg
