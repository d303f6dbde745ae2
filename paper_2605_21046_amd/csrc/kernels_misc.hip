// Grid transfers, coarsest-level solve and the vector kernels of the Krylov solver.
//
// Transfers: the prolongation is nodal interpolation of the coarse Q_k function at the fine nodes
// (zero on Dirichlet nodes); on a uniform hierarchy it is the tensor product of one 1D matrix per
// direction, so both P and R = P^T are applied as d banded 1D passes.
//
// Reductions are deterministic: a fixed number of blocks writes partial sums, and one block adds
// them in a fixed order.
#include <algorithm>

#include "fastdiv.hpp"
#include "kernels.hpp"

namespace sg {

namespace {

// One 1D transfer pass, one output element per thread.  Narrow form: every index of the pass fits
// in 31 bits (the launcher checks) and the divisions by the output extents use FastDiv.  W > 0: the
// band width as a compile-time constant, so the W table entries and inputs of an element are loaded
// together, unconditionally (every table entry holds a valid index), before the sum; the sum runs
// over w in order and skips zero weights, the same arithmetic as the runtime-width loop (W = 0),
// where each load waits for the weight test of its term.
template <typename T, int W>
__global__ void k_transfer_1d_narrow(int dim, unsigned total, int i0, int i1, FastDiv f0, FastDiv f1, FastDiv f2,
                                     int dir, const int* __restrict__ tidx, const T* __restrict__ tw, int width,
                                     const T* __restrict__ in, T* __restrict__ out, bool accumulate, unsigned in_comp) {
    const unsigned istr = dir == 0 ? 1u : (dir == 1 ? (unsigned)i0 : (unsigned)i0 * (unsigned)i1);
    for (unsigned idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        unsigned r = idx;
        unsigned q = fast_quot(f0, r);
        const int x0 = (int)(r - q * f0.d);
        r = q;
        q = fast_quot(f1, r);
        const int x1 = (int)(r - q * f1.d);
        r = q;
        int x2 = 0;
        if (dim == 3) {
            q = fast_quot(f2, r);
            x2 = (int)(r - q * f2.d);
            r = q;
        }
        const unsigned c = r;
        const int o = dir == 0 ? x0 : (dir == 1 ? x1 : x2);
        // input offset of the element with its coordinate along dir set to 0
        const unsigned ib = c * in_comp + ((unsigned)(dir == 2 ? 0 : x2) * (unsigned)i1 + (unsigned)(dir == 1 ? 0 : x1)) *
                                              (unsigned)i0 + (unsigned)(dir == 0 ? 0 : x0);
        T acc = T(0);
        if constexpr (W > 0) {
            T wt[W], v[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                wt[w] = tw[o * W + w];
                v[w] = in[ib + (unsigned)tidx[o * W + w] * istr];
            }
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (wt[w] != T(0)) acc += wt[w] * v[w];
        } else {
            for (int w = 0; w < width; ++w) {
                const T wt = tw[o * width + w];
                if (wt == T(0)) continue;
                acc += wt * in[ib + (unsigned)tidx[o * width + w] * istr];
            }
        }
        if (accumulate) out[idx] += acc;
        else out[idx] = acc;
    }
}

// The same pass with the inputs staged through LDS: a workgroup owns 64 columns (a column = every input
// along dir at one position of the other directions and one component) and loads each of their inputs
// from memory once, coalesced (for dir = 0 the 64 lines are one contiguous block), instead of once per
// table term; then wave v computes the outputs o = v, v + 4, ... of its lane's column, o being uniform
// over the wave, so the table entries are scalar loads.  Same terms in the same order as above (zero
// weights skipped), so the results are bitwise those of k_transfer_1d_narrow.
// Columns: c = outer n_inner + q; input (outer n_in + f) n_inner + q; output (outer n_out + o) n_inner + q.
template <typename T, int W>
__global__ void __launch_bounds__(256)
    k_transfer_1d_lds(unsigned ncols, unsigned n_in, unsigned n_out, unsigned n_inner, FastDiv f_inner,
                      const int* __restrict__ tidx, const T* __restrict__ tw, const T* __restrict__ in,
                      T* __restrict__ out, bool accumulate) {
    extern __shared__ unsigned char lds_raw[];
    T* const st = reinterpret_cast<T*>(lds_raw);
    const unsigned lane = threadIdx.x & 63u;
    const unsigned wave = (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const unsigned c0 = blockIdx.x * 64u;
    const unsigned c = c0 + lane;
    const bool live = c < ncols;
    const unsigned outer = n_inner == 1u ? c : fast_quot(f_inner, c);
    const unsigned q = c - outer * n_inner;
    if (n_inner == 1u) {
        // contiguous block of min(64, ncols - c0) lines of n_in values: st[line n_in + f]
        const unsigned nl = min(64u, ncols - c0);
        const T* const blk = in + (size_t)c0 * n_in;
        for (unsigned e = threadIdx.x; e < nl * n_in; e += 256u) st[e] = blk[e];
    } else {
        // st[f 64 + lane]
        for (unsigned f = wave; f < n_in; f += 4u)
            st[f * 64u + lane] = live ? in[((size_t)outer * n_in + f) * n_inner + q] : T(0);
    }
    __syncthreads();
    if (!live) return;
    const unsigned sstr = n_inner == 1u ? 1u : 64u;                  // LDS stride between inputs
    const T* const col = st + (n_inner == 1u ? lane * n_in : lane);
    for (unsigned o = wave; o < n_out; o += 4u) {
        T acc = T(0);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const T wt = tw[o * W + w];
            const T v = col[(unsigned)tidx[o * W + w] * sstr];
            if (wt != T(0)) acc += wt * v;
        }
        T* const dst = out + ((size_t)outer * n_out + o) * n_inner + q;
        if (accumulate) *dst += acc;
        else *dst = acc;
    }
}

// The same with 64-bit indices, for passes whose indices do not fit the narrow form.
template <typename T>
__global__ void k_transfer_1d(int dim, long long total, int i0, int i1, int o0, int o1, int o2, int dir,
                              const int* __restrict__ tidx, const T* __restrict__ tw, int width,
                              const T* __restrict__ in, T* __restrict__ out, bool accumulate,
                              long long in_comp) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        long long r = idx;
        const int x0 = r % o0;
        r /= o0;
        const int x1 = r % o1;
        r /= o1;
        int x2 = 0;
        if (dim == 3) { x2 = r % o2; r /= o2; }
        const long long c = r;
        const int o = dir == 0 ? x0 : (dir == 1 ? x1 : x2);
        T acc = T(0);
        for (int w = 0; w < width; ++w) {
            const T wt = tw[o * width + w];
            if (wt == T(0)) continue;
            const int src = tidx[o * width + w];
            const int y0 = dir == 0 ? src : x0;
            const int y1 = dir == 1 ? src : x1;
            const int y2 = dir == 2 ? src : x2;
            acc += wt * in[c * in_comp + ((long long)y2 * i1 + y1) * i0 + y0];
        }
        if (accumulate) out[idx] += acc;
        else out[idx] = acc;
    }
}

// Sum of the broken copies of each node (fixed order: lower cell first in every direction), then the
// requested update; one thread per node of one component (component = blockIdx.y), consecutive
// threads on consecutive x nodes.
// Quotients of the gather by its run-time extents as multiply-shift: nodes per direction, the x and z
// segment lengths.
struct GatherDivs {
    FastDiv n1, sx, sz;
};

template <typename T, int OP, int DIM, int K>
__global__ void __launch_bounds__(256)
    k_node_gather(Grid g, const T* __restrict__ s_in, const T* __restrict__ x, const T* __restrict__ b,
                  T* __restrict__ out, T omega, unsigned sx, unsigned sz, GatherDivs dv) {
    constexpr int N1 = K + 1;
    const unsigned n1 = g.n1, nc = g.n;
    const unsigned nb1 = nc * N1;
    // x (and z in 3D): segments of sx (sz) node intervals (K: one cell), sx + 1 broken entries each
    // except a shorter last one: (n1 - 1) + nsx entries in all
    const unsigned nsx = (n1 - 1 + sx - 1) / sx;
    const unsigned nbx = (n1 - 1) + nsx;
    const unsigned nsz = (n1 - 1 + sz - 1) / sz;
    const unsigned nbz = (n1 - 1) + nsz;
    unsigned nbn = nbx;
    if (DIM >= 2) nbn *= nb1;
    if (DIM == 3) nbn *= nbz;
    const unsigned nn = (unsigned)g.n_nodes;
    const long long comp = blockIdx.y;
    const T* sc = s_in + comp * (long long)nbn;
    const long long vbase = comp * (long long)nn;
    for (unsigned node = blockIdx.x * 256u + threadIdx.x; node < nn; node += gridDim.x * 256u) {
        unsigned r = node;
        // per direction: the broken index of this node in the lower and the upper cell (equal, with
        // weight 0 for the upper one, when the node lies inside a cell along that direction)
        unsigned lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        T whi[3] = {T(0), T(0), T(0)};
        T mult[3] = {T(1), T(1), T(1)};   // cells sharing the node along d (a layout may hold their sum)
        bool bnd = false;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            unsigned i = r;
            if (d < DIM - 1) {
                const unsigned q = fast_quot(dv.n1, r);
                i = r - q * n1;
                r = q;
            }
            bnd |= (i == 0) | (i == n1 - 1);
            if (i % (unsigned)K == 0) mult[d] = T(2);
            const unsigned sl = d == 0 ? sx : (d == 2 ? sz : (unsigned)K);   // segment length along d
            const unsigned ns = d == 0 ? nsx : (d == 2 ? nsz : nc);           // segments along d
            const unsigned c = d == 0 ? fast_quot(dv.sx, i) : (d == 2 ? fast_quot(dv.sz, i) : i / (unsigned)K);
            if (i == c * sl && i > 0 && i < n1 - 1) {
                lo[d] = (c - 1) * (sl + 1) + sl;
                hi[d] = c * (sl + 1);
                whi[d] = T(1);
            } else {
                const unsigned cl = c < ns ? c : ns - 1;
                lo[d] = cl * (sl + 1) + (i - cl * sl);
                hi[d] = lo[d];
            }
        }
        const long long gi = vbase + node;
        if (bnd) {
            if (OP == GATHER_SET) out[gi] = x[gi];
            else if (OP == GATHER_RESIDUAL) out[gi] = b[gi] - x[gi];
            else if (OP == GATHER_INTERIOR) out[gi] = T(0);
            else out[gi] = b[gi];
            continue;
        }
        // fixed summation order: lower before upper in x, then y, then z
        T sum = T(0);
        T cnt = T(1);
        if (DIM == 2) {
            const unsigned y0 = lo[1] * nbx, y1 = hi[1] * nbx;
            sum = (sc[y0 + lo[0]] + whi[0] * sc[y0 + hi[0]]) + whi[1] * (sc[y1 + lo[0]] + whi[0] * sc[y1 + hi[0]]);
            cnt = mult[0] * mult[1];
        } else {
            const unsigned z0 = lo[2] * nb1 * nbx, z1 = hi[2] * nb1 * nbx;
            const unsigned y0 = lo[1] * nbx, y1 = hi[1] * nbx;
            const T s00 = sc[z0 + y0 + lo[0]] + whi[0] * sc[z0 + y0 + hi[0]];
            const T s01 = sc[z0 + y1 + lo[0]] + whi[0] * sc[z0 + y1 + hi[0]];
            const T s10 = sc[z1 + y0 + lo[0]] + whi[0] * sc[z1 + y0 + hi[0]];
            const T s11 = sc[z1 + y1 + lo[0]] + whi[0] * sc[z1 + y1 + hi[0]];
            sum = (s00 + whi[1] * s01) + whi[2] * (s10 + whi[1] * s11);
            cnt = mult[0] * mult[1] * mult[2];
        }
        if (OP == GATHER_SET || OP == GATHER_INTERIOR) out[gi] = sum;
        else if (OP == GATHER_RESIDUAL) out[gi] = b[gi] - sum;
        else out[gi] = out[gi] + omega * sum / cnt;
    }
}

// Mean and unbiased variance over the N samples (component blocks s * nt + i) at every (i, node).
__global__ void __launch_bounds__(256)
    k_sample_stats(const double* __restrict__ u, int N, int nt, long long nn, double* __restrict__ mean,
                   double* __restrict__ var) {
    const long long total = (long long)nt * nn;
    for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
        const long long i = idx / nn, node = idx % nn;
        const double* p = u + i * nn + node;
        const long long stride = (long long)nt * nn;
        double s = 0.0;
        for (int k = 0; k < N; ++k) s += p[k * stride];
        const double m = s / N;
        mean[idx] = m;
        if (var) {
            double q = 0.0;
            for (int k = 0; k < N; ++k) {
                const double d = p[k * stride] - m;
                q += d * d;
            }
            var[idx] = N > 1 ? q / (N - 1) : 0.0;
        }
    }
}


// Chaos moments per member: mean = the member's first mode, var = sum of squares of its other modes.
__global__ void __launch_bounds__(256)
    k_chaos_moments(const double* __restrict__ u, const int* __restrict__ off, int n_members, int nt, long long nn,
                    double* __restrict__ mean, double* __restrict__ var) {
    const long long per = (long long)nt * nn;
    const long long total = (long long)n_members * per;
    for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
        const int j = (int)(idx / per);
        const long long r = idx % per;
        const int a0 = off[j], a1 = off[j + 1];
        mean[idx] = u[(long long)a0 * per + r];
        if (var) {
            double q = 0.0;
            for (int a = a0 + 1; a < a1; ++a) {
                const double v = u[(long long)a * per + r];
                q += v * v;
            }
            var[idx] = q;
        }
    }
}

// One workgroup per cell: sum of lam * s over the cell's (component, local node) pairs.
__global__ void __launch_bounds__(256)
    k_cell_dot(int dim, int k, Grid g, int ncomp, const double* __restrict__ lam, const double* __restrict__ s_in,
               double* __restrict__ out) {
    __shared__ double sh[256];
    const int n1l = k + 1;
    const int np = dim == 2 ? n1l * n1l : n1l * n1l * n1l;
    const long long cell = blockIdx.x;
    int cc[3] = {0, 0, 0};
    {
        long long r = cell;
        for (int d = 0; d < dim; ++d) { cc[d] = (int)(r % g.n); r /= g.n; }
    }
    const long long nb1 = (long long)g.n * n1l;
    long long nbn = 1;
    for (int d = 0; d < dim; ++d) nbn *= nb1;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < ncomp * np; idx += 256) {
        const int comp = idx / np, a = idx % np;
        long long node = 0, brk = 0, m = 1, bm = 1;
        for (int d = 0, aa = a; d < dim; ++d, aa /= n1l) {
            const int ad = aa % n1l;
            node += (long long)(cc[d] * k + ad) * m;
            brk += ((long long)cc[d] * n1l + ad) * bm;
            m *= g.n1;
            bm *= nb1;
        }
        acc += lam[comp * g.n_nodes + node] * s_in[comp * nbn + brk];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[cell] = sh[0];
}

__global__ void __launch_bounds__(1024)
    k_form_accumulate(const double* __restrict__ form, long long n, double scale, double* __restrict__ cells,
                      double* __restrict__ total) {
    __shared__ double sh[1024];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += 1024) {
        const double v = scale * form[i];
        if (cells) cells[i] += v;
        acc += v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) total[0] += sh[0];
}

constexpr int kCoarseModes = 2;   // modes per workgroup when every mode uses the same inverse
constexpr int kCoarseWaves = 8;   // waves per workgroup, each summing one range of l

// x[al][dofs[r]] = sum_l AinvT[l][r] b[al][dofs[l]].  A workgroup takes 64 rows r (one per lane) and
// mb modes (kCoarseModes, or 1 when every mode has its own inverse), so one load of the inverse
// serves mb modes; its kCoarseWaves waves take consecutive ranges of l, and the range sums are added
// in wave order.
template <typename T>
__global__ void __launch_bounds__(64 * kCoarseWaves)
    k_coarse_solve(const double* __restrict__ AinvT_all, long long inv_stride, int nint, const int* __restrict__ dofs,
                   int n_xi, int mb, long long mode_len, const T* __restrict__ b, T* __restrict__ x) {
    extern __shared__ unsigned char smem_raw[];
    double* bl = reinterpret_cast<double*>(smem_raw);     // [mb][nint]
    double* part = bl + (size_t)mb * nint;                 // [kCoarseWaves][mb][64]
    const int m0 = blockIdx.y * mb;
    const int nm = min(mb, n_xi - m0);
    for (int i = threadIdx.x; i < mb * nint; i += blockDim.x) {
        const int m = i / nint, l = i - m * nint;
        bl[i] = m < nm ? (double)b[(m0 + m) * mode_len + dofs[l]] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = blockIdx.x * 64 + lane;
    const int rc = min(row, nint - 1);
    const double* A = AinvT_all + (long long)m0 * inv_stride;   // inv_stride 0: one inverse for all modes
    const int range = (nint + kCoarseWaves - 1) / kCoarseWaves;
    const int l0 = wv * range, l1 = min(nint, l0 + range);
    double acc[kCoarseModes];
#pragma unroll
    for (int m = 0; m < kCoarseModes; ++m) acc[m] = 0.0;
#pragma unroll 4
    for (int l = l0; l < l1; ++l) {
        const double a = A[(long long)l * nint + rc];
#pragma unroll
        for (int m = 0; m < kCoarseModes; ++m)
            if (m < mb) acc[m] += a * bl[m * nint + l];
    }
#pragma unroll
    for (int m = 0; m < kCoarseModes; ++m)
        if (m < mb) part[(wv * mb + m) * 64 + lane] = acc[m];
    __syncthreads();
    if (wv == 0 && row < nint) {
        for (int m = 0; m < nm; ++m) {
            double sum = 0.0;
            for (int w = 0; w < kCoarseWaves; ++w) sum += part[(w * mb + m) * 64 + lane];
            x[(m0 + m) * mode_len + dofs[row]] = (T)sum;
        }
    }
}

template <typename T>
__global__ void k_copy(const T* __restrict__ in, T* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = in[i];
}

constexpr int kDotThreads = 256;
constexpr int kG = 8;   // vectors per register group

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// partial[blk][j] = sum over this block's share of V[j][i] w[i], j < k
__global__ void __launch_bounds__(kDotThreads)
    k_multidot(const double* __restrict__ V, long long ldv, int k, const double* __restrict__ w, long long n,
               double* __restrict__ partial) {
    __shared__ double sh[kDotThreads];
    for (int j0 = 0; j0 < k; j0 += kG) {
        double acc[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) acc[u] = 0.0;
        for (long long i = blockIdx.x * (long long)kDotThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kDotThreads) {
            const double wv = w[i];
#pragma unroll
            for (int u = 0; u < kG; ++u)
                if (j0 + u < k) acc[u] += V[(j0 + u) * ldv + i] * wv;
        }
#pragma unroll
        for (int u = 0; u < kG; ++u) {
            if (j0 + u < k) {
                const double s = block_sum(acc[u], sh);
                if (threadIdx.x == 0) partial[(long long)blockIdx.x * k + j0 + u] = s;
            }
        }
    }
}

// wout = w - sum_j h[j] V[j], and by mode:
//   kUpdDotNorm: partial[blk][j] = sum V[j] wout (j < k) and partial[blk][k] = |wout|^2;
//   kUpdNorm:    partial[blk][0] = |wout|^2;
//   kUpdScaled:  wout is divided by hn = sqrt(h[k] - sum_j h[j]^2) (h[k] = |w|^2, V orthonormal: the
//                norm of the updated vector by Pythagoras; 0 where that is not positive), no partials.
template <int KMAX>
__global__ void __launch_bounds__(kDotThreads)
    k_update_dot(const double* __restrict__ V, long long ldv, int k, const double* __restrict__ h,
                 const double* __restrict__ w, double* __restrict__ wout, long long n, double* __restrict__ partial,
                 int mode) {
    __shared__ double sh[kDotThreads];
    double hc[KMAX];
    double acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        hc[j] = j < k ? h[j] : 0.0;
        acc[j] = 0.0;
    }
    double scale = 1.0;
    if (mode == kUpdScaled) {
        double ss = 0.0;
        for (int j = 0; j < k; ++j) ss += h[j] * h[j];
        const double hn2 = h[k] - ss;
        scale = hn2 > 0.0 ? 1.0 / sqrt(hn2) : 0.0;
    }
    double nrm = 0.0;
    for (long long i = blockIdx.x * (long long)kDotThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kDotThreads) {
        double v[KMAX];
        double s = w[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
            v[j] = j < k ? V[j * ldv + i] : 0.0;
            s -= hc[j] * v[j];
        }
        wout[i] = mode == kUpdScaled ? s * scale : s;
        if (mode == kUpdDotNorm) {
#pragma unroll
            for (int j = 0; j < KMAX; ++j) acc[j] += v[j] * s;
        }
        nrm += s * s;
    }
    if (mode == kUpdDotNorm) {
        for (int j = 0; j < k; ++j) {
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < KMAX; ++u) if (u == j) a = acc[u];
            const double sum = block_sum(a, sh);
            if (threadIdx.x == 0) partial[(long long)blockIdx.x * (k + 1) + j] = sum;
        }
        const double sum = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[(long long)blockIdx.x * (k + 1) + k] = sum;
    } else if (mode == kUpdNorm) {
        const double sum = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = sum;
    }
}

__global__ void __launch_bounds__(kDotThreads) k_reduce_partials(const double* __restrict__ partial, int nblk, int k,
                                                                  double* __restrict__ out) {
    __shared__ double sh[kDotThreads];
    for (int j = 0; j < k; ++j) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kDotThreads) a += partial[(long long)b * k + j];
        const double s = block_sum(a, sh);
        if (threadIdx.x == 0) out[j] = s;
    }
}

// x += sum_j y[j] V[j]
template <int KMAX>
__global__ void k_multi_axpy(const double* __restrict__ V, long long ldv, int k, const double* __restrict__ y,
                             double* __restrict__ x, long long n) {
    double yc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) yc[j] = j < k ? y[j] : 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double s = x[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) s += yc[j] * V[j * ldv + i];
        x[i] = s;
    }
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ in, D* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (D)in[i];
}

template <typename T>
__global__ void k_fill(T* __restrict__ out, T v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = v;
}

unsigned grid_for(long long n, int threads, unsigned cap = 8192) {
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

template <typename T>
hipError_t launch_transfer_1d(int dim, int ncomp, const int* in_dims, const int* out_dims, int dir, const int* tidx,
                              const T* tw, int width, const T* in, T* out, bool accumulate, hipStream_t s) {
    long long out_comp = (long long)out_dims[0] * out_dims[1] * (dim == 3 ? out_dims[2] : 1);
    long long in_comp = (long long)in_dims[0] * in_dims[1] * (dim == 3 ? in_dims[2] : 1);
    const long long total = out_comp * ncomp;
    const unsigned grid = grid_for(total, 256, 65536);
    // 32-bit indices when the output loop (with one grid stride of headroom) and the input fit in 2^31
    const bool narrow = total + (long long)grid * 256 < (1LL << 31) && in_comp * ncomp < (1LL << 31);
    const int n_in = in_dims[dir], n_out = out_dims[dir];
    const long long inner = dir == 0 ? 1LL : (dir == 1 ? (long long)in_dims[0] : (long long)in_dims[0] * in_dims[1]);
    const long long ncols = in_comp / n_in * ncomp;
    const size_t lds = (size_t)n_in * 64 * sizeof(T);
    // In 3D the staged form pays where each output has many table terms (the restriction of Q3 and Q4: 11
    // and 13 fine nodes per coarse vertex, about 2 inputs per output) and in the y and z passes of the
    // prolongation (about half an input per output; the last pass also reads the output it adds to);
    // elsewhere (Q1/Q2 restriction, the x pass of the prolongation, whose staged stores are one line
    // per lane, and the 2D passes) the direct form with its higher occupancy was faster on MI355X.
    const bool lds_ok = dim == 3 && narrow && lds <= 64 * 1024 && ncols < (1LL << 31) &&
                        (width == 11 || width == 13 ||
                         (dir >= 1 && n_out > n_in && (width == 2 || width == 3 || width == 4 || width == 5)));
    if (lds_ok) {
        const unsigned blocks = (unsigned)((ncols + 63) / 64);
        const FastDiv fi = make_fastdiv((unsigned)inner);
#define SG_TL(W_)                                                                                                  \
    hipLaunchKernelGGL((k_transfer_1d_lds<T, W_>), dim3(blocks), dim3(256), lds, s, (unsigned)ncols, (unsigned)n_in, \
                       (unsigned)n_out, (unsigned)inner, fi, tidx, tw, in, out, accumulate)
        switch (width) {
            case 2: SG_TL(2); break;
            case 3: SG_TL(3); break;
            case 4: SG_TL(4); break;
            case 5: SG_TL(5); break;
            case 11: SG_TL(11); break;
            default: SG_TL(13); break;
        }
#undef SG_TL
        return hipGetLastError();
    }
    if (narrow) {
        const FastDiv f0 = make_fastdiv((unsigned)out_dims[0]), f1 = make_fastdiv((unsigned)out_dims[1]),
                      f2 = make_fastdiv(dim == 3 ? (unsigned)out_dims[2] : 1u);
#define SG_TR(W_)                                                                                              \
    hipLaunchKernelGGL((k_transfer_1d_narrow<T, W_>), dim3(grid), dim3(256), 0, s, dim, (unsigned)total, in_dims[0], \
                       in_dims[1], f0, f1, f2, dir, tidx, tw, width, in, out, accumulate, (unsigned)in_comp)
        switch (width) {
            case 2: SG_TR(2); break;
            case 3: SG_TR(3); break;
            case 4: SG_TR(4); break;
            case 5: SG_TR(5); break;
            case 6: SG_TR(6); break;
            case 7: SG_TR(7); break;
            case 11: SG_TR(11); break;    // restriction of Q3 (fine nodes per coarse vertex)
            case 13: SG_TR(13); break;    // restriction of Q4
            default: SG_TR(0); break;
        }
#undef SG_TR
    } else
        hipLaunchKernelGGL(k_transfer_1d<T>, dim3(grid), dim3(256), 0, s, dim, total, in_dims[0], in_dims[1],
                           out_dims[0], out_dims[1], dim == 3 ? out_dims[2] : 1, dir, tidx, tw, width, in, out,
                           accumulate, in_comp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_node_gather(GatherOp op, int dim, int k, Grid g, int ncomp, const T* s_in, const T* x, const T* b,
                              T* out, T omega, int sx, int sz, hipStream_t s) {
    if (ncomp > 65535 || g.n_nodes > 0x7fffffffLL || k < 1 || k > 4 || sx < k || sx % k || sz < k || sz % k)
        return hipErrorInvalidConfiguration;
    const unsigned bx = std::min<long long>((g.n_nodes + 255) / 256, 4096);
    const dim3 grid(bx, ncomp), block(256);
    const GatherDivs dv{make_fastdiv((unsigned)g.n1), make_fastdiv((unsigned)sx), make_fastdiv((unsigned)sz)};
#define SG_NG(OP_, D_, K_) \
    hipLaunchKernelGGL((k_node_gather<T, OP_, D_, K_>), grid, block, 0, s, g, s_in, x, b, out, omega, (unsigned)sx, \
                       (unsigned)sz, dv)
#define SG_NG_K(OP_, D_)                          \
    switch (k) {                                  \
        case 1: SG_NG(OP_, D_, 1); break;         \
        case 2: SG_NG(OP_, D_, 2); break;         \
        case 3: SG_NG(OP_, D_, 3); break;         \
        default: SG_NG(OP_, D_, 4); break;        \
    }
    if (dim == 2) {
        if (op == GATHER_SET) { SG_NG_K(GATHER_SET, 2) }
        else if (op == GATHER_RESIDUAL) { SG_NG_K(GATHER_RESIDUAL, 2) }
        else if (op == GATHER_INTERIOR) { SG_NG_K(GATHER_INTERIOR, 2) }
        else { SG_NG_K(GATHER_VANKA, 2) }
    } else {
        if (op == GATHER_SET) { SG_NG_K(GATHER_SET, 3) }
        else if (op == GATHER_RESIDUAL) { SG_NG_K(GATHER_RESIDUAL, 3) }
        else if (op == GATHER_INTERIOR) { SG_NG_K(GATHER_INTERIOR, 3) }
        else { SG_NG_K(GATHER_VANKA, 3) }
    }
#undef SG_NG_K
#undef SG_NG
    return hipGetLastError();
}

hipError_t launch_sample_stats(const double* u, int N, int nt, long long nn, double* mean, double* var, hipStream_t s) {
    const long long total = (long long)nt * nn;
    const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_sample_stats, dim3(blocks), dim3(256), 0, s, u, N, nt, nn, mean, var);
    return hipGetLastError();
}

hipError_t launch_chaos_moments(const double* u, const int* off, int n_members, int nt, long long nn, double* mean,
                                double* var, hipStream_t s) {
    const long long total = (long long)n_members * nt * nn;
    const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_chaos_moments, dim3(blocks), dim3(256), 0, s, u, off, n_members, nt, nn, mean, var);
    return hipGetLastError();
}

hipError_t launch_cell_dot(int dim, int k, Grid g, int ncomp, const double* lam, const double* s_in, double* out,
                           hipStream_t s) {
    if (g.n_cells > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_cell_dot, dim3((unsigned)g.n_cells), dim3(256), 0, s, dim, k, g, ncomp, lam, s_in, out);
    return hipGetLastError();
}

hipError_t launch_form_accumulate(const double* form, long long n, double scale, double* cells, double* total,
                                  hipStream_t s) {
    if (n < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_form_accumulate, dim3(1), dim3(1024), 0, s, form, n, scale, cells, total);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(const double* AinvT, long long inv_stride, int nint, const int* dofs, int n_xi,
                               long long mode_len, const T* b, T* x, hipStream_t s) {
    const long long n = mode_len * n_xi;
    hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, b, x, n);
    // modes per workgroup: kCoarseModes when they share the inverse and the LDS (160 KB) holds them
    int mb = inv_stride ? 1 : kCoarseModes;
    auto lds_of = [&](int m) { return (size_t)m * nint * sizeof(double) + (size_t)kCoarseWaves * m * 64 * sizeof(double); };
    while (mb > 1 && lds_of(mb) > 160 * 1024) --mb;
    const size_t lds = lds_of(mb);
    const int gy = (n_xi + mb - 1) / mb;
    if (nint < 1 || lds > 160 * 1024 || gy > 65535) return hipErrorInvalidConfiguration;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)k_coarse_solve<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3((nint + 63) / 64, gy), dim3(64 * kCoarseWaves), lds, s, AinvT, inv_stride,
                       nint, dofs, n_xi, mb, mode_len, b, x);
    return hipGetLastError();
}

hipError_t launch_multidot(const double* V, long long ldv, int k, const double* w, long long n, double* partial,
                           int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(kDotThreads), 0, s, V, ldv, k, w, n, partial);
    return hipGetLastError();
}

hipError_t launch_update_dot(const double* V, long long ldv, int k, const double* h, const double* w, double* wout,
                             long long n, double* partial, int nblk, int mode, hipStream_t s) {
    if (mode != kUpdDotNorm && mode != kUpdNorm && mode != kUpdScaled) return hipErrorInvalidValue;
#define SG_UD(KM)                                                                                               \
    if (k <= KM) {                                                                                              \
        hipLaunchKernelGGL((k_update_dot<KM>), dim3(nblk), dim3(kDotThreads), 0, s, V, ldv, k, h, w, wout, n, partial, mode); \
        return hipGetLastError();                                                                              \
    }
    SG_UD(8)
    SG_UD(16)
    SG_UD(32)
    SG_UD(65)
#undef SG_UD
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_partials(const double* partial, int nblk, int k, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kDotThreads), 0, s, partial, nblk, k, out);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* V, long long ldv, int k, const double* y, double* x, long long n,
                             hipStream_t s) {
#define SG_MA(KM)                                                                                   \
    if (k <= KM) {                                                                                  \
        hipLaunchKernelGGL((k_multi_axpy<KM>), dim3(grid_for(n, 256)), dim3(256), 0, s, V, ldv, k, y, x, n); \
        return hipGetLastError();                                                                  \
    }
    SG_MA(8)
    SG_MA(16)
    SG_MA(32)
    SG_MA(64)
#undef SG_MA
    return hipErrorInvalidValue;
}

hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* out, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n, 256)), dim3(256), 0, s, a, x, b, y, out, n);
    return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_convert(const S* in, D* out, long long n, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<S, D>), dim3(grid_for(n, 256)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* out, T v, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, out, v, n);
    return hipGetLastError();
}

template hipError_t launch_transfer_1d<double>(int, int, const int*, const int*, int, const int*, const double*, int,
                                               const double*, double*, bool, hipStream_t);
template hipError_t launch_transfer_1d<float>(int, int, const int*, const int*, int, const int*, const float*, int,
                                              const float*, float*, bool, hipStream_t);
template hipError_t launch_node_gather<double>(GatherOp, int, int, Grid, int, const double*, const double*,
                                               const double*, double*, double, int, int, hipStream_t);
template hipError_t launch_node_gather<float>(GatherOp, int, int, Grid, int, const float*, const float*, const float*,
                                              float*, float, int, int, hipStream_t);
template hipError_t launch_coarse_solve<double>(const double*, long long, int, const int*, int, long long,
                                                const double*, double*, hipStream_t);
template hipError_t launch_coarse_solve<float>(const double*, long long, int, const int*, int, long long, const float*,
                                               float*, hipStream_t);
template hipError_t launch_convert<double, float>(const double*, float*, long long, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, long long, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, long long, hipStream_t);
template hipError_t launch_fill<double>(double*, double, long long, hipStream_t);
template hipError_t launch_fill<float>(float*, float, long long, hipStream_t);

}  // namespace sg
