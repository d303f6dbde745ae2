// The coarse segment of the V-cycle in one launch (a persistent kernel): levels l0 .. L-1 of the
// block-Jacobi multigrid cycle (Remark solver-matrix-free-sg: one V-cycle with the space-time Vanka
// smoother per stochastic diagonal block), for every stochastic mode at once.
//
// With the mean-based diagonal block every mode is cycled with the same operator A_0 and nothing
// couples two modes, so one workgroup runs the whole lower part of the cycle for one mode, from the
// right-hand side on level l0 to the correction on level l0, with workgroup barriers between the
// steps and no grid-wide synchronisation: pre-smoothing, residual, restriction down to the coarsest
// level, the dense coarsest solve, then prolongation and post-smoothing back up.  On small levels
// this replaces a dozen small launches per level (and the idle gaps between them) with one.
//
// The steps are the same as the kernel-by-kernel cycle's, written for one mode and a workgroup:
//   * operator A_0 = A_t (x) M_K + B_t (x) K_K per cell from the cell's element matrices (the set-up's
//     element stiffness of the mean coefficient and the element mass), Dirichlet columns dropped,
//     cell-local results summed per node in a fixed order (lower cell first in x, then y, then z);
//   * Vanka: the patch residual of every cell times its stored inverse (fragment layout, one inverse
//     per cell or per position class), then x <- x + omega sum_K c_K / (cells sharing the node);
//     Dirichlet DoFs take b;
//   * transfers: the same banded 1D passes (prolongation P, restriction R = P^T) along each direction;
//   * coarsest level: x = b, then x = A_0^{-1} b on the interior DoFs with FP64 accumulation.
//
// One mode's working set of a small level is a few tens of KB, so the launch places as much of it
// as fits in LDS (patch residuals and corrections first, then the first level's b, x, r, the
// transfer temporaries and the lower levels' vectors); the rest stays in the level buffers and the
// scratch area.  The steps address both through generic pointers.  Loops over a row of an element
// matrix or an inverse keep several independent loads in flight (the latency of one load otherwise
// bounds a workgroup that runs alone on its compute unit).
#include "fastdiv.hpp"
#include "kernels.hpp"

namespace sg {

namespace {

constexpr int kSegThreads = 1024;
constexpr int kSegLds = 160 * 1024 - 256;   // LDS of one compute unit (gfx950) less the time matrices

// divisions by the run-time sizes of the levels as multiply-shift (an integer division would
// otherwise dominate the index arithmetic of these small, latency-bound steps)
struct SegDivs {
    FastDiv npp;
    FastDiv n[kSegMaxLevels], n1[kSegMaxLevels], nn[kSegMaxLevels];
};

__device__ __forceinline__ int qdiv(const FastDiv& f, int x) { return (int)fast_quot(f, (unsigned)x); }

// local node a of cell `cell` on a level with n cells and n1 nodes per direction: global node index
// and whether it is a Dirichlet node (the levels of the segment are small: 32-bit indices)
template <int DIM, int K>
__device__ __forceinline__ int seg_node(const FastDiv& fn, int n1, int cell, int a, bool* bnd) {
    constexpr int N1 = K + 1;
    int node = 0, mul = 1, c = cell;
    bool b = false;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int q = qdiv(fn, c);
        const int cd = c - q * (int)fn.d;
        c = q;
        const int ad = a % N1;
        a /= N1;
        const int id = cd * K + ad;
        b |= (id == 0) | (id == n1 - 1);
        node += id * mul;
        mul *= n1;
    }
    *bnd = b;
    return node;
}

template <int DIM>
__device__ __forceinline__ bool seg_boundary(const FastDiv& fn1, int n1, int node) {
    bool bnd = false;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int q = qdiv(fn1, node);
        const int i = node - q * n1;
        node = q;
        bnd |= (i == 0) | (i == n1 - 1);
    }
    return bnd;
}

// Sum over the cells that contain the interior node `node` of their cell-local values
// vals[cell * stride + off + local index], lower cell first in x, then y, then z; also returns the
// number of cells.  The (up to 2^DIM) loads are issued before the ordered sum.
template <int DIM, int K, typename T>
__device__ __forceinline__ T seg_node_sum(int n, const FastDiv& fn1, int n1, int node, const T* vals, int stride, int off,
                                          int* cnt) {
    constexpr int N1 = K + 1;
    int lo[3] = {0, 0, 0}, la[3] = {0, 0, 0}, two[3] = {0, 0, 0};
    int r = node;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int q = qdiv(fn1, r);
        const int i = r - q * n1;
        r = q;
        if (i % K == 0) {              // interior node on a cell face: the lower and the upper cell
            lo[d] = i / K - 1;
            la[d] = K;
            two[d] = 1;
        } else {
            lo[d] = i / K;
            la[d] = i - lo[d] * K;
        }
    }
    constexpr int NC = 1 << DIM;
    T v[NC];
    bool on[NC];
    int first = 0;
    // every candidate is loaded (the absent ones from the first cell's entry) before the ordered sum
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int x = q & 1, y = (q >> 1) & 1, z = DIM == 3 ? (q >> 2) & 1 : 0;
        on[q] = x <= two[0] && y <= two[1] && (DIM == 2 || z <= two[2]);
        const int c0 = lo[0] + x, c1 = lo[1] + y, c2 = DIM == 3 ? lo[2] + z : 0;
        const int a0 = x ? 0 : la[0], a1 = y ? 0 : la[1], a2 = DIM == 3 ? (z ? 0 : la[2]) : 0;
        const int cell = (c2 * n + c1) * n + c0;
        const int a = (a2 * N1 + a1) * N1 + a0;
        const int addr = cell * stride + off + a;
        if (q == 0) first = addr;
        v[q] = vals[on[q] ? addr : first];
    }
    T sum = T(0);
    int count = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q)
        if (on[q]) {
            sum += v[q];
            ++count;
        }
    *cnt = count;
    return sum;
}

struct SegView {
    int nt, npp;
    int n, n1, nn, cells;
    FastDiv fnpp, fn, fn1, fnn;
    int classes;
    const double* E;       // element stiffness: [n_cells][np][np], or one cell's [np][np] (e_cellwise = 0)
    int e_cellwise;
    const double* Me;
    const void* inv;
    const double* At;
    const double* Bt;
};

// the rows of the cell-local products for NT time basis functions (straight-line loads)
template <int DIM, int K, int NT, typename T>
__device__ __forceinline__ void seg_cell_rows(const SegView& v, T* Y, const T* Xc) {
    constexpr int NP = ipow(K + 1, DIM);
    constexpr int NPP = NT * NP;
    const int total = v.cells * NPP;
    for (int idx = threadIdx.x; idx < total; idx += kSegThreads) {
        const int cell = qdiv(v.fnpp, idx), row = idx - cell * NPP;
        const int ti = row / NP, a = row - ti * NP;
        const double* E = v.E + ((v.e_cellwise ? (long long)cell * NP : 0) + a) * NP;
        const double* Me = v.Me + a * NP;
        const T* xc = Xc + cell * NPP;
        double m[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) m[j] = 0.0;
        double s = 0.0;
#pragma unroll NT > 2 ? 3 : 9
        for (int b = 0; b < NP; ++b) {
            const double me = Me[b];
#pragma unroll
            for (int j = 0; j < NT; ++j) m[j] += me * (double)xc[j * NP + b];
            s += E[b] * (double)xc[ti * NP + b];
        }
        double acc = v.Bt[ti] * s;
#pragma unroll
        for (int j = 0; j < NT; ++j) acc += v.At[ti * NT + j] * m[j];
        Y[idx] = (T)acc;
    }
}

// y_K = A_0 restricted to cell K applied to x (Dirichlet columns dropped), for every cell: Y[cell][npp].
// The cell's values are gathered first (Xc[cell][j][b], 0 on Dirichlet nodes), then
// y[ti][a] = sum_j At[ti][j] (Me x_j)[a] + Bt[ti] (E_K x_ti)[a].
template <int DIM, int K, typename T>
__device__ void seg_cell_apply(const SegView& v, const T* x, T* Y, T* Xc) {
    constexpr int NP = ipow(K + 1, DIM);
    const int nt = v.nt, npp = v.npp;
    const int total = v.cells * npp;
    for (int idx = threadIdx.x; idx < total; idx += kSegThreads) {
        const int cell = qdiv(v.fnpp, idx), row = idx - cell * npp;
        const int j = row / NP, b = row - j * NP;
        bool bnd;
        const int node = seg_node<DIM, K>(v.fn, v.n1, cell, b, &bnd);
        const T xv = x[j * v.nn + node];      // a valid node either way: load, then select
        Xc[idx] = bnd ? T(0) : xv;
    }
    __syncthreads();
    switch (nt) {
    case 1: seg_cell_rows<DIM, K, 1, T>(v, Y, Xc); break;
    case 2: seg_cell_rows<DIM, K, 2, T>(v, Y, Xc); break;
    case 3: seg_cell_rows<DIM, K, 3, T>(v, Y, Xc); break;
    default: seg_cell_rows<DIM, K, 4, T>(v, Y, Xc); break;
    }
    __syncthreads();
}

// r = b - A_0 x (Dirichlet rows: b - x)
template <int DIM, int K, typename T>
__device__ void seg_residual(const SegView& v, const T* x, const T* b, T* r, T* Y, T* Xc) {
    constexpr int NP = ipow(K + 1, DIM);
    seg_cell_apply<DIM, K, T>(v, x, Y, Xc);
    for (int idx = threadIdx.x; idx < v.nn * v.nt; idx += kSegThreads) {
        const int ti = qdiv(v.fnn, idx), node = idx - ti * v.nn;
        if (seg_boundary<DIM>(v.fn1, v.n1, node)) {
            r[idx] = b[idx] - x[idx];
        } else {
            int cnt;
            r[idx] = b[idx] - seg_node_sum<DIM, K, T>(v.n, v.fn1, v.n1, node, Y, v.npp, ti * NP, &cnt);
        }
    }
    __syncthreads();
}

// one additive Vanka sweep: x <- x + omega sum_K R_K^T W_K A_K^{-1} R_K (b - A_0 x); with x_zero the
// residual is b itself.  G, C: [n_cells][npp] (patch residuals, corrections).
template <int DIM, int K, typename T>
__device__ void seg_vanka(const SegView& v, const T* b, T* x, T* r, T* G, T* C, double omega, bool x_zero) {
    constexpr int NP = ipow(K + 1, DIM);
    const int npp = v.npp;
    const T* rs = b;
    if (!x_zero) {
        seg_residual<DIM, K, T>(v, x, b, r, C, G);
        rs = r;
    }
    const int total = v.cells * npp;
    // patch residuals (Dirichlet rows 0)
    for (int idx = threadIdx.x; idx < total; idx += kSegThreads) {
        const int cell = qdiv(v.fnpp, idx), row = idx - cell * npp;
        const int j = row / NP;
        bool bnd;
        const int node = seg_node<DIM, K>(v.fn, v.n1, cell, row - j * NP, &bnd);
        const T rv = rs[j * v.nn + node];
        G[idx] = bnd ? T(0) : rv;
    }
    __syncthreads();
    // corrections c_K = A_K^{-1} R_K r; the inverse holds B[c][I] = A^{-1}[I][c] in the fragment layout
    const T* inv = static_cast<const T*>(v.inv);
    const int spl = vanka_spl(npp, sizeof(T));
    const long long istride = vanka_inv_stride(npp);
    for (int idx = threadIdx.x; idx < total; idx += kSegThreads) {
        const int cell = qdiv(v.fnpp, idx), I = idx - cell * npp;
        int cc[3] = {0, 0, 0};
        {
            int q = cell;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const int qq = qdiv(v.fn, q);
                cc[d] = q - qq * v.n;
                q = qq;
            }
        }
        const T* Ai = inv + inverse_slot<DIM>(cell, cc, v.n, v.classes) * istride;
        const T* g = G + cell * npp;
        T acc[4] = {T(0), T(0), T(0), T(0)};
        int c = 0;
        for (; c + 4 <= npp; c += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += Ai[vanka_inv_offset(npp, spl, c + u, I)] * g[c + u];
        }
        for (; c < npp; ++c) acc[0] += Ai[vanka_inv_offset(npp, spl, c, I)] * g[c];
        C[idx] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    __syncthreads();
    // x <- x + omega sum / cells sharing the node; Dirichlet: x = b
    for (int idx = threadIdx.x; idx < v.nn * v.nt; idx += kSegThreads) {
        const int ti = qdiv(v.fnn, idx), node = idx - ti * v.nn;
        if (seg_boundary<DIM>(v.fn1, v.n1, node)) {
            x[idx] = b[idx];
        } else {
            int cnt;
            const T s = seg_node_sum<DIM, K, T>(v.n, v.fn1, v.n1, node, C, npp, ti * NP, &cnt);
            // 1 / cnt for the 1, 2, 4 or 8 cells sharing a node: exact, so the product equals the quotient
            const T rc = cnt == 1 ? T(1) : (cnt == 2 ? T(0.5) : (cnt == 4 ? T(0.25) : T(0.125)));
            x[idx] = x[idx] + (T)omega * s * rc;
        }
    }
    __syncthreads();
}

// One banded 1D pass along `dir` for nc components of a transfer between n_src and n_dst nodes per
// direction (directions before `dir` already at n_dst):
//     out[c][.., o, ..] (+)= sum_w tw[o w_] in[c][.., tidx[o w_], ..]
template <int DIM, typename T>
__device__ void seg_pass(int nc, int n_src, int n_dst, const FastDiv& f_src, const FastDiv& f_dst, int dir,
                         const int* tidx, const T* tw, int width, const T* in, T* out, bool accumulate) {
    const int i0 = dir > 0 ? n_dst : n_src, i1 = dir > 1 ? n_dst : n_src, i2 = DIM == 3 ? n_src : 1;
    const int o0 = n_dst;                             // direction 0 is at n_dst after any pass
    const int o1 = 1 <= dir ? n_dst : n_src;
    const int o2 = DIM == 3 ? (2 <= dir ? n_dst : n_src) : 1;
    const FastDiv& f0 = f_dst;
    const FastDiv& f1 = 1 <= dir ? f_dst : f_src;
    const FastDiv& f2 = 2 <= dir ? f_dst : f_src;
    const int in_comp = i0 * i1 * i2;
    const int total = nc * o0 * o1 * o2;
    const int istr = dir == 0 ? 1 : (dir == 1 ? i0 : i0 * i1);
    for (int idx = threadIdx.x; idx < total; idx += kSegThreads) {
        int r = idx;
        int q = qdiv(f0, r);
        const int x0 = r - q * o0;
        r = q;
        q = qdiv(f1, r);
        const int x1 = r - q * o1;
        r = q;
        int x2 = 0;
        if (DIM == 3) {
            q = qdiv(f2, r);
            x2 = r - q * o2;
            r = q;
        }
        const int c = r;
        const int o = dir == 0 ? x0 : (dir == 1 ? x1 : x2);
        const int base = c * in_comp + ((dir == 2 ? 0 : x2) * i1 + (dir == 1 ? 0 : x1)) * i0 + (dir == 0 ? 0 : x0);
        // every table entry holds a valid index: the loads are unconditional, the zero weights skipped
        T acc = T(0);
#pragma unroll 4
        for (int w = 0; w < width; ++w) {
            const T wt = tw[o * width + w];
            const T iv = in[base + tidx[o * width + w] * istr];
            acc = wt != T(0) ? acc + wt * iv : acc;
        }
        if (accumulate) out[idx] += acc;
        else out[idx] = acc;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void seg_copy(const T* src, T* dst, int n) {
    for (int i = threadIdx.x; i < n; i += kSegThreads) dst[i] = src[i];
    __syncthreads();
}

template <typename T, int DIM, int K>
__global__ void __launch_bounds__(kSegThreads) k_vcycle_segment(SegArgs a, SegDivs dv) {
    extern __shared__ __align__(16) unsigned char seg_lds[];
    // the time matrices, read with per-lane indices: from LDS, not from the argument segment
    __shared__ double s_At[kMaxNT * kMaxNT], s_Bt[kMaxNT];
    if (threadIdx.x < kMaxNT * kMaxNT) s_At[threadIdx.x] = a.At[threadIdx.x];
    if (threadIdx.x < kMaxNT) s_Bt[threadIdx.x] = a.Bt[threadIdx.x];
    const int al = blockIdx.x;
    const int nt = a.nt;
    T* scr = static_cast<T*>(a.scratch) + (long long)al * a.scratch_per_mode;
    // scratch of this mode: G, C [n_cells(l0)][npp] and two transfer temporaries
    const long long cells0 = a.lv[0].g.n_cells * (long long)(nt * a.np);
    auto place = [&](int off, T* global) -> T* { return off >= 0 ? reinterpret_cast<T*>(seg_lds + off) : global; };
    T* G = place(a.lds_G, scr);
    T* C = place(a.lds_C, scr + cells0);
    T* t0 = place(a.lds_t0, scr + 2 * cells0);
    T* t1 = place(a.lds_t1, scr + 2 * cells0 + a.tmp_len);
    auto mode_vec = [&](void* p, int l) -> T* { return static_cast<T*>(p) + (long long)al * nt * a.lv[l].g.n_nodes; };
    auto Xl = [&](int l) -> T* { return place(a.lv[l].lds_x, mode_vec(a.lv[l].x, l)); };
    auto Bl = [&](int l) -> T* { return place(a.lv[l].lds_b, mode_vec(a.lv[l].b, l)); };
    auto Rl = [&](int l) -> T* { return place(a.lv[l].lds_r, mode_vec(a.lv[l].r, l)); };
    const int L = a.nlev;
    constexpr int NP = ipow(K + 1, DIM);
    const int npp = nt * NP;
    // the view of level l (element matrices and inverses from LDS where staged)
    auto view = [&](int l) -> SegView {
        const SegLevelArgs& q = a.lv[l];
        SegView v;
        v.nt = nt;
        v.npp = npp;
        v.n = q.g.n;
        v.n1 = q.g.n1;
        v.nn = (int)q.g.n_nodes;
        v.cells = (int)q.g.n_cells;
        v.fnpp = dv.npp;
        v.fn = dv.n[l];
        v.fn1 = dv.n1[l];
        v.fnn = dv.nn[l];
        v.classes = q.classes;
        v.At = s_At;
        v.Bt = s_Bt;
        v.E = q.lds_E >= 0 ? reinterpret_cast<const double*>(seg_lds + q.lds_E) : q.E;
        v.e_cellwise = q.lds_E >= 0 ? 0 : 1;
        v.Me = q.lds_Me >= 0 ? reinterpret_cast<const double*>(seg_lds + q.lds_Me) : q.Me;
        v.inv = q.lds_inv >= 0 ? static_cast<const void*>(seg_lds + q.lds_inv) : q.inv;
        return v;
    };
    for (int l = 0; l < L; ++l) {
        const SegLevelArgs& q = a.lv[l];
        if (q.lds_E >= 0)
            for (int i = threadIdx.x; i < NP * NP; i += kSegThreads)
                reinterpret_cast<double*>(seg_lds + q.lds_E)[i] = q.E[i];
        if (q.lds_Me >= 0)
            for (int i = threadIdx.x; i < NP * NP; i += kSegThreads)
                reinterpret_cast<double*>(seg_lds + q.lds_Me)[i] = q.Me[i];
        if (q.lds_inv >= 0) {
            const int len = (int)(ipow(3, DIM) * vanka_inv_stride(npp));
            for (int i = threadIdx.x; i < len; i += kSegThreads)
                reinterpret_cast<T*>(seg_lds + q.lds_inv)[i] = static_cast<const T*>(q.inv)[i];
        }
    }
    if (a.lv[0].lds_b >= 0) {
        T* b0 = Bl(0);
        const T* src = mode_vec(a.lv[0].b, 0);
        for (int i = threadIdx.x; i < nt * (int)a.lv[0].g.n_nodes; i += kSegThreads) b0[i] = src[i];
    }
    __syncthreads();
    // descend: x = 0, pre-smoothing, residual, restriction
    for (int l = 0; l < L - 1; ++l) {
        const SegView v = view(l);
        T* x = Xl(l);
        T* b = Bl(l);
        T* r = Rl(l);
        for (int i = threadIdx.x; i < nt * v.nn; i += kSegThreads) x[i] = T(0);
        __syncthreads();
        for (int s = 0; s < a.pre; ++s) seg_vanka<DIM, K, T>(v, b, x, r, G, C, a.omega, s == 0);
        seg_residual<DIM, K, T>(v, x, b, r, C, G);
        // b_{l+1} = R r along every direction (temporaries t0 / t1, the last pass into b_{l+1})
        const T* in = r;
        for (int dir = 0; dir < DIM; ++dir) {
            T* o = dir == DIM - 1 ? Bl(l + 1) : (dir % 2 ? t1 : t0);
            seg_pass<DIM, T>(nt, v.n1, a.lv[l + 1].g.n1, dv.n1[l], dv.n1[l + 1], dir, a.lv[l].r_idx,
                             static_cast<const T*>(a.lv[l].r_w), a.lv[l].wr, in, o, false);
            in = o;
        }
    }
    // coarsest level: x = b, then x = A_0^{-1} b on the interior DoFs (FP64 accumulation).  b on the
    // interior DoFs is staged in G; with coarse_split > 1 the rows' partial sums over consecutive
    // column ranges go to C (as doubles) and are added in range order.
    {
        const int l = L - 1;
        const int nn = (int)a.lv[l].g.n_nodes;
        const T* b = Bl(l);
        T* x = Xl(l);
        const int nint = a.nint;
        T* bl = G;
        for (int i = threadIdx.x; i < nt * nn; i += kSegThreads) x[i] = b[i];
        for (int i = threadIdx.x; i < nint; i += kSegThreads) bl[i] = b[a.coarse_dofs[i]];
        __syncthreads();
        const double* inv = a.coarse_invT;
        const int S = a.coarse_split;
        const int chunk = (nint + S - 1) / S;
        double* part = reinterpret_cast<double*>(C);
        if (nint % 2 == 0) {
            // two consecutive rows per thread, one 16-byte load per column
            const int np2 = nint / 2;
            for (int item = threadIdx.x; item < np2 * S; item += kSegThreads) {
                const int s = item / np2, row = 2 * (item - s * np2);
                const int c0 = s * chunk, c1 = min(nint, c0 + chunk);
                double2 acc[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = make_double2(0.0, 0.0);
                int c = c0;
                for (; c + 8 <= c1; c += 8) {
                    double2 col[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        col[u] = *reinterpret_cast<const double2*>(inv + (long long)(c + u) * nint + row);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const double bv = (double)bl[c + u];
                        acc[u & 3].x += col[u].x * bv;
                        acc[u & 3].y += col[u].y * bv;
                    }
                }
                for (; c < c1; ++c) {
                    const double2 col = *reinterpret_cast<const double2*>(inv + (long long)c * nint + row);
                    const double bv = (double)bl[c];
                    acc[0].x += col.x * bv;
                    acc[0].y += col.y * bv;
                }
                const double s0 = (acc[0].x + acc[1].x) + (acc[2].x + acc[3].x);
                const double s1 = (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y);
                if (S == 1) {
                    x[a.coarse_dofs[row]] = (T)s0;
                    x[a.coarse_dofs[row + 1]] = (T)s1;
                } else {
                    part[s * nint + row] = s0;
                    part[s * nint + row + 1] = s1;
                }
            }
        } else {
            for (int item = threadIdx.x; item < nint * S; item += kSegThreads) {
                const int s = item / nint, row = item - s * nint;
                const int c0 = s * chunk, c1 = min(nint, c0 + chunk);
                double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                int c = c0;
                for (; c + 8 <= c1; c += 8) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[u] += inv[(long long)(c + u) * nint + row] * (double)bl[c + u];
                }
                for (; c < c1; ++c) acc[0] += inv[(long long)c * nint + row] * (double)bl[c];
                const double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
                if (S == 1) x[a.coarse_dofs[row]] = (T)sum;
                else part[s * nint + row] = sum;
            }
        }
        __syncthreads();
        if (S > 1) {
            for (int row = threadIdx.x; row < nint; row += kSegThreads) {
                double sum = 0.0;
                for (int s = 0; s < S; ++s) sum += part[s * nint + row];
                x[a.coarse_dofs[row]] = (T)sum;
            }
            __syncthreads();
        }
    }
    // ascend: x_l += P x_{l+1}, post-smoothing
    for (int l = L - 2; l >= 0; --l) {
        const SegView v = view(l);
        T* x = Xl(l);
        const T* in = Xl(l + 1);
        for (int dir = 0; dir < DIM; ++dir) {
            const bool last = dir == DIM - 1;
            T* o = last ? x : (dir % 2 ? t1 : t0);
            seg_pass<DIM, T>(nt, a.lv[l + 1].g.n1, v.n1, dv.n1[l + 1], dv.n1[l], dir, a.lv[l].p_idx,
                             static_cast<const T*>(a.lv[l].p_w), a.lv[l].wp, in, o, last);
            in = o;
        }
        for (int s = 0; s < a.post; ++s) seg_vanka<DIM, K, T>(v, Bl(l), x, Rl(l), G, C, a.omega, false);
    }
    if (a.lv[0].lds_x >= 0) seg_copy<T>(Xl(0), mode_vec(a.lv[0].x, 0), nt * (int)a.lv[0].g.n_nodes);
}

// LDS placement of one mode's working set: patch residuals and corrections, the first level's b,
// x, r, its element matrices (E only where one cell's stands for all: position classes) and class
// inverses, the transfer temporaries, then the lower levels' b, x, r, each where it still fits.
template <typename T>
void plan_lds(SegArgs& a) {
    const int npp = a.nt * a.np;
    const long long cells0 = a.lv[0].g.n_cells * (long long)npp;
    int used = 0;
    auto place = [&](long long count, int elem) -> int {
        const long long bytes = (count * elem + 15) / 16 * 16;
        if (used + bytes > kSegLds) return -1;
        const int off = used;
        used += (int)bytes;
        return off;
    };
    const int te = (int)sizeof(T);
    for (int l = 0; l < a.nlev; ++l) a.lv[l].lds_b = a.lv[l].lds_x = a.lv[l].lds_r = a.lv[l].lds_E = a.lv[l].lds_Me =
        a.lv[l].lds_inv = -1;
    a.lds_G = place(cells0, te);
    a.lds_C = place(cells0, te);
    const long long len0 = a.nt * a.lv[0].g.n_nodes;
    a.lv[0].lds_b = place(len0, te);
    a.lv[0].lds_x = place(len0, te);
    a.lv[0].lds_r = place(len0, te);
    a.lv[0].lds_Me = place((long long)a.np * a.np, 8);
    if (a.lv[0].classes) {
        a.lv[0].lds_E = place((long long)a.np * a.np, 8);
        a.lv[0].lds_inv = place(ipow(3, a.dim) * vanka_inv_stride(npp), te);
    }
    a.lds_t0 = place(a.tmp_len, te);
    a.lds_t1 = a.dim == 3 ? place(a.tmp_len, te) : -1;
    for (int l = 1; l < a.nlev; ++l) {
        const long long len = a.nt * a.lv[l].g.n_nodes;
        a.lv[l].lds_b = place(len, te);
        a.lv[l].lds_x = place(len, te);
        a.lv[l].lds_r = l + 1 < a.nlev ? place(len, te) : -1;
    }
    a.lds_bytes = used;
    // partial sums of the coarsest rows over column ranges: as many ranges as the threads (two rows
    // each for an even row count) allow and C holds
    const long long units = a.nint % 2 == 0 ? a.nint / 2 : a.nint;
    int S = 1;
    while (S < 8 && units * (S + 1) <= kSegThreads &&
           (long long)a.nint * (S + 1) * (long long)sizeof(double) <= cells0 * te)
        ++S;
    a.coarse_split = S;
}

template <typename T, int DIM, int K>
hipError_t launch_dk(const SegArgs& a, hipStream_t s) {
    SegDivs dv{};
    dv.npp = make_fastdiv((unsigned)(a.nt * a.np));
    for (int l = 0; l < a.nlev; ++l) {
        dv.n[l] = make_fastdiv((unsigned)a.lv[l].g.n);
        dv.n1[l] = make_fastdiv((unsigned)a.lv[l].g.n1);
        dv.nn[l] = make_fastdiv((unsigned)a.lv[l].g.n_nodes);
    }
    if (a.lds_bytes > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)k_vcycle_segment<T, DIM, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  a.lds_bytes);
    hipLaunchKernelGGL((k_vcycle_segment<T, DIM, K>), dim3((unsigned)a.n_xi), dim3(kSegThreads), a.lds_bytes, s, a, dv);
    return hipGetLastError();
}

}  // namespace

long long segment_scratch_per_mode(int nt, int np, long long cells0, long long tmp_len) {
    return 2 * cells0 * nt * np + 2 * tmp_len;
}

template <typename T>
hipError_t launch_vcycle_segment(const SegArgs& args, hipStream_t s) {
    if (args.nlev < 2 || args.nlev > kSegMaxLevels || args.n_xi < 1 || args.n_xi > 65535 || args.nint < 1 ||
        args.nt < 1 || args.nt > kMaxNT || args.np != ipow(args.k + 1, args.dim))
        return hipErrorInvalidValue;
    // 32-bit indices inside a mode
    if (args.lv[0].g.n_cells * (long long)(args.nt * args.np) >= (1LL << 30)) return hipErrorInvalidValue;
    SegArgs a = args;
    plan_lds<T>(a);
    switch (a.dim * 10 + a.k) {
    case 21: return launch_dk<T, 2, 1>(a, s);
    case 22: return launch_dk<T, 2, 2>(a, s);
    case 23: return launch_dk<T, 2, 3>(a, s);
    case 24: return launch_dk<T, 2, 4>(a, s);
    case 31: return launch_dk<T, 3, 1>(a, s);
    case 32: return launch_dk<T, 3, 2>(a, s);
    case 33: return launch_dk<T, 3, 3>(a, s);
    case 34: return launch_dk<T, 3, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_vcycle_segment<double>(const SegArgs&, hipStream_t);
template hipError_t launch_vcycle_segment<float>(const SegArgs&, hipStream_t);

}  // namespace sg
