// Matrix-free application of the stochastic-Galerkin space-time slab operator
//     AA = I_xi (x) A_t (x) M_x + sum_mu G_mu (x) B_t (x) K_mu      (eq. local_rhs_tensor)
// on a uniform Cartesian Q_k mesh, by sum factorisation (Remark solver-matrix-free-sg: only the
// action of AA is formed).
//
// Work decomposition (gfx950, wave64):
//   * one launch over every cell; one workgroup = a segment of `cpb` consecutive cells of one cell
//     row (along x) x all N_xi * N_t components; one thread owns one (cell, component) pair and
//     keeps its (k+1)^d point values in registers; each XCD walks its own contiguous range of rows,
//     in chunks of a few y-rows with z running (tiled_row), so rows in flight share node planes in
//     its L2;
//   * per thread: gather the cell's nodal values (Dirichlet columns dropped), interpolate to the
//     Gauss points (d 1D sweeps with the GLL-basis table), take reference derivatives by Gauss
//     collocation (d sweeps), and integrate back with the transposed sweeps;
//   * the two couplings that cross components go through LDS:
//       - time: the mass term needs sum_j A_t[i][j] u_j at each point,
//       - chaos: the stiffness flux of mode alpha is sum_mu a_mu(x_q) sum_beta [G_mu]_{alpha beta}
//         grad u_beta, read from the neighbours listed in the coupling CSR
//     (with the mean coefficient alone the chaos coupling is the identity and stays in registers);
//   * no scatter: each cell writes its local result to a "broken" node array (every cell owns its
//     (k+1)^d nodes, shared nodes are duplicated); k_node_gather then sums the copies of each node
//     in a fixed order, so the result is deterministic and no atomics or colouring are needed.
#pragma once

#include <algorithm>
#include <mutex>
#include <vector>

#include "fastdiv.hpp"
#include "kernels.hpp"

namespace sg {

namespace {

template <typename T>
struct ApplyArgs {
    const T* x;
    T* s;                 // broken-layout output [comp][b_z][b_y][b_x], b = c (k+1) + a
    const T* coef;
    long long coef_mode_stride;
    const int* cptr;
    const int* cbeta;
    const int* cmu;
    const T* cw;
    int n_xi, n_mu;
    int n_ent;            // coupling entries (length of cbeta / cw / cmu)
    Grid g;
    int cpb;
    int nblocks;
    int mu0;              // position of mu = 0 in the coefficient list
    int mum[8];           // position of mu = e_m (m = 1..M) in the coefficient list, -1 if absent
    int merge;            // 1: sum the x faces shared by the workgroup's cells before storing
    int ss;               // slot stride of the exchange rows (>= N_xi N_t row_stride((k+1)^d))
    // quotients by the launch's run-time sizes as multiply-shift (set with cpb): cells per workgroup,
    // segments per cell row, cells per direction, cells of a row chunk of the traversal, coefficient
    // modes; segs and the log2 of the chunk's rows
    FastDiv fcpb, fsegs, fn, ftyn, fnmu;
    int segs, tylg;
};

// Sets the multiply-shift quotients of a launch with `cpb` cells per workgroup.
template <typename T>
inline void set_apply_divisors(ApplyArgs<T>& a, int cpb) {
    const int n = a.g.n;
    const int ty = row_tile(n);
    a.segs = (n + cpb - 1) / cpb;
    a.tylg = ty == 4 ? 2 : (ty == 2 ? 1 : 0);
    a.fcpb = make_fastdiv((unsigned)cpb);
    a.fsegs = make_fastdiv((unsigned)a.segs);
    a.fn = make_fastdiv((unsigned)n);
    a.ftyn = make_fastdiv((unsigned)(ty * n));
    a.fnmu = make_fastdiv((unsigned)a.n_mu);
}

__device__ __forceinline__ int apply_quot(const FastDiv& f, int x) { return (int)fast_quot(f, (unsigned)x); }

// Stride of one component's row of point values in the exchange rows: odd, so the rows of consecutive
// components start on different banks (a power-of-two point count, as 64 for Q3 cells, would put every
// component of a wave instruction on the same bank).
__host__ __device__ constexpr int row_stride(int np) { return np % 2 ? np : np + 1; }

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

// In-place variant: one line of N1 values is staged in registers at a time.
template <int DIM, int N1, int DIR, bool TR, typename T>
__device__ __forceinline__ void sweep_ip(T (&v)[ipow(N1, DIM)], const T* __restrict__ M) {
    constexpr int NP = ipow(N1, DIM);
    constexpr int st = ipow(N1, DIR);
#pragma unroll
    for (int base = 0; base < NP; ++base) {
        if ((base / st) % N1 != 0) continue;
        T tmp[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) tmp[i] = v[base + i * st];
#pragma unroll
        for (int o = 0; o < N1; ++o) {
            T acc = T(0);
#pragma unroll
            for (int i = 0; i < N1; ++i) acc += (TR ? M[i * N1 + o] : M[o * N1 + i]) * tmp[i];
            v[base + o * st] = acc;
        }
    }
}

template <int DIM, int N1, bool TR, typename T>
__device__ __forceinline__ void sweeps_ip(T (&v)[ipow(N1, DIM)], const T* __restrict__ M) {
    sweep_ip<DIM, N1, 0, TR>(v, M);
    sweep_ip<DIM, N1, 1, TR>(v, M);
    if constexpr (DIM == 3) sweep_ip<DIM, N1, 2, TR>(v, M);
}

// Keeps the scheduler from hoisting every unrolled load of a long loop ahead of its uses, which
// would otherwise blow the register budget and spill.
#define SG_FENCE() __builtin_amdgcn_sched_barrier(0)

template <int NT, typename T>
__device__ __forceinline__ T bt_of(const Tables<T>& tb, int ti) {
    T v = tb.Bt[0];
#pragma unroll
    for (int i = 1; i < NT; ++i) v = (ti == i) ? tb.Bt[i] : v;
    return v;
}

// Store the (k+1)^d results of one (cell, component) into the broken layout.
template <int DIM, int K, typename T>
__device__ __forceinline__ void store_broken(T* __restrict__ s, const T (&Y)[ipow(K + 1, DIM)], T scale,
                                             const int* cc, int n, int comp) {
    constexpr int N1 = K + 1;
    const long long nb1 = (long long)n * N1;
    long long base = comp;
#pragma unroll
    for (int d = DIM - 1; d >= 0; --d) base = base * nb1 + (long long)cc[d] * N1;
#pragma unroll
    for (int p = 0; p < ipow(N1, DIM); ++p) {
        long long off = 0, mul = 1;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            off += ((p / ipow(N1, d)) % N1) * mul;
            mul *= nb1;
        }
        s[base + off] = Y[p] * scale;
    }
}

// Store into the x-merged layout: along x the broken index is seg (cpb k + 1) + (local x node of the
// segment), n k + segs entries in all (no more than the n (k + 1) of the per-cell layout), so the faces
// shared by the cells of one segment appear once; y and z as in store_broken.
// write_face: this cell also stores its x = k face (the last cell of the segment).
template <int DIM, int K, typename T>
__device__ __forceinline__ void store_merged(T* __restrict__ s, const T (&Y)[ipow(K + 1, DIM)], const int* cc, int n,
                                             int comp, int seg, int segs, int cpb, int slot, bool write_face) {
    constexpr int N1 = K + 1;
    const long long nb1 = (long long)n * N1;
    const long long sw = (long long)cpb * K + 1;       // broken x entries of a full segment
    const long long nbx = (long long)n * K + segs;     // all x entries (the last segment may be shorter)
    long long base = comp;
#pragma unroll
    for (int d = DIM - 1; d >= 1; --d) base = base * nb1 + (long long)cc[d] * N1;
    base = base * nbx + seg * sw + (long long)slot * K;
#pragma unroll
    for (int p = 0; p < ipow(N1, DIM); ++p) {
        const int ax = p % N1;
        if (ax == K && !write_face) continue;
        long long off = ax, mul = nbx;
#pragma unroll
        for (int d = 1; d < DIM; ++d) {
            off += ((p / ipow(N1, d)) % N1) * mul;
            mul *= nb1;
        }
        s[base + off] = Y[p];
    }
}

// ---- compile-time chaos structure for affine coefficients ------------------------------------------
// Total-degree index set Lambda_p in graded, lexicographically descending order, and for every
// alpha the positions of alpha - e_m and alpha + e_m (or -1).  For mu = e_m the Galerkin tensor is
// [G_{e_m}]_{alpha beta} = sqrt(max(alpha_m, beta_m)) when beta = alpha +- e_m, zero otherwise.
constexpr int binom_c(int n, int k) {
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int)r;
}

template <int M, int P>
struct ChaosTab {
    static constexpr int N = binom_c(M + P, P);
    int idx[N][M];
    int nbm[N][M];
    int nbp[N][M];
    constexpr ChaosTab() : idx{}, nbm{}, nbp{} {
        int pos = 0;
        for (int deg = 0; deg <= P; ++deg) {
            int a[M] = {};
            a[0] = deg;
            while (true) {
                for (int m = 0; m < M; ++m) idx[pos][m] = a[m];
                ++pos;
                int j = -1;
                for (int m = M - 2; m >= 0; --m)
                    if (a[m] > 0) { j = m; break; }
                if (j < 0) break;
                int tail = 0;
                for (int m = j + 1; m < M; ++m) { tail += a[m]; a[m] = 0; }
                a[j] -= 1;
                a[j + 1] = tail + 1;
            }
        }
        for (int al = 0; al < N; ++al)
            for (int m = 0; m < M; ++m) {
                nbm[al][m] = -1;
                nbp[al][m] = -1;
                for (int be = 0; be < N; ++be) {
                    bool minus = true, plus = true;
                    for (int k = 0; k < M; ++k) {
                        const int dm = idx[al][k] - (k == m ? 1 : 0);
                        const int dp = idx[al][k] + (k == m ? 1 : 0);
                        minus = minus && idx[be][k] == dm;
                        plus = plus && idx[be][k] == dp;
                    }
                    if (minus) nbm[al][m] = be;
                    if (plus) nbp[al][m] = be;
                }
            }
    }
};

// sqrt(k) for the Hermite weights (k <= 8)
__device__ constexpr double kSqrtTab[9] = {0.0, 1.0, 1.4142135623730951, 1.7320508075688772, 2.0,
                                           2.2360679774997896, 2.4494897427831781, 2.6457513110645907,
                                           2.8284271247461903};

// Chaos coupling at one (cell, point, time index) for all modes, in registers: g[alpha] -> flux
//     f[alpha] = a_0(x_q) g[alpha] + sum_m a_{e_m}(x_q) (sqrt(alpha_m) g[alpha - e_m] + sqrt(alpha_m + 1) g[alpha + e_m]).
// The products a_{e_m}(x_q) sqrt(k), k = 1 .. P, are formed once per point, so every neighbour entry of
// the Galerkin tensor costs one FMA.
template <int M, int P, int NT, int NP, int RS, typename T>
__device__ __forceinline__ void couple_point(T* rows, const T* crow, int q, int ti, int mu0, const int* mum) {
    constexpr ChaosTab<M, P> tab{};
    constexpr int N = ChaosTab<M, P>::N;
    T g[N];
#pragma unroll
    for (int al = 0; al < N; ++al) g[al] = rows[(al * NT + ti) * RS + q];
    const T c0 = crow[mu0 * NP + q];
    T w[M][P];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const T cm = mum[m] >= 0 ? crow[mum[m] * NP + q] : T(0);
#pragma unroll
        for (int k = 0; k < P; ++k) w[m][k] = cm * T(kSqrtTab[k + 1]);
    }
#pragma unroll
    for (int al = 0; al < N; ++al) {
        T f = c0 * g[al];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int bm = tab.nbm[al][m], bp = tab.nbp[al][m];
            if (bm >= 0) f += w[m][tab.idx[al][m] - 1] * g[bm];
            if (bp >= 0) f += w[m][tab.idx[al][m]] * g[bp];
        }
        rows[(al * NT + ti) * RS + q] = f;
    }
}

// Makes the values opaque to the compiler at this point, so the arithmetic that forms them is done
// here: left alone, the compiler sinks the integration of every direction to the end of the cell
// work, past the barriers, and keeps all the flux values it reads live until then (register spills).
template <int N, typename T>
__device__ __forceinline__ void pin_values(T (&W)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) asm volatile("" : "+v"(W[q]));
}

// Points u_q of one (cell, component) at the Gauss points are in U; W accumulates the integrand.
template <int DIM, int K, int NT, typename T, bool MEAN, int CM, int CP, bool WIDE = false>
__device__ __forceinline__ void apply_body(const ApplyArgs<T>& a, const Tables<T>& tb, T (&U)[ipow(K + 1, DIM)],
                                           T (&W)[ipow(K + 1, DIM)], T* slot_rows, const T* slot_coef,
                                           const int* ent_g, const int* ent_c, const T* ent_w, int e0, int e1,
                                           int comp, int alpha, int ti, bool active, const int* cc,
                                           T* exch_all, const T* cl_all, int SS, int CS, long long cell_id) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int NS = NP / N1;   // points per slice
    constexpr int RS = row_stride(NP);
    T* const my_row = slot_rows + comp * RS;

    // time coupling of the mass term: W[q] = w_q h^d sum_j (A_t[i][j] / B_t[i]) u_j(q)
#pragma unroll
    for (int q = 0; q < NP; ++q) my_row[q] = U[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) W[q] = T(0);
#pragma unroll 1
    for (int j = 0; j < NT; ++j) {
        // row ti of A_t / B_t picked with selects (ti varies per lane; the table is uniform)
        T as = tb.As[j];
#pragma unroll
        for (int i = 1; i < NT; ++i) as = (ti == i) ? tb.As[i * NT + j] : as;
        const T* row = slot_rows + (alpha * NT + j) * RS;
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
    pin_values(W);

    if constexpr (MEAN) {
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
                pin_values(W);
            }
        }
    } else if constexpr (CM > 0) {
        // affine chaos coupling transposed: (cell, component) threads write d u / d x_dir, then
        // (cell, point, time) threads couple all modes in registers in place, then each
        // (cell, component) thread integrates its own flux row
        __syncthreads();
        const int cpb = a.cpb;
        const int ntask = cpb * NP * NT;
        // workgroup size from the arguments (blockDim would be read from the dispatch packet in memory)
        const int nthreads = cpb * a.n_xi * NT;
#pragma unroll
        for (int dir = 0; dir < DIM; ++dir) {
            const int st = ipow(N1, dir);
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
            for (int task = threadIdx.x; task < ntask; task += nthreads) {
                const int q = task % NP;
                const int tb_i = (task / NP) % NT;
                const int sl = task / (NP * NT);
                couple_point<CM, CP, NT, NP, RS, T>(exch_all + (size_t)sl * SS, cl_all + (size_t)sl * CS, q, tb_i, a.mu0,
                                                a.mum);
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < N1; ++s) {
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int q = (j / st) * st * N1 + s * st + (j % st);
                    const int base = q - s * st;
                    const T f = my_row[q];
#pragma unroll
                    for (int o = 0; o < N1; ++o) W[base + o * st] += tb.D[s * N1 + o] * f;
                }
            }
            pin_values(W);
        }
    } else {
        __syncthreads();
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
                    // entries from LDS, or (wide workgroups, whose LDS holds only the rows) from memory
                    const T w = WIDE ? a.cw[e] : ent_w[e];
                    const T* cp = slot_coef + (WIDE ? a.cmu[e] * NP : ent_c[e]);
                    const T* gp = slot_rows + (WIDE ? a.cbeta[e] * NT * RS : ent_g[e]) + ti * RS;
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
            pin_values(W);
            __syncthreads();
        }
    }

    // integrate back to the nodes (the caller scales by B_t and stores)
    sweeps_ip<DIM, N1, true>(W, tb.S);
}

// Minimum resident waves per SIMD the register allocator must allow (more waves hide the LDS and
// barrier latency of the exchange phases).  The FP64 mean block of cells up to 27 points fits the
// 168 registers of 3 waves without spilling (with its integration pinned slice by slice); the
// coupled FP64 kernels need about 210 and keep 2.
template <int NP, typename T, bool MEAN>
constexpr int apply_waves_per_eu() {
    return NP > 27 ? 1 : (sizeof(T) == 8 && !MEAN ? 2 : 3);
}

// Per-slot LDS strides padded so consecutive slots start on different banks.
template <typename T>
__host__ __device__ constexpr int padded_stride(int n) {
    constexpr int nb = sizeof(T) == 8 ? 16 : 32;   // 32 four-byte banks
    return n + ((1 - n) % nb + nb) % nb;
}

// LDS bank model of the exchange rows: the cycles of the wave instructions of the two access patterns
// (a (cell, component) thread at one point of its own row; a coupling task of (cell, point, time
// index) reading one mode), summed over `nb` banks of 4 bytes served `grp` lanes at a time.
inline long exch_bank_cycles(int np, int rs, int nt, int nc, int cpb, int ss, int words, int nb, int grp) {
    const int nthreads = nc * cpb;
    const int ntask = cpb * np * nt;
    long tot = 0;
    std::vector<int> cnt(nb), last(nb);
    std::vector<long long> addr(64);
    auto wave = [&](int nl) {
        for (int g0 = 0; g0 < nl; g0 += grp) {
            std::fill(cnt.begin(), cnt.end(), 0);
            std::fill(last.begin(), last.end(), -1);
            int worst = 0;
            for (int l = g0; l < std::min(nl, g0 + grp); ++l) {
                if (addr[l] < 0) continue;
                for (int w = 0; w < words; ++w) {
                    const int b = (int)((addr[l] * words + w) % nb);
                    bool dup = false;     // lanes reading the same word are served together
                    for (int l2 = g0; l2 < l; ++l2)
                        if (addr[l2] == addr[l]) { dup = true; break; }
                    if (!dup) worst = std::max(worst, ++cnt[b]);
                }
            }
            tot += worst;
        }
    };
    for (int w0 = 0; w0 < nthreads; w0 += 64) {
        const int nl = std::min(64, nthreads - w0);
        for (int q = 0; q < np; ++q) {
            for (int l = 0; l < nl; ++l) {
                const int t = w0 + l;
                addr[l] = (long long)(t % cpb) * ss + (long long)(t / cpb) * rs + q;
            }
            wave(nl);
        }
        for (int al = 0; al < std::min(nc / nt, 64); ++al) {
            for (int l = 0; l < nl; ++l) {
                const int t = w0 + l;
                addr[l] = t < ntask ? (long long)(t / (np * nt)) * ss + (long long)(al * nt + (t / np) % nt) * rs + t % np
                                    : -1;
            }
            wave(nl);
        }
    }
    return tot;
}

// Slot stride of the exchange rows (>= nc rs elements): the residue, modulo the bank period, with the
// fewest modelled cycles under both a 32- and a 64-bank LDS.
template <typename T>
inline int exch_slot_stride(int np, int nt, int nc, int cpb) {
    const int rs = row_stride(np);
    const int words = sizeof(T) / 4;
    const int period = 32 / words;
    const int base = nc * rs;
    if (cpb == 1) return base;
    int best = base;
    long best_c = -1;
    for (int r = 0; r < period; ++r) {
        const int ss = base + r;
        const long c = exch_bank_cycles(np, rs, nt, nc, cpb, ss, words, 32, 32 / words) +
                       exch_bank_cycles(np, rs, nt, nc, cpb, ss, words, 64, 64 / words);
        if (best_c < 0 || c < best_c) { best_c = c; best = ss; }
    }
    return best;
}

// Position of thread t of workgroup b: its cell slot and component, the workgroup's segment of cpb
// cells along x (segs per cell row; rows in the XCD-local tiled order) and the cell's coordinates.
template <int DIM>
struct ApplyPos {
    int slot, comp, seg, segs, x0;
    bool active;
    long long cell0;   // first cell of the segment
    int cc[3];
};
template <int DIM, typename T>
__device__ __forceinline__ ApplyPos<DIM> apply_position(const ApplyArgs<T>& a, int cpb, int t, int b) {
    ApplyPos<DIM> P;
    const int n = a.g.n;
    P.comp = apply_quot(a.fcpb, t);
    P.slot = t - P.comp * cpb;
    P.segs = a.segs;
    const int lb = xcd_position(b, a.nblocks);
    const int o = apply_quot(a.fsegs, lb);        // row in traversal order
    P.seg = lb - o * P.segs;
    P.x0 = P.seg * cpb;
    int row = o;                                   // tiled_row with the quotients precomputed
    if constexpr (DIM == 3) {
        const int chunk = apply_quot(a.ftyn, o);
        const int rem = o - chunk * (n << a.tylg);
        row = (chunk << a.tylg) + (rem & ((1 << a.tylg) - 1)) + n * (rem >> a.tylg);
    }
    const int c0 = row * n + P.x0;                 // cell indices fit 32 bits
    P.cell0 = c0;
    P.active = P.x0 + P.slot < n;
    int r = P.active ? c0 + P.slot : 0;
    P.cc[0] = P.cc[1] = P.cc[2] = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int q = apply_quot(a.fn, r);
        P.cc[d] = r - q * n;
        r = q;
    }
    return P;
}

// WIDE: one cell per workgroup of up to 1024 threads (N_xi N_t > 512 components), coupling entries
// read from memory instead of LDS.
template <int DIM, int K, int NT, typename T, bool MEAN, int CM = 0, int CP = 0, bool WIDE = false>
__global__ void __launch_bounds__(WIDE ? 1024 : (ipow(K + 1, DIM) > 27 ? 256 : 512))
    __attribute__((amdgpu_waves_per_eu(WIDE ? 4 : apply_waves_per_eu<ipow(K + 1, DIM), T, MEAN>())))
    k_apply(ApplyArgs<T> a, Tables<T> tb) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    extern __shared__ unsigned char smem_raw[];
    const int cpb = a.cpb;
    const int NC = a.n_xi * NT;
    const int SS = a.ss;                                     // slot stride of the exchange rows
    const int CS = padded_stride<T>(a.n_mu * NP);            // slot stride of the coefficient rows
    T* exch = reinterpret_cast<T*>(smem_raw);               // [cpb][SS]: rows [NC][NP]
    T* cl = exch + (size_t)SS * cpb;                         // [cpb][CS]: rows [n_mu][NP]
    T* ent_w = cl + (size_t)CS * cpb;                        // [n_ent] G_mu[alpha][beta]
    int* ent_g = reinterpret_cast<int*>(ent_w + a.n_ent);    // [n_ent] LDS row offset of beta
    int* ent_c = ent_g + a.n_ent;                            // [n_ent] LDS row offset of mu

    const int t = threadIdx.x;
    const int nthreads = NC * cpb;                           // the workgroup size
    const ApplyPos<DIM> P = apply_position<DIM>(a, cpb, t, blockIdx.x);
    const int slot = P.slot, comp = P.comp, x0 = P.x0;
    const int alpha = comp / NT;
    const int ti = comp % NT;
    const int n = a.g.n, n1 = a.g.n1;
    const long long cell0 = P.cell0;
    const long long ci = cell0 + slot;
    const bool active = P.active;
    const long long nn = a.g.n_nodes;
    const int* const cc = P.cc;

    // All loads of the prologue are issued before the first wait: the coefficient values of this block's
    // cells (contiguous in memory; into registers when every thread's share fits CPF of them), then the
    // cell's nodal values.  Loads complete in order, so storing the coefficients to LDS waits only for
    // their own loads, and one memory round trip serves the whole prologue.
    constexpr int CPF = 4;
    const int ncoef = a.n_mu * NP * cpb;
    const bool cpf_ok = ncoef <= CPF * nthreads;
    T cv[CPF];
    if (cpf_ok) {
#pragma unroll
        for (int i = 0; i < CPF; ++i) {
            const int idx = t + i * nthreads;
            const int j = idx / NP, q = idx - j * NP;
            const int s = apply_quot(a.fnmu, j), mu = j - s * a.n_mu;
            cv[i] = (idx < ncoef && x0 + s < n) ? a.coef[mu * a.coef_mode_stride + (cell0 + s) * NP + q] : T(0);
        }
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

    if (cpf_ok) {
#pragma unroll
        for (int i = 0; i < CPF; ++i) {
            const int idx = t + i * nthreads;
            if (idx < ncoef) {
                const int j = idx / NP, q = idx - j * NP;
                const int s = apply_quot(a.fnmu, j), mu = j - s * a.n_mu;
                cl[s * CS + mu * NP + q] = cv[i];
            }
        }
    } else {
        for (int idx = t; idx < ncoef; idx += nthreads) {
            const int j = idx / NP, q = idx - j * NP;
            const int s = apply_quot(a.fnmu, j), mu = j - s * a.n_mu;
            const long long c2 = cell0 + s;
            cl[s * CS + mu * NP + q] = (x0 + s < n) ? a.coef[mu * a.coef_mode_stride + c2 * NP + q] : T(0);
        }
    }
    // stage the coupling entries (beta, mu, w) as LDS offsets
    if constexpr (!MEAN && CM == 0 && !WIDE) {
        for (int e = t; e < a.n_ent; e += nthreads) {
            ent_w[e] = a.cw[e];
            ent_g[e] = a.cbeta[e] * NT * row_stride(NP);
            ent_c[e] = a.cmu[e] * NP;
        }
    }
    int e0 = 0, e1 = 0;
    if constexpr (!MEAN && CM == 0) {
        e0 = a.cptr[alpha * a.n_mu];
        e1 = a.cptr[(alpha + 1) * a.n_mu];
    }

    T* const slot_rows = exch + (size_t)slot * SS;
    const T* const slot_coef = cl + (size_t)slot * CS;
    // values at the Gauss points, then the rest of the cell work
    sweeps_ip<DIM, N1, false>(A, tb.S);
    apply_body<DIM, K, NT, T, MEAN, CM, CP, WIDE>(a, tb, A, B, slot_rows, slot_coef, ent_g, ent_c, ent_w, e0, e1, comp, alpha,
                                            ti, active, cc, exch, cl, SS, CS, active ? ci : 0);

    // Register-resident chaos coupling on cells of up to 27 points: the position is formed again from
    // opaque copies of the ids, since the first one, kept alive across the cell work, would take
    // registers at its peak (and be spilled to scratch memory).  The other variants keep it (their
    // register allocation does as well or better with it).
    int t2 = threadIdx.x, b2 = blockIdx.x;
    if constexpr (CM > 0 && NP <= 27) asm volatile("" : "+v"(t2), "+s"(b2));
    const ApplyPos<DIM> E = apply_position<DIM>(a, cpb, t2, b2);
    const T scale = bt_of<NT>(tb, E.comp % NT);
#pragma unroll
    for (int p = 0; p < NP; ++p) B[p] *= scale;
    if constexpr (!WIDE) {
        if (a.merge) {
            // x faces shared by consecutive cells of the segment: the upper cell adds the lower cell's
            // x = k face (the same two-term sum the gather would form) and the lower one skips it
            constexpr int NS = NP / N1;
            __syncthreads();                              // the exchange rows are free again
            T* const mine = exch + (size_t)E.slot * SS + E.comp * row_stride(NP);
#pragma unroll
            for (int j = 0; j < NS; ++j) mine[j] = B[j * N1 + K];
            __syncthreads();
            if (E.slot > 0) {
                const T* const prev = mine - SS;
#pragma unroll
                for (int j = 0; j < NS; ++j) B[j * N1] = prev[j] + B[j * N1];
            }
            if (E.active)
                store_merged<DIM, K, T>(a.s, B, E.cc, a.g.n, E.comp, E.seg, E.segs, cpb, E.slot,
                                        E.slot == cpb - 1 || E.x0 + E.slot == a.g.n - 1);
            return;
        }
    }
    if (E.active) store_broken<DIM, K, T>(a.s, B, T(1), E.cc, a.g.n, E.comp);
}

// Cells per workgroup: the largest number of busy lanes per CU, with the number of resident
// workgroups per CU from the runtime's occupancy calculator (registers, LDS, wave slots), among the
// sizes that keep at least two workgroups per CU when there are any (a second workgroup runs while
// the first waits at one of its barriers).
inline int choose_cpb_uncached(const void* kern, int nc, size_t lds_fixed, size_t lds_per_cell, int max_threads) {
    int best = 1;
    long best_score = -1;
    for (int cpb = 1; nc * cpb <= max_threads; ++cpb) {
        const int threads = nc * cpb;
        const size_t lds = lds_fixed + lds_per_cell * cpb;
        if (lds > 160 * 1024) break;
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, threads, lds) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        const long score = (long)blocks * threads + (blocks >= 2 ? (1L << 30) : 0);
        if (blocks > 0 && score > best_score) {
            best_score = score;
            best = cpb;
        }
    }
    return best;
}

// The slot stride depends only on the sizes; remember it (the apply launch path is hot).
template <typename T>
inline int cached_slot_stride(int np, int nt, int nc, int cpb) {
    struct Entry {
        int np, nt, nc, cpb, ss;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry& e : cache)
            if (e.np == np && e.nt == nt && e.nc == nc && e.cpb == cpb) return e.ss;
    }
    const int ss = exch_slot_stride<T>(np, nt, nc, cpb);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({np, nt, nc, cpb, ss});
    return ss;
}

// The choice depends only on the kernel and the sizes; remember it (the apply launch path is hot).
inline int choose_cpb(const void* kern, int nc, size_t lds_fixed, size_t lds_per_cell, int max_threads) {
    struct Entry {
        const void* kern;
        int nc;
        size_t fixed, per_cell;
        int cpb;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry& e : cache)
            if (e.kern == kern && e.nc == nc && e.fixed == lds_fixed && e.per_cell == lds_per_cell) return e.cpb;
    }
    const int cpb = choose_cpb_uncached(kern, nc, lds_fixed, lds_per_cell, max_threads);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({kern, nc, lds_fixed, lds_per_cell, cpb});
    return cpb;
}

template <int DIM, int K, int NT, typename T>
hipError_t run_apply(const ApplyOp<T>& op, const T* x, T* s_out, hipStream_t s) {
    constexpr int N1 = K + 1;
    constexpr int NP = ipow(N1, DIM);
    constexpr int MAXT = NP > 27 ? 256 : 512;
    auto kern = op.mean ? k_apply<DIM, K, NT, T, true> : k_apply<DIM, K, NT, T, false>;
    // register-resident chaos coupling for the affine index sets of the benchmark workloads
    if (!op.mean && op.affine) {
        if constexpr (DIM == 3 && K == 2 && NT == 2) {
            if (op.chaos_m == 4 && op.chaos_p == 3) kern = k_apply<DIM, K, NT, T, false, 4, 3>;
        }
        if constexpr (DIM == 3 && K == 3 && NT == 3) {
            if (op.chaos_m == 3 && op.chaos_p == 4) kern = k_apply<DIM, K, NT, T, false, 3, 4>;
        }
        if constexpr (DIM == 2 && K == 2 && NT == 2) {
            if (op.chaos_m == 2 && op.chaos_p == 2) kern = k_apply<DIM, K, NT, T, false, 2, 2>;
        }
        if constexpr (DIM == 3 && K == 2 && NT == 2) {
            if (op.chaos_m == 3 && op.chaos_p == 2) kern = k_apply<DIM, K, NT, T, false, 3, 2>;
        }
    }
    ApplyArgs<T> a{};
    a.x = x;
    a.s = s_out;
    a.coef = op.coef;
    a.coef_mode_stride = op.coef_mode_stride;
    a.cptr = op.cptr;
    a.cbeta = op.cbeta;
    a.cmu = op.cmu;
    a.cw = op.cw;
    a.n_xi = op.n_xi;
    a.n_mu = op.n_mu;
    a.n_ent = op.n_ent;
    a.g = op.g;
    a.mu0 = op.mu0;
    for (int m = 0; m < 8; ++m) a.mum[m] = op.mum[m];
    const int nc = op.n_xi * NT;
    constexpr int RS = row_stride(NP);
    const size_t cs_bytes = (size_t)padded_stride<T>(op.n_mu * NP) * sizeof(T);
    // upper bound of one cell's LDS (the slot stride adds less than one bank period to nc RS)
    const size_t per_cell = (size_t)(nc * RS + 32 / (sizeof(T) / 4)) * sizeof(T) + cs_bytes;
    if (nc > MAXT) {
        // more components than one regular workgroup: one cell per workgroup of nc <= 1024 threads (2D)
        if constexpr (DIM == 2) {
            auto wk = op.mean ? k_apply<DIM, K, NT, T, true, 0, 0, true> : k_apply<DIM, K, NT, T, false, 0, 0, true>;
            a.cpb = 1;
            set_apply_divisors(a, 1);
            a.merge = 0;
            a.ss = nc * RS;
            if (op.used_cpb) *op.used_cpb = 1;
            if (op.used_lz) *op.used_lz = 1;
            const size_t lds = (size_t)a.ss * sizeof(T) + cs_bytes + 16;
            if (nc > 1024 || lds > 160 * 1024) return hipErrorInvalidConfiguration;
            if (lds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)wk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            const long long blocks = op.g.n_cells;
            a.nblocks = (int)blocks;
            hipLaunchKernelGGL(wk, dim3((unsigned)blocks), dim3(nc), lds, s, a, *op.tables);
            return hipGetLastError();
        } else {
            return hipErrorInvalidConfiguration;
        }
    }
    const size_t fixed = op.mean ? 16 : (size_t)op.n_ent * (sizeof(T) + 2 * sizeof(int)) + 16;
    const int cpb = op.cells_per_block > 0 ? op.cells_per_block : choose_cpb((const void*)kern, nc, fixed, per_cell, MAXT);
    a.cpb = cpb;
    set_apply_divisors(a, cpb);
    a.merge = op.merge && cpb > 1;
    a.ss = cached_slot_stride<T>(NP, NT, nc, cpb);
    if (op.used_cpb) *op.used_cpb = cpb;
    if (op.used_lz) *op.used_lz = 1;     // one cell layer per workgroup: the z layout is per cell
    const int threads = nc * cpb;
    const size_t lds = fixed + ((size_t)a.ss * sizeof(T) + cs_bytes) * cpb;
    if (threads > MAXT || lds > 160 * 1024) return hipErrorInvalidConfiguration;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const long long rows = op.g.n_cells / op.g.n;
    const long long blocks = rows * ((op.g.n + cpb - 1) / cpb);
    a.nblocks = (int)blocks;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), lds, s, a, *op.tables);
    return hipGetLastError();
}

template <int DIM, int K, typename T>
hipError_t dispatch_nt(const ApplyOp<T>& op, const T* x, T* s_out, hipStream_t s) {
    switch (op.nt) {
        case 1: return run_apply<DIM, K, 1, T>(op, x, s_out, s);
        case 2: return run_apply<DIM, K, 2, T>(op, x, s_out, s);
        case 3: return run_apply<DIM, K, 3, T>(op, x, s_out, s);
        case 4: return run_apply<DIM, K, 4, T>(op, x, s_out, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// All (k, N_t) instances of one dimension and precision; instantiated in apply_<d>d_<type>.hip.
template <int DIM, typename T>
hipError_t apply_dim(const ApplyOp<T>& op, const T* x, T* s_out, hipStream_t s) {
    switch (op.k) {
        case 1: return dispatch_nt<DIM, 1, T>(op, x, s_out, s);
        case 2: return dispatch_nt<DIM, 2, T>(op, x, s_out, s);
        case 3: return dispatch_nt<DIM, 3, T>(op, x, s_out, s);
        case 4: return dispatch_nt<DIM, 4, T>(op, x, s_out, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace sg
