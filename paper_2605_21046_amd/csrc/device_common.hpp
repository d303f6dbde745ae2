// Shared device-side definitions: constant tables passed by value to kernels, small index helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace sg {

constexpr int kMaxN1 = 5;   // k + 1 <= 5 (Q1 .. Q4)
constexpr int kMaxNT = 4;   // r + 1 <= 4 (dG(0) .. dG(3))

// b^e, iterative: device code with a run-time exponent inlines and folds it (a recursive form is
// not inlined, and such a call forces the whole kernel onto the call ABI with scratch spills)
__host__ __device__ __forceinline__ constexpr int ipow(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// 1D reference tables and time matrices, copied into the kernel argument segment.
//   S[q][a]  = l_a(g_q): GLL Lagrange basis a at Gauss point q          (interpolation to points)
//   D[q][p]  = m_p'(g_q): derivative of the Gauss-point Lagrange basis   (collocation derivative)
//   w[q]     = Gauss weight on (0,1)
//   As[i][j] = A_t[i][j] / B_t[i]   (the evolution matrix scaled so B_t factors out at the end)
//   Bt[i]    = B_t[i][i]
//   vol      = h^d (mass scaling);  stiffness scaling h^(d-2) is folded into the coefficients.
template <typename T>
struct Tables {
    T S[kMaxN1 * kMaxN1];
    T D[kMaxN1 * kMaxN1];
    T w[kMaxN1];
    T As[kMaxNT * kMaxNT];
    T Bt[kMaxNT];
    T vol;
};

// Uniform Cartesian mesh of one level.
struct Grid {
    int n;              // cells per direction
    int n1;             // nodes per direction = n k + 1
    long long n_nodes;  // n1^d
    long long n_cells;  // n^d
};

// Traversal order of cell rows (a row = the n cells along x at fixed y, z).  Workgroups are
// dispatched round-robin over the 8 XCDs; XCD x gets the contiguous position range
// [x q + min(x, r), ...) of the nb positions, so the rows it walks in turn stay in its L2.  In 3D the
// rows are visited in chunks of `ty` consecutive y (ty | n), z running over the chunk, y fastest:
// rows in flight together then share node planes in both y and z.
__device__ __forceinline__ int xcd_position(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int x = b % 8;
    return x * q + min(x, r) + b / 8;
}
__host__ __device__ constexpr int row_tile(int n) { return n % 4 == 0 ? 4 : (n % 2 == 0 ? 2 : 1); }
// row (y + n z, or y in 2D) of the o-th row in traversal order
template <int DIM>
__device__ __forceinline__ int tiled_row(int o, int n) {
    if constexpr (DIM == 2) {
        return o;
    } else {
        const int ty = row_tile(n);
        const int chunk = o / (ty * n), rem = o % (ty * n);
        return chunk * ty + rem % ty + n * (rem / ty);
    }
}

}  // namespace sg
