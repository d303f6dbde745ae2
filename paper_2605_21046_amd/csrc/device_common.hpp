// Shared device-side definitions: constant tables passed by value to kernels, small index helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace sg {

constexpr int kMaxN1 = 5;   // k + 1 <= 5 (Q1 .. Q4)
constexpr int kMaxNT = 4;   // r + 1 <= 4 (dG(0) .. dG(3))

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

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

// Index of the multigrid node line / cell colouring helpers.
struct Grid {
    int n;              // cells per direction
    int n1;             // nodes per direction = n k + 1
    long long n_nodes;  // n1^d
    long long n_cells;  // n^d
};

}  // namespace sg
