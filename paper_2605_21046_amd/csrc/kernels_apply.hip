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
#include "kernels.hpp"

namespace sg {

template <int DIM, typename T>
hipError_t apply_dim(const ApplyOp<T>& op, const T* x, T* y, const T* b, hipStream_t s);

template <typename T>
hipError_t launch_apply(const ApplyOp<T>& op, const T* x, T* y, const T* b, hipStream_t s) {
    if (op.dim == 2) return apply_dim<2, T>(op, x, y, b, s);
    if (op.dim == 3) return apply_dim<3, T>(op, x, y, b, s);
    return hipErrorInvalidValue;
}

template <typename T>
size_t apply_lds_bytes(const ApplyOp<T>& op, int cpb) {
    size_t np = 1;
    for (int d = 0; d < op.dim; ++d) np *= (size_t)(op.k + 1);
    return (size_t)(op.n_xi * op.nt + op.n_mu) * np * cpb * sizeof(T);
}

template hipError_t launch_apply<double>(const ApplyOp<double>&, const double*, double*, const double*, hipStream_t);
template hipError_t launch_apply<float>(const ApplyOp<float>&, const float*, float*, const float*, hipStream_t);
template size_t apply_lds_bytes<double>(const ApplyOp<double>&, int);
template size_t apply_lds_bytes<float>(const ApplyOp<float>&, int);

}  // namespace sg
