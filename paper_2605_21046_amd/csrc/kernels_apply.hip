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
//   * no scatter: cell-local results go to a broken node array that k_node_gather sums per node.
#include "kernels.hpp"

namespace sg {

template <int DIM, typename T>
hipError_t apply_dim(const ApplyOp<T>& op, const T* x, T* s_out, hipStream_t s);

template <typename T>
hipError_t launch_apply(const ApplyOp<T>& op, const T* x, T* s_out, hipStream_t s) {
    if (op.dim == 2) return apply_dim<2, T>(op, x, s_out, s);
    if (op.dim == 3) return apply_dim<3, T>(op, x, s_out, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_apply<double>(const ApplyOp<double>&, const double*, double*, hipStream_t);
template hipError_t launch_apply<float>(const ApplyOp<float>&, const float*, float*, hipStream_t);

}  // namespace sg
