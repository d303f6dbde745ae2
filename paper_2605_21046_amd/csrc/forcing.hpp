// Forcing assembly, separable slab vectors and space-time error sums (kernels_forcing.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sg {

// 1D tables of the GLL Lagrange basis at an nq1-point Gauss rule on (0, 1): values V[q][a], reference
// derivatives D[q][a], weights w[q] (nq1 <= 8, k <= 4).
constexpr int kMaxQ1 = 8;
struct QTables {
    double V[kMaxQ1][5];
    double D[kMaxQ1][5];
    double w[kMaxQ1];
};
// Time rule on one slab: basis values v[i][k] at the rule's points, weights w[k] (times tau) and the
// temporal factor theta at the points' physical times.
constexpr int kMaxTimeQ = 8;
struct TimeTables {
    double v[4][kMaxTimeQ];
    double w[kMaxTimeQ];
    double theta[kMaxTimeQ];
    int ntq;
};
// S[field][broken node] = sum_q w_q |K| (f psi_a + g . grad psi_a) for nf fields
hipError_t launch_load_cells(int dim, int k, Grid g, int nq1, const QTables& tb, double h, const double* f,
                             const double* gq, int nf, double* S, hipStream_t s);
// y = beta y + sum_t W[t][comp] V[t][node]
hipError_t launch_separable(int n_terms, int ncomp, long long nn, const double* W, const double* V, double beta,
                            double* y, hipStream_t s);
// per-cell error sums [n_cells][8]: full L2, full H1, mean L2, mean H1, var L2, var H1, |theta s|^2,
// |theta grad s|^2 against c_alpha theta(t) s(x)
bool error_cells_supported(int dim, int k, int nt);
hipError_t launch_error_cells(int dim, int k, int nt, Grid g, int nq1, const QTables& tb, double h,
                              const TimeTables& tt, int n_xi, const double* u, const double* c, double C2,
                              const double* s_qp, const double* gs_qp, double* part, hipStream_t s);

// acc[cell][q][tq][2] += (sum_s u_s, sum_s u_s^2) at the quadrature points, over the n_s samples of u
hipError_t launch_sample_qp_moments(int dim, int k, int nt, Grid g, int nq1, const QTables& tb, const TimeTables& tt,
                                    int n_s, const double* u, double* acc, hipStream_t s);
// part[cell][6]: squared errors of the sample mean / unbiased variance (from acc) against m_j theta s and
// v_j theta^2 s^2, then |theta s|^2 and |theta^2 s^2|^2
hipError_t launch_moment_errors(int dim, Grid g, int nq1, const QTables& tb, double h, const TimeTables& tt, double n_tot,
                                const double* acc, const double* s_qp, double m0, double m1, double v0, double v1,
                                double* part, hipStream_t s);

}  // namespace sg
