// Host-side discretisation data: 1D quadrature and Lagrange tables, dG(r) time matrices, the
// total-degree Hermite index set and the Galerkin coupling lists.  Plain C++17, no device code.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sg {

// Legendre polynomial P_n(x) and its derivative by the three-term recurrence.
void legendre(int n, double x, double* p, double* dp);

// Nodes and weights on the reference interval (0, 1).
std::vector<double> gauss_points(int n, std::vector<double>* weights);      // n-point Gauss-Legendre
std::vector<double> gll_points(int k);                                      // k+1 Gauss-Lobatto points
std::vector<double> right_radau_points(int r);                              // r+1 points, last = 1

// Lagrange basis on `nodes` evaluated at `x`: value and first derivative of basis function a.
double lagrange_value(const std::vector<double>& nodes, int a, double x);
double lagrange_deriv(const std::vector<double>& nodes, int a, double x);

// Time matrices of dG(r) on a slab of length tau (Section 2.5, eqs. At, Bt):
//   At[i][j] = int_0^1 l_j' l_i ds + l_j(0) l_i(0),  Bt[i][j] = tau int_0^1 l_j l_i ds.
// Bt is diagonal for the right-Radau basis (the (r+1)-point Radau rule is exact to degree 2r);
// the function checks that and returns only its diagonal.
bool time_matrices(int r, double tau, std::vector<double>* At, std::vector<double>* Bt_diag);

// Total-degree index set in graded, lexicographically descending order (Section 2.6).
std::vector<std::vector<int>> total_degree_set(int M, int p);

// E[psi_a psi_b psi_c] for orthonormal probabilists' Hermite polynomials (linearisation formula).
double hermite_triple_1d(int a, int b, int c);

// Coupling lists of sum_mu a_mu(x) G_mu: for every (alpha, mu) the nonzero entries
// (beta, [G_mu]_{alpha beta}), stored CSR-like with row index alpha * n_mu + mu.
struct Coupling {
    int n_xi = 0, n_mu = 0;
    std::vector<int> ptr;     // n_xi * n_mu + 1
    std::vector<int> beta;
    std::vector<double> w;
    bool affine = true;       // every mu in {0, e_1, ..., e_M}
    int mu0 = -1;             // position of mu = 0
};
bool build_coupling(int M, int p, int n_mu, const int* mu, Coupling* out, std::string* err);

// Normalised probabilists' Hermite polynomial He_n(x) / sqrt(n!).
double hermite_normalized(int n, double x);

// A batch of pathwise problems (Section 5.1: one deterministic problem per sample xi^(s)) in the
// same Kronecker form: "mode" s is sample s and G_mu = diag(Psi_mu(xi^(s))), so sum_mu G_mu a_mu is
// the sampled coefficient a(x, xi^(s)) on the diagonal.  xi is [n_samples][M].
bool build_sample_coupling(int M, int n_samples, const double* xi, int n_mu, const int* mu, Coupling* out,
                           std::string* err);

// A batch of independent stochastic Galerkin problems in one Kronecker form: member j has the
// total-degree set of degree degrees[j] and the coefficient sum_mu scale[j][mu] a_mu, so G_mu is
// block diagonal with blocks scale[j][mu] G_mu(Lambda_{p_j}).  Global mode = offsets[j] + local mode;
// offsets has n_members + 1 entries.  scale[j][mu = 0] must be 1 (the members share the mean field).
bool build_batch_coupling(int M, int n_members, const int* degrees, const double* scale, int n_mu, const int* mu,
                          Coupling* out, std::vector<int>* offsets, std::string* err);

}  // namespace sg
