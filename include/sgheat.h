/*
 * sgheat.h -- C ABI of libsgheat.so: matrix-free stochastic-Galerkin space-time slab operator, its
 * Vanka-smoothed geometric-multigrid preconditioner and the flexible-GMRES slab solve, on one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem is the slab system of the paper (Problem "tensor-product-slab-system", eqs.
 * local_tensor_system and local_rhs_tensor):
 *
 *     AA U = rhs,   AA = I_xi (x) A_t (x) M_x + sum_{mu in M_a} G_mu (x) B_t (x) K_mu,
 *
 * with the dG(r) right-Radau time matrices A_t (evolution, eq. At) and B_t (mass, eq. Bt), the
 * Hermite triple-product tensors G_mu (eq. triple_stoch) and the Q_k mass / coefficient-weighted
 * stiffness matrices M_x, K_mu on a uniform Cartesian mesh of (lo, hi)^d.
 *
 * Conventions shared by every entry point:
 *   - Vectors are DEVICE pointers owned by the caller, contiguous, in the precision named by the
 *     argument type, laid out mode-major: index = alpha * (N_t * N_x) + i * N_x + node, where
 *     alpha runs over the total-degree chaos index set (graded by |alpha|, lexicographically
 *     descending inside a degree), i over the N_t = r+1 time DoFs, and node over the
 *     (n k + 1)^d Lagrange nodes (Gauss-Lobatto support points), lexicographic with x fastest.
 *     Boundary nodes are part of the vector.
 *   - Homogeneous Dirichlet condition: rows of boundary DoFs are identity rows; boundary columns
 *     are dropped from the other rows.
 *   - Streams: `hip_stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     enqueued on that stream only.  Calls on one handle share its work buffers: calls on different
 *     streams must be ordered by the caller (events), as they would race otherwise.  Every
 *     asynchronous call records an event of the handle on its stream at the end (unless the stream
 *     is being captured into a graph); sg_update_coefficients, sg_set_vcycle_segment,
 *     sg_set_vcycle_graph and sg_destroy wait for that event, i.e. for the handle's last call and
 *     everything ordered before it, never for the whole device.
 *   - Errors: every call returns an sg_status; arguments are checked before anything is enqueued.
 *     No C++ exception crosses the ABI.  sg_last_error() gives a thread-local message for the last
 *     non-OK status of the calling thread.
 *   - Aliasing: input and output vectors of one call must not overlap (SG_EINVAL).
 */
#ifndef SGHEAT_H
#define SGHEAT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_handle_s* sg_handle;

typedef enum {
    SG_OK = 0,
    SG_NOT_CONVERGED = 1,   /* fgmres_solve_slab hit max_iter; x and info still hold the best iterate */
    SG_EINVAL = -1,         /* invalid argument (null pointer, bad size, aliasing, unsupported combination) */
    SG_ENOMEM = -2,         /* device or host allocation failed */
    SG_EHIP = -3,           /* a HIP runtime call failed; the message names it */
    SG_ESINGULAR = -4,      /* a Vanka patch matrix or the coarsest-level matrix is singular */
    SG_EUNSUPPORTED = -5    /* valid request the library does not implement (e.g. too many components per cell) */
} sg_status;

typedef enum {
    SG_FP64 = 0,            /* every step in FP64 */
    SG_MIXED = 1            /* V-cycle and Vanka in FP32 on fine levels, FP64 coarsest-level inverse, FP64 outer FGMRES */
} sg_precision;

/* Problem description (all arrays are HOST memory, copied by sg_create). */
typedef struct {
    int dim;                /* d in {2, 3} (Section 2.1)                                              */
    int n_cells_1d;         /* finest mesh: n^d cells of (lo, hi)^d                                   */
    double lo, hi;          /* domain bounds                                                          */
    int fe_degree;          /* k of Q_k, 1..4 (Section 2.4)                                          */
    int time_degree;        /* r of dG(r), 0..3, right Gauss-Radau nodal basis (Section 2.5)          */
    double tau;             /* slab length                                                            */
    int n_vars;             /* M, number of standard Gaussian variables (eq. random_varibale_law)     */
    int chaos_degree;       /* p_xi, total degree of the chaos space (Section 2.6)                   */
    int n_coef_modes;       /* |M_a|, active coefficient modes (eq. coeff_expansion)                  */
    const int* coef_mu;     /* [n_coef_modes][n_vars] multi-indices; must contain mu = 0              */
    const double* coef_qp;  /* [n_levels][n_coef_modes][n_cells(l)][(k+1)^d]: a_mu at the Gauss points
                               of level l (cells and points lexicographic, x fastest)                */
    int n_levels;           /* multigrid levels, 0 = finest; n_cells_1d must be divisible by 2^(n_levels-1) */
    int pre_smooth, post_smooth;  /* Vanka sweeps before / after the coarse correction               */
    double vanka_omega;     /* damping of the additive Vanka correction                              */
    int fgmres_restart;     /* Krylov basis length before restart (<= 64)                            */
    sg_precision precision;
    int n_samples;          /* 0: stochastic Galerkin (modes = the total-degree set of degree p_xi).
                             * > 0: a batch of pathwise problems (Section 5.1, Problem
                             * mc-pathwise-deterministic): "mode" s is the sample xi^(s) = samples[s],
                             * G_mu = diag(Psi_mu(xi^(s))), so row block s is the deterministic slab
                             * system with coefficient a(x, xi^(s)); chaos_degree is then ignored.  The
                             * preconditioner keeps the mean block A_0 for every sample.             */
    const double* samples;  /* host [n_samples][n_vars] (copied), used when n_samples > 0            */
    int n_members;          /* 0: one stochastic Galerkin problem.  > 0: a batch of independent SG
                             * problems in one handle (exclusive with n_samples): member j has the
                             * total-degree index set of degree member_degree[j] (chaos_degree is then
                             * ignored) and the coefficient sum_mu member_scale[j][mu] a_mu, so each
                             * G_mu is block diagonal over the members.  Modes are numbered member by
                             * member (member j's modes follow those of members 0..j-1, each in the
                             * graded order of a single problem).                                       */
    const int* member_degree;     /* host [n_members] (copied)                                       */
    const double* member_scale;   /* host [n_members][n_coef_modes] (copied); the mu = 0 entry must be 1 */
    int diag_blocks;        /* 0: the block-Jacobi preconditioner uses the mean block A_0 for every mode
                             * (exact for an affine coefficient).  1: every mode alpha gets its own
                             * diagonal block A_alpha = A_t (x) M_x + B_t (x) K_{a_alpha},
                             * a_alpha = sum_mu [G_mu]_{alpha alpha} a_mu (for a sample batch: the
                             * sample's coefficient), on every level: per-mode Vanka patch inverses,
                             * residuals and coarsest-level inverses (N_xi times the memory of the
                             * patch inverses; the coarsest level should be small).                   */
    int transpose;          /* 0: the slab operator AA; 1: its transpose AA^T (the adjoint slab
                             * problem).  Every G_mu (a triple-product matrix), M_x and K_mu is symmetric
                             * and B_t is diagonal, so AA^T is AA with A_t replaced by A_t^T; every entry
                             * point of the handle (apply, Vanka, V-cycle, FGMRES) then acts on AA^T. */
} sg_problem_desc;

/* Counters of one slab solve (mirrors the paper's Table tab:finite-size-work-solver-performance). */
typedef struct {
    int iterations;         /* FGMRES iterations (= preconditioner calls)                             */
    int restarts;           /* Arnoldi cycles started                                                 */
    int vcycles;            /* gmg V-cycles applied                                                   */
    int applies;            /* operator applications (vmult calls), including true-residual checks    */
    int converged;          /* 1 if ||b - AA x|| / ||b|| <= rtol                                      */
    double rel_residual_true;
    double t_apply_ms, t_prec_ms, t_total_ms;   /* accumulated, from HIP events on the stream         */
    double work_proxy;      /* N_SG,slab * preconditioner calls (eq. work-proxy)                     */
} sg_solve_info;

/* Build the handle for one slab problem (Problem tensor-product-slab-system: the description fixes
 * the spatial mesh and Q_k space, the dG(r) slab of length tau, the chaos index set and the active
 * coefficient modes of eq. local_rhs_tensor; the multigrid fields configure the block-Jacobi
 * preconditioner of Remark solver-matrix-free-sg).  Copies the description, builds the chaos
 * coupling lists, time matrices, 1D tables and level data, uploads the coefficients, forms every
 * Vanka patch matrix and inverts it on the device (Gauss-Jordan elimination with partial pivoting in
 * FP64), and inverts the coarsest-level matrix on the device the same way.  Synchronous.
 * Returns SG_EINVAL for inconsistent descriptions (a multi-index listed twice in coef_mu included),
 * SG_ESINGULAR for a singular patch or coarsest-level matrix. */
sg_status sg_create(const sg_problem_desc* desc, sg_handle* out);

/* Release every device and host resource of the handle after its last asynchronous call has
 * completed.  NULL is accepted. */
sg_status sg_destroy(sg_handle h);

/* Number of entries N_xi * N_t * N_x(level) of a vector on multigrid level `level`. */
sg_status sg_vector_length(sg_handle h, int level, long long* n);

/* y = AA x on the finest level (Problem tensor-product-slab-system, left-hand side; Remark
 * solver-matrix-free-sg: only the action is formed).  FP64.  Asynchronous on the stream. */
sg_status sg_operator_apply(sg_handle h, const double* x, double* y, void* hip_stream);

/* y = AA x exactly as sg_operator_apply (same kernels, same result), for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the call allocates nothing and does not use the handle's cell-local workspace; the kernels write
 * their cell-local results to a fixed scratch area of 64 MiB that the library holds on every GPU it
 * runs on until the process ends (resolved once per device by sg_create).  Limit: the problem's
 * N_xi * N_t * n_cells(0) * (k+1)^d doubles of cell-local results must fit those 64 MiB (8,388,608
 * doubles), else SG_EINVAL and nothing is enqueued.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap in time on one GPU (different streams, or different handles) race and must be
 * ordered by the caller.  x, y as for sg_operator_apply.  Asynchronous on the stream. */
sg_status sg_operator_apply_noalloc(sg_handle h, const double* x, double* y, void* hip_stream);

/* `sweeps` additive Vanka sweeps on the mean block I_xi (x) A_0 of level `level`, A_0 =
 * A_t (x) M_x + B_t (x) K_{a_0} (Remark solver-matrix-free-sg), or with desc.diag_blocks = 1 on the
 * block-diagonal operator diag_alpha(A_alpha) with each mode's own patch inverses:
 *     x <- x + omega sum_K R_K^T W_K A_{0,K}^{-1} R_K (b - A_0 x),   then x_D = b_D on Dirichlet DoFs.
 * A_{0,K}^{-1} is the exact patch inverse: on a level whose mean coefficient is one constant it is
 * applied by fast diagonalisation of the patch matrix (a Kronecker product of the cell's restricted 1D
 * mass and stiffness matrices with A_t, B_t: generalised eigenvectors per direction, one N_t x N_t
 * time block per eigen index), otherwise as the dense inverse formed at set-up; the two agree up to
 * rounding (the environment variable SGHEAT_VANKA_FDM=0 selects the dense one everywhere).
 * b and x are FP64 on every level; with SG_MIXED the sweep runs in FP32 internally for level 0 and
 * the levels above the coarsest.  x is updated in place.  Asynchronous on the stream. */
sg_status sg_vanka_smooth(sg_handle h, int level, const double* b, double* x, int sweeps, void* hip_stream);

/* z = one V-cycle for (I_xi (x) A_0) z = r (Remark solver-matrix-free-sg: one geometric-multigrid
 * cycle with the space-time Vanka smoother per stochastic diagonal block, applied matrix-free): the
 * stochastic block-Jacobi preconditioner with the mean-based diagonal block (every diagonal block equals A_0 for an affine coefficient; for a
 * non-affine coefficient set, such as the finite-chaos benchmark's, the diagonal blocks differ and A_0
 * stands in for all of them, so FGMRES needs more iterations but converges to the same solution).
 * With desc.diag_blocks = 1 each mode alpha is cycled with its own block A_alpha instead.
 * FP64 interface; FP32 inside with SG_MIXED.  Asynchronous on the stream. */
sg_status gmg_vcycle(sg_handle h, const double* r, double* z, void* hip_stream);

/* Solve the slab system AA x = b (Problem tensor-product-slab-system) by right-preconditioned
 * flexible GMRES with the block-Jacobi multigrid preconditioner of Remark solver-matrix-free-sg
 * (restart fgmres_restart, preconditioner gmg_vcycle) starting from the x passed in, until
 * ||b - AA x||_2 / ||b||_2 <= rtol (true residual) or max_iter iterations.  The basis is orthogonalised
 * by classical Gram-Schmidt with reorthogonalisation, the second projection of each basis vector delayed
 * into the next step (DCGS2: two passes over the basis per step); the convergence test of a step uses
 * its provisional Hessenberg column.  Synchronises the stream (Krylov scalars go to the host).
 * `info` may be NULL.  Returns SG_NOT_CONVERGED if the tolerance was not reached. */
sg_status fgmres_solve_slab(sg_handle h, const double* b, double* x, double rtol, int max_iter,
                            sg_solve_info* info, void* hip_stream);

/* Physical coordinates of the Gauss points of level `level`, written to the HOST array
 * xyz[n_cells(l)][(k+1)^d][d] (the points at which coef_qp is sampled).  Needs no handle. */
sg_status sg_quadrature_points(const sg_problem_desc* desc, int level, double* xyz);

/* Physical coordinates of the nodes of level `level` in global lexicographic order (x fastest),
 * written to the HOST array xyz[n_nodes(l)][d] (Section 2.4: nodal Q_k basis; the support points are
 * taken as the Gauss-Lobatto points, the paper naming none).  Needs no handle. */
sg_status sg_node_coordinates(const sg_problem_desc* desc, int level, double* xyz);

/* Replace the coefficient values of a handle (same index set, same layout as sg_problem_desc.coef_qp:
 * HOST [n_levels][n_coef_modes][n_cells(l)][(k+1)^d], copied) and redo everything that depends on
 * them: the Vanka patch inverses of every level and the coarsest-level inverse (Remark
 * solver-matrix-free-sg).  Keeps every device allocation of the handle, so a parameter sweep (e.g.
 * the forward/adjoint solves of an optimisation loop) pays no allocation.  Waits for the handle's
 * last asynchronous call, then runs synchronously on the null stream; must not overlap other calls on
 * the handle.  SG_ESINGULAR if a patch or the coarse matrix is singular. */
sg_status sg_update_coefficients(sg_handle h, const double* coef_qp);

/* y = AA^T x for a handle made with transpose = 0 (y = AA x for transpose = 1): the operator of the
 * adjoint slab problem (Problem tensor-product-slab-system with A_t transposed; the other factors of
 * eq. local_rhs_tensor are symmetric).  FP64, finest level, identity rows on Dirichlet DoFs.  x and
 * y are device vectors of sg_vector_length(h, 0) doubles and must not overlap.  Asynchronous. */
sg_status sg_operator_apply_T(sg_handle h, const double* x, double* y, void* hip_stream);

/* Slab transfer (eq. local_rhs_tensor, J = M_xi (x) C_t (x) M_x with [C_t]_ij = v_j(t_{n-1}^-)
 * v_i(t_{n-1}^+), eq. Ct):  y = (I (x) C_t (x) M_x) x  (transpose = 0), the right-hand side that the
 * previous slab's solution x induces on the next slab, or y = (I (x) C_t^T (x) M_x) x (transpose = 1),
 * the same for the backward adjoint sweep.  For the right-Radau basis C_t = v(0) e_r^T: only the
 * last time component of x (the end-of-slab trace) enters.  Rows of Dirichlet DoFs of y are 0 and
 * columns of Dirichlet DoFs are dropped.  With x = the end-of-slab trace of an initial value u_0 in
 * time component r (others 0), y is the initial trace vector B_0 (eq. initial_vector).  Asynchronous. */
sg_status sg_slab_transfer(sg_handle h, int transpose, const double* x, double* y, void* hip_stream);

/* Cell-wise stiffness bilinear form, the building block of the parameter gradient of an adjoint:
 *     out[K] = lam^T (G_mu (x) B_t (x) K_{c|K}) u,   K = 0 .. n_cells(0) - 1 (x fastest),
 * where mu = coef_mu[mu_index] selects the Galerkin tensor, c is the field given by its values at
 * the Gauss points coef_qp[n_cells(0)][(k+1)^d] (HOST array, same layout and points as one mode of
 * the create-time coef_qp on level 0) and K_{c|K} is the stiffness matrix of c restricted to cell K.
 * lam and u are device slab vectors that vanish on Dirichlet DoFs; out is a device array of
 * n_cells(0) doubles.  d/d theta of lam^T AA u for a_mu = theta c is sum_K out[K].  The scaled field
 * stays on the device per mode: only a call whose coef_qp differs from the last one given for that
 * mode uploads it and synchronises the stream.  Asynchronous otherwise. */
sg_status sg_stiffness_form_cells(sg_handle h, int mu_index, const double* coef_qp, const double* lam,
                                  const double* u, double* out, void* hip_stream);

/* The same forms accumulated on the device, for the parameter gradient of an adjoint sweep over many
 * slabs (each slab n contributes lam_n^T (dAA/dtheta) u_n, with no copy to the host per slab):
 *     cells[K] += scale out[K]        (cells: device array of n_cells(0) doubles, may be NULL),
 *     total[0] += scale sum_K out[K]  (total: one device double, may be NULL; the sum over K in one
 *                                      fixed order, so repeated runs agree bitwise),
 * with out[K] as in sg_stiffness_form_cells.  SG_EINVAL if both are NULL.  Same field caching and
 * synchronisation as sg_stiffness_form_cells. */
sg_status sg_stiffness_form_accumulate(sg_handle h, int mu_index, const double* coef_qp, const double* lam,
                                       const double* u, double scale, double* cells, double* total,
                                       void* hip_stream);

/* Mean/variance quantity of interest at the end of a slab.  With u(T) the end-of-slab trace of the
 * slab vector u (time component r) and Q(xi) = int_D u(x, T, xi)^2 dx = sum_{alpha,beta} m_{alpha beta}
 * Psi_alpha Psi_beta, m_{alpha beta} = u_alpha(T)^T M_x u_beta(T), the chaos expansion of Q is
 * q_eps = sum_{alpha,beta} m_{alpha beta} E[Psi_alpha Psi_beta Psi_eps] (|eps| <= 2 p_xi), so
 * E[Q] = q_0 and Var[Q] = sum_{eps != 0} q_eps^2 (Section 3.1, eqs. qoi-mean-chaos and
 * qoi-variance-chaos applied to Q).  Writes qoi[0] = E[Q], qoi[1] = Var[Q] (HOST array of 2) and, if
 * grad != NULL, grad = dJ/du for J = w_mean E[Q] + w_var Var[Q] (a device slab vector, nonzero only in
 * time component r on interior DoFs).  Synchronises the stream. */
sg_status sg_qoi_mean_var(sg_handle h, const double* u, double w_mean, double w_var, double* qoi, double* grad,
                          void* hip_stream);   /* SG_EUNSUPPORTED for sample and member batches */

/* Monte-Carlo estimators over the samples of a handle made with n_samples = N > 1 (Section 5.2, eqs.
 * mc-mean-estimator and mc-variance-estimator-unbiased), per time component and node:
 *     mean[i][node] = (1/N) sum_s u[s][i][node],
 *     var[i][node]  = 1/(N-1) sum_s (u[s][i][node] - mean[i][node])^2.
 * u is a device slab vector of the handle; mean and var are device arrays of N_t * n_nodes(0)
 * doubles (var may be NULL).  Two passes over the samples, FP64.  Asynchronous. */
sg_status sg_sample_statistics(sg_handle h, const double* u, double* mean, double* var, void* hip_stream);

/* Chaos moments of a slab vector (Section 3.1, eqs. qoi-mean-chaos and qoi-variance-chaos): per member j
 * of the handle (one member for a plain SG handle), time component i and node,
 *     mean[j][i][node] = u[first mode of j][i][node],
 *     var[j][i][node]  = sum over the member's other modes alpha of u[alpha][i][node]^2.
 * mean and var are device arrays of n_members * N_t * n_nodes(0) doubles (var may be NULL).
 * SG_EINVAL for a sample-batch handle.  Asynchronous. */
sg_status sg_chaos_moments(sg_handle h, const double* u, double* mean, double* var, void* hip_stream);

/* ---- Prescribed solutions and their forcing (Section 3.2, the finite-chaos benchmark; eqs.
 * load_vector, finite_rhs_factorized, and the error quantities of Definition
 * def:error-norms-and-quantities).  These let a caller march a slab sequence with a forcing term
 * F^(n) and measure the error against a separable exact solution u = theta(t) s(x) sum_a c_a Psi_a. */

/* Physical points of the nq1-point Gauss rule per direction on every cell of a level,
 * [n_cells][nq1^d][d] (cells and points lexicographic, x fastest).  Host only. */
sg_status sg_gauss_points(const sg_problem_desc* desc, int level, int nq1, double* xyz);

/* The handle's chaos index set, alpha[N_xi][n_vars], in the order of the modes of a slab vector
 * (total degree, graded).  Single stochastic Galerkin handles only.  Host only. */
sg_status sg_index_set(sg_handle h, int* alpha);

/* Galerkin projection weights of the product of the coefficient modes with a given chaos expansion
 * (eq. triple_stoch): out[mu][beta] = sum_s src_c[s] E[Psi_mu Psi_{src_alpha[s]} Psi_beta] for the
 * handle's coefficient modes mu and modes beta.  With src = the exact solution's chaos coefficients,
 * sum_mu out[mu][beta] a_mu is E[a G Psi_beta], the factor of the projected forcing f_beta.  Host only. */
sg_status sg_chaos_projection(sg_handle h, int n_src, const int* src_alpha, const double* src_c, double* out);

/* The ntq-point Gauss rule of one slab: reference points s[k] in (0, 1) and weights w[k] (times tau).
 * Host only. */
sg_status sg_time_rule(sg_handle h, int ntq, double* s, double* w);

/* Time loads of n_g functions g given at that rule's points of a slab: out[g][i] = int_{I_n} g v_i dt
 * (v_i the right-Radau nodal basis), gvals [n_g][ntq].  Host only. */
sg_status sg_time_load_weights(sg_handle h, int ntq, int n_g, const double* gvals, double* out);

/* Spatial load vectors on the finest level: out[f][j] = sum_K sum_q w_q |K| (fval[f][K][q] psi_j(x_q)
 * + sum_e fgrad[f][K][q][e] d_e psi_j(x_q)) at the nq1-point Gauss rule (points as sg_gauss_points),
 * Dirichlet entries 0.  fval [n_fields][n_cells][nq1^d] and fgrad [n_fields][n_cells][nq1^d][d] are device
 * arrays (either may be NULL), out a device array [n_fields][n_nodes(0)].  Asynchronous. */
sg_status sg_load_vectors(sg_handle h, int nq1, int n_fields, const double* fval, const double* fgrad, double* out,
                          void* hip_stream);

/* Separable slab vector: y[alpha][i][node] = beta * y + sum_t W[t][alpha][i] V[t][node] (a load vector
 * F^(n) = sum_t (chaos x time weights) (x) spatial load).  W host [n_terms][N_xi][N_t] (copied; the call
 * waits for the stream first), V device [n_terms][n_nodes(0)], y a device slab vector. */
sg_status sg_separable_vector(sg_handle h, int n_terms, const double* W, const double* V, double beta, double* y,
                              void* hip_stream);

/* Error sums of one slab vector u against u_ex = theta(t) s(x) sum_a c[a] Psi_a on that slab, by the
 * nq1-point Gauss rule per space direction and the ntq-point rule in time (sg_time_rule):
 *   out[0] = sum_a |c_a theta s - u_a|^2,  out[1] = the same for the gradients,
 *   out[2], out[3] = the a = 0 terms alone (mean error),
 *   out[4] = |C2 theta^2 s^2 - sum_{a != 0} u_a^2|^2, out[5] = the same for the gradients (variance error),
 *   out[6] = |theta s|^2, out[7] = |theta grad s|^2,
 * each integrated over the slab and D.  s_qp [n_cells][nq1^d], gs_qp [n_cells][nq1^d][d] are device
 * arrays; theta [ntq] and c [N_xi] host arrays; C2 = sum of c^2 over the exact solution's nonzero modes.
 * Single SG handles; 2D k <= 4 or 3D k <= 2.  Synchronous. */
sg_status sg_separable_error(sg_handle h, const double* u, int nq1, const double* s_qp, const double* gs_qp, int ntq,
                             const double* theta, const double* c, double C2, double* out, void* hip_stream);

/* ---- Monte-Carlo estimators at quadrature points and their error split (Section 5.2-5.4, eqs.
 * mc-mean-estimator, mc-variance-estimator-unbiased, mc-error-mean-L2,mc-error-var-L2, mc-disc-mean-error,
 * mc-disc-var-error).  The estimators are formed pointwise at the space-time quadrature points from
 * running sums over the samples, so several sample-batch handles (on the same mesh) can feed one
 * estimate. */

/* Psi_alpha(xi^(s)) for the handle's samples and the given multi-indices: out[s][j], alpha [n_idx][n_vars].
 * Sample-batch handles only.  Host only. */
sg_status sg_sample_psi(sg_handle h, int n_idx, const int* alpha, double* out);

/* acc[cell][q][k][0] += sum_s u_s(x_q, t_k), acc[cell][q][k][1] += sum_s u_s(x_q, t_k)^2 over the samples of
 * the sample-batch slab vector u, at the nq1-point Gauss rule per space direction (points as
 * sg_gauss_points) and the ntq-point time rule (sg_time_rule).  acc is a caller-owned device array of
 * n_cells * nq1^d * ntq * 2 doubles, zeroed by the caller.  Asynchronous. */
sg_status sg_sample_qp_moments(sg_handle h, const double* u, int nq1, int ntq, double* acc, void* hip_stream);

/* From such sums over n_tot >= 2 samples: mean M = S1/n_tot and unbiased variance V = (S2 - n_tot M^2)/(n_tot - 1)
 * at every quadrature point, and over the slab and D
 *   out[0], out[1] = int |M - mean_targets[j] theta s|^2,   out[2], out[3] = int |V - var_targets[j] theta^2 s^2|^2,
 *   out[4] = int |theta s|^2,  out[5] = int |theta s|^4,
 * for a separable reference theta(t) s(x) (s_qp device [n_cells][nq1^d], theta host [ntq]).  Synchronous. */
sg_status sg_moment_errors(sg_handle h, const double* acc, long long n_tot, int nq1, const double* s_qp, int ntq,
                           const double* theta, const double* mean_targets, const double* var_targets, double* out,
                           void* hip_stream);

/* Run the lower part of every V-cycle (the levels from the first one of at most 512 cells below the
 * finest, down to the coarsest: pre-smoothing, residuals, restrictions, the coarsest solve,
 * prolongations, post-smoothing) as one persistent launch with one workgroup per stochastic mode
 * (enable = 1), or kernel by kernel (enable = 0, the default; sg_autotune times both and keeps the
 * faster).  Both compute the block-Jacobi cycle of Remark solver-matrix-free-sg with the mean block;
 * they differ only in rounding order.  Waits for the handle's last asynchronous call and drops a
 * captured V-cycle graph.
 * enable = -1 changes nothing (a query).  first_level (host pointer, may be NULL) receives the first
 * level the segment covers (for enable = -1: -1 while the cycle runs kernel by kernel); -1 when the
 * hierarchy has no such levels or uses one diagonal block per mode (then every setting runs kernel by
 * kernel). */
sg_status sg_set_vcycle_segment(sg_handle h, int enable, int* first_level);

/* Replay the V-cycle (gmg_vcycle, and the preconditioner inside fgmres_solve_slab) from a HIP graph
 * (enable = 1) or launch it kernel by kernel (0, the default).  With the graph, each V-cycle copies r
 * into the handle's level-0 work vector, replays the captured cycle and copies the result to z; the
 * graph is captured on the second V-cycle after enabling (the first runs kernel by kernel) on a stream
 * of the handle's own, and dropped by sg_update_coefficients, sg_autotune and enable = 0.  Results are
 * bitwise those of the kernel-by-kernel cycle.  It pays for small problems, where launching the tens
 * of kernels of a cycle costs more than running them.  enable = 0 waits for the handle's last
 * asynchronous call before dropping the graph; enable = 1 is host only. */
sg_status sg_set_vcycle_graph(sg_handle h, int enable);

/* Tile autotuner of the operator kernel: for the full operator on level 0 and the mean-block operator
 * on every level (and their FP32 versions with SG_MIXED), times `reps` launches of the cell kernel and
 * its node gather for
 * every feasible number of cells per workgroup (1, 2, 3, 4, 5, 6, 8, 10, 12, 16; limited by 512 threads
 * and 160 KB of LDS per workgroup) on this handle's own sizes and keeps the fastest (median) for all
 * later calls.  Without it the number comes from the runtime occupancy calculator.  The
 * SGHEAT_APPLY_CPB environment variable, if set, overrides both.  cpb_out (may be NULL) receives
 * [2 (FP64, FP32)][2 (mean, full)][n_levels] choices (0 = not tuned).  Where the hierarchy has a coarse
 * segment (sg_set_vcycle_segment), it then times `reps` V-cycles with the segment as one launch and
 * kernel by kernel and keeps the faster.  Synchronous; uses the handle's level work vectors, so no
 * other call on the handle may run meanwhile. */
sg_status sg_autotune(sg_handle h, int reps, int* cpb_out, void* hip_stream);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SGHEAT_H */
