"""Plain FP64 CPU oracle for the stochastic-Galerkin space-time slab operator and its solver.

TEST INFRASTRUCTURE ONLY.  This package is the reference the HIP path is checked against.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import it; the product path
(``paper_2605_21046_amd``) never does, and this package imports nothing from it.

Everything here follows the paper's definitions directly (explicit element assembly, sparse and
Kronecker products, dense LU, textbook GMRES).  No sum factorisation, no fusion, no blocking.

Modules
  chaos      -- total-degree Hermite index set and triple-product tensors (Section 2.6, eq. triple_stoch)
  timebasis  -- right Gauss-Radau dG(r) time matrices A_t, B_t, C_t (eqs. At, Bt, Ct)
  fem        -- Q_k Lagrange elements on a uniform Cartesian mesh; sparse M_x and K_mu (Section 2.4)
  slab       -- the slab operator (Problem tensor-product-slab-system), two independent routes
  multigrid  -- Vanka patch smoother, transfers, V-cycle, coarse LU (Remark solver-matrix-free-sg)
  krylov     -- flexible GMRES with CGS2 and restart (Remark solver-matrix-free-sg)
"""
