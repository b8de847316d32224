"""CPU oracle for the interior-point Hessian-equation solve (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import, call or execute anything in this package.  The product (the HIP library
and its Python binding) never touches it, and it shares no code with them.

Modules, each citing the passage of the paper it follows:
  hessian  plain definitions of H = A^T (W kron W) A (eqs hesseqn2, hesseqn1),
           explicit H, SPD check, dense Cholesky solve (Section 2.1)
  alg1     Algorithm 1 (Section 3.3): formation, factorization, SMW preconditioner,
           PCG (Barrett et al. templates)
  dd       double-double arithmetic and the true relative residual ||r - H y|| / ||r||
  refine   split H v (eq hessExp1), double-double SMW pieces (Section 4's warning),
           outer iterative refinement
  mp       exact (50-digit) solves of tiny instances with mpmath
  ipm      a tiny primal-dual path-following interior-point method (Section 2,
           NT scaling) on the bipartite matrix-completion SDP (eq matcomp_sdp)

Every function here is pinned by a `-m "not gpu"` test against something other
than itself (closed forms, lemmas, special cases, brute force, exact arithmetic);
see tests/test_oracle_*.py.  Parity unpinned: agreement with the paper's own
solver (SeDuMi with the modified preconditioner) and its figures, which are not
available.
"""
