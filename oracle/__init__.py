"""Plain FP64 CPU oracle for the spectral-element Poisson hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.

Each module restates one part of arXiv:2110.07663 ("Tuning Spectral Element
Preconditioners for Parallel Scalability on GPUs") in the slowest, most
readable form: NumPy float64, vectorised over elements only where that keeps
the formula visible.

Module map (paper passage each one follows):
  gll       GLL nodes/weights, cardinal-basis derivative and interpolation
            matrices (Sec. 2.1, isoparametric mapping and GLL quadrature).
  mesh      structured hex numbering, Boolean gather Q, Dirichlet mask,
            multiplicity (Sec. 2.1, u_L = Q u).
  geom      isoparametric Jacobian, geometric factors G, diagonal mass B_L
            (Sec. 2.1, eqs. 2-3).
  operator  A_L by sum factorisation, A = Q^T A_L Q, right-hand side B f,
            Jacobi diagonal (Sec. 2.1 eq. 3; Sec. 2.2.3 Jacobi surrogate).
  fdm       box approximation, separable extended-box operator, generalised
            eigenproblems, FDM inverse, ASM/RAS weights (Sec. 2.2.2, eqs. 4-9).
  cheby     Chebyshev smoother and Arnoldi spectral proxy (Sec. 2.2.3,
            Algorithm 2).
  mg        p-multigrid transfers and the single-pass V-cycle
            (Sec. 2.2.2, Algorithm 1).
  krylov    PCG, flexible CG and flexible GMRES (Sec. 2.2).
  rng       SplitMix64 counter-based generator (Steele, Lea, Flood 2014),
            used for the Arnoldi start vector.
  hierarchy convenience wrapper assembling the above into a solver.

The V-cycle output for a real (p, p_c, ..., 1) schedule has no closed form;
it is pinned through its special cases (schedule (p, p) is the exact solve,
two-level contraction), its matrix composition from the separately pinned
smoother, transfers and dense coarse solve (the multiplicative cycle of
Algorithm 1 and the additive cycle of the unaccelerated smoothers), and the
final solve.
"""
