"""FP64 CPU oracle for the masked pressure-correction Poisson solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or run anything in this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it.

Contents, each following the paper (arXiv:1810.08572) or, where the paper is
silent, the stated reading:
  assembly     - active set, open/blocked faces, components and pins, the
                 pinned pressure matrix (section 2.4.2, Eq. 9, Eq. 11)
  direct       - exact references: dense Cholesky and sparse LU solves
  closed_form  - DCT solution of the Neumann box problem
  hash         - the 32-bit MurmurHash3 finaliser used for MIS-2 priorities
  amg          - smoothed-aggregation AMG: strength, MIS-2, aggregates,
                 tentative and smoothed prolongators, Galerkin coarse
                 operators, Chebyshev smoother, V-cycle (section 2.5)
  pcg          - preconditioned conjugate gradients (section 2.5)
  mlp          - the warm-start network's forward and backward pass
  projection   - the pressure-correction step with cross diffusion, the
                 smeared face gradients and the flux and velocity correction
                 (section 2.3-2.4, Eq. 11-17)
  uq           - polynomial chaos by stochastic collocation (section 3)
  flow         - one fractional step: momentum predictor, projection,
                 energy with the latent-heat Picard loop (section 2.2, Eq.
                 2-9, 18-21)

Nothing here is blocked, fused or reordered beyond what each definition
states, so every function can be checked against its definition by eye.
"""
