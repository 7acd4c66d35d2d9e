"""Plain FP64 CPU oracle for the parity-projected matrix-P hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything here; the product library
never does, and it shares no code, tables or constants with this package.

Contents (each function cites the passage of the paper it follows):
  philox     counter-based Philox4x64-10 generator (Salmon et al., SC'11),
             written from the published round definition
  sampler    Box-Muller normals and the real (alpha, beta) phase-space
             amplitudes of squeezed inputs (main text, squeezed-state
             integral and its parity-projected +P sampling)
  estimator  propagation alpha' = T alpha, beta' = T* beta, bin occupations,
             and the per-sample c-number observable G(m) evaluated directly
             in count space (eq. c-number-variable), averaged over
             sub-ensembles with the sigma_T error estimate (Appendix A)
  exact      exact references the estimator converges to: the lossless
             uniform-squeezing law (eq. Exact_multi_mode_squeezed_state),
             the uniform-loss and general Gaussian generating functions,
             closed-form count moments, the Appendix-B count cutoffs
  fock       brute-force Fock-space probabilities for M <= 4 modes

Parity status: every function above is pinned by tests marked "not gpu"
(closed forms, brute force, a library generator, printed values of the paper).
"""
