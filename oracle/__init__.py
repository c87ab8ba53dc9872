"""CPU FP64 oracle for the adaptive Hessian-sketch ridge solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the paper (Lacotte & Pilanci, "Effective Dimension Adaptive
Sketching Methods for Faster Regularized Least-Squares Optimization", NeurIPS
2020) computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
routes through it, and it shares no code with the GPU library.

Modules
-------
philox  : Philox4x32-10 counter-based generator (Salmon et al., SC'11), the
          stream map used to draw the sketches' randomness, and the CountSketch
          hash.
sketch  : SRHT (dense Walsh-Hadamard, no fast transform), Gaussian embeddings
          (Section 1; Appendix C.2 "SRHT matrices") and the CountSketch for
          sparse A.
ridge   : the problem (eq. (1)), its direct solution, gradient (dense, dual and
          sparse), error metric and effective dimension (Section 1.1
          "Notations").
ihs     : algorithmic parameters (Theorems 1-2, Definitions 3.1-3.2), the
          sketched Hessian and its Woodbury inverse (proof of Theorem 7), the
          sketched Newton decrement (Lemma 1), Algorithm 1, the regularization
          path with warm starts, the dual and sparse solves and the IHS with
          refreshed embeddings.
lowprec : BF16 rounding and the FP8-E4M3 encoder with per-column power-of-two
          scales (the low-precision sketch form).
certify : an upper bound on delta(x)/delta(0) from one FP64 pass over the rows of
          A (Nystrom approximation of A^T A below H, and the dual bound on
          delta(0)), for problems too large for the FP64 Gram.
learned : features and the FP64 reference of the small MLP of the learned
          starting-m form, its gradient and Adam step.

Parity status: every function is pinned by a ``-m "not gpu"`` test except those
whose docstring says "parity unpinned".
"""
