"""FP64 CPU oracle for the Positively Split Ewald (PSE) Brownian sampler.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of what the PSE method computes (Fiore, Balboa Usabiaga, Donev,
Swan, "Rapid Sampling of Stochastic Displacements in Brownian Dynamics
Simulations", arXiv:1611.09322).  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  It shares no code with the
HIP library; the product path never calls it.

Modules
  rpy      real-space scalar functions F, G (Appendix A), the free-space RPY
           tensor (eq. RPY_free_space), the H-weighted wave integrals that
           complete them (eqs. int1/int2), and the dense real-space block M_r.
  ewald    wave-space objects: the k-set, the split kernel B(k) (eq. Mwave),
           the dense wave block M_w, direct non-uniform Fourier sums for the
           wave-space sample and for M_w F.
  philox   Philox-4x64-10 counter-based generator (Salmon et al., SC'11) and
           the Box-Muller normals and Hermitian k-space noise built from it.
  lanczos  Krylov square-root iterate (Chow-Saad) with full
           re-orthogonalisation, and the eigendecomposition square root.
  precond  the learned block preconditioner of the Krylov sample: geometry
           features, the bf16 MLP, the per-particle fallback, the
           preconditioned root P^-1 (P M_r P^T)^1/2 z and the training target.
  sampler  the composed sample Delta x = sqrt(2 kT dt)(y_r + y_w) + dt M F
           (eqs. langevin, split) and the truncation-error bounds.

Every function states the passage of the paper it restates.  Functions whose
result is not pinned by an independent check say "parity unpinned".
"""
