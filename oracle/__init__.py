"""Plain FP64 CPU oracle for the block Krylov-Schur (BKS) method of Elden and
Dehghan for the best rank-(r, r, r3) approximation of (1,2)-symmetric tensors.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference the HIP library is checked against.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the library's
product path never does.  It shares no code with the HIP path.

Modules
  sptensor : stored-entry representation, densification, norms
  ttmc     : the three tensor-times-block contractions (section "Multilinear tensor-matrix multiplication")
  orth     : order-preserving Gram-Schmidt with reorthogonalisation and
             deflation (Algorithm 3 steps (ii)-(iv), Appendix B)
  bk       : block-Krylov schedules (Tables 1-3) and the basis builder
  core     : dense projected problem: HOSVD, HOOI and Newton-Grassmann
             (Algorithm 5 step (i), section "Experiments")
  bks      : tensor Krylov-Schur driver, gradient and S-values
             (Algorithm 5, Proposition 3.2, section "Conditioning of the best approximation problem")
  hooi     : sparse HOOI (section "Higher Order Orthogonal Iteration")
"""
