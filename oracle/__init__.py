"""FP64 CPU oracle for Chebyshev-polynomial-approximation (CPA) singular value
shrinkage (Onuki, Ono, Shirai, Tanaka, "Fast Singular Value Shrinkage with
Chebyshev Polynomial Approximation Based on Signal Sparsity").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants); the only common
dependency is the ``synth`` input generators, which hold none of the method's
arithmetic.

Everything here is plain numpy in float64, written to be checked against the
paper by eye: no blocking, fusion or reordering beyond what the paper's
definitions and Algorithm 1 state.  Library primitives used as steps: matrix
product (``@``), ``numpy.linalg.svd`` and ``numpy.linalg.eigh`` (only for the
exact shrinkage definitions and the spectral cross-check form).

Modules
  chebyshev  - scalar Chebyshev machinery (Sec. II-B, Sec. III-A)
  shrinkage  - the generic shrinkage response family (Sec. IV-A)
  cpa        - Algorithm 1 (Sec. III-B) with T = Id and no truncation, plus
               equivalent evaluation orders used only as cross-checks
  bound      - spectral bound on the Gram (Algorithm 1, step computing the
               maximum eigenvalue) by power iteration
  exact      - exact singular value shrinkage by SVD and by EVD (Sec. III-B,
               Sec. V-A)
  drivers    - ADMM background modelling (Appendix B) and SVT completion
  mlp        - FP64 reference for the spectral-bound/order predictor network
  metrics    - relative Frobenius error and RMSE (Sec. V-A)

Parity status per function is listed in each module header.
"""
