"""Plain FP64 CPU oracle for KP-SVD-preconditioned Tikhonov deblurring.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or
links this package; only the tests, __graft_entry__.smoke() and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library.

It follows Chen, Ji & Nagy, "Half-Precision Kronecker Product SVD
Preconditioner for Structured Inverse Problems" (arXiv:2311.15393):

  operator.py  the blurring matrix A and its transpose (zero boundary, true
               convolution), direct and FFT forms, dense A for tiny images
  kp.py        the one-term Kronecker approximation A ~ A_r (x) A_c (Section 3,
               eq. (KronSumDecomp)), the factor SVDs (eq. (AKronSVD)) and the
               preconditioner solve Z = V_c (S .* (V_c^T R V_r)) V_r^T
               (eq. (PreconSolve))
  solvers.py   CG, PCG (Fletcher-Reeves) and flexible PCG (Polak-Ribiere) on
               the normal equations (A^T A + lambda^2 I) x = A^T b
               (eq. (tik:normal2)), plus the exact Tikhonov minimiser x_lambda
  lam.py       lambda_opt, GCV, weighted GCV and the discrepancy principle in
               a spectral basis (eqs. (OptTikSVD), (GCVTikSVD), (wGCVTikSVD),
               (DSCTikSVD)), and the trace form of GCV (eq. (GCVTik))
  periodic.py  the periodic boundary: block-circulant A and A^T, the
               circulant one-term Kronecker approximation, and the exact
               Tikhonov minimiser through the 2-D DFT
  reflexive.py the reflexive boundary for PSFs symmetric in both axes
               (A = A^T, Toeplitz-plus-Hankel factors) and the exact
               Tikhonov minimiser through the 2-D DCT
  quant.py     FP16 and FP8-e4m3 rounding and the emulated reduced-precision
               preconditioner chain
  mlp.py       FP64 reference of the small lambda-predicting network

Parity status of each function is stated in its module header.
"""
