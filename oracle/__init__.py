"""Plain FP64 CPU reference for Erb, "Krylov subspace methods to accelerate
kernel machines on graphs" (arXiv 2301.06384).

TEST INFRASTRUCTURE ONLY.  This package is the parity oracle: slow, plain
numpy/scipy code that follows the paper's definitions and algorithms step by
step in float64.  It shares no code with the GPU library and must never be
called by the product path.  Only the test-suite, the smoke check of the
graft entry point and the CPU-baseline leg of the benchmark may import it.

Modules
  phi     -- the kernel functions phi of Sec. 2.4 (diffusion, variational
             spline) and a polynomial phi used for exactness checks.
  dense   -- exact kernel columns phi(L) E_W through the full spectral
             decomposition of L (Sec. 3, the naive two-step approach), and
             the exact RLS kernel machine of Sec. 2.3.
  krylov  -- classical block Lanczos (Alg. 1), global block Lanczos (Alg. 2),
             sequential Lanczos (Sec. 3.3) and the RLS predictor (Alg. 3).
  cheb    -- Chebyshev interpolation and squared Chebyshev (Sec. 3.4).
  bounds  -- error bounds of Sec. 4 (Theorem 4.2, Example 3) used as pins.

Parity status: every function here is pinned by a test in tests/ against a
closed form, an invariant, a textbook special case or brute force, except
where its docstring says "parity unpinned".
"""
