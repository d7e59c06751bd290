"""FP64 CPU oracle for the sparsifying-preconditioned Lippmann-Schwinger solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg may import this package.  The GPU library
never calls it and shares no code with it.

Every function is a plain, slow, obviously-correct restatement of the method
in "Sparsifying Preconditioner for the Lippmann-Schwinger Equation"
(L. Ying, 2014), numpy/scipy only, complex128 throughout:

  greens   -- free-space Green's function (Section 1), kernel table k_t
              (Section 2.1) and the self-term k_0 (reading: cell integral)
  operator -- the discrete operator I + K w^2 m (eq:lso): dense K, direct
              O(N^2) summation, FFT circulant embedding; RHS g
  stencil  -- the 3^d stencil classes and their null vectors (Section 3.1,
              eq:Fmin / eq:Emin / eq:Cmin and the 3D sets), C = A K(mu,mu)
  sparse   -- Q = [A; B] and M = [A + C w^2 m; B] (eq:PC, eq:ABop), sparse LU
  gmres    -- restarted right-preconditioned GMRES (Section 3.3 experiments)
  solve    -- the pipeline: setup, factor, solve

Readings of passages the paper leaves open are stated where they are used.
"""
