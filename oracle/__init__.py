"""Plain FP64 CPU oracle for the SEM / H-matrix fractional diffusion solver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the C-ABI library and
its Python binding) imports, calls, links or executes anything in this
package; only the tests, the package smoke check and the benchmark's
CPU-baseline leg do. It shares no code with the HIP implementation.

Each module follows the paper's definitions in its own notation:
  quadrature  -- Gauss-Legendre / Gauss-Jacobi rules (library routines)
  sem         -- basis, DOF order, element-pair moments, dense A, M, G (Section 2)
  toeplitz    -- FFT block-Toeplitz apply on uniform / geometric meshes (Section 4.3)
  hmatrix     -- cluster/block trees, Taylor low-rank factors, H-LU, H-solves
                 (Sections 3 and 4.1)
  krylov      -- dense LU, preconditioned FGMRES and BiCGSTAB (Section 4.2)

Parity status of each function is stated in its docstring; every function
listed here is pinned by a test in tests/test_oracle_*.py unless it says
"parity unpinned".
"""
