"""Plain FP64 CPU oracle for the two-grid deflated Krylov method
(Morgan, Whyte, Wilcox, Yang, "Two-grid deflated Krylov methods for linear
equations", arXiv 2005.03070).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke entry
point and the CPU-baseline leg of the benchmark may import it. The product
path (the HIP library and its Python binding) never calls into it and shares
no code with it; the only thing both sides use is the seeded input generator
module ``workloads``.

Everything here is slow and written to be checked against the paper by eye:
numpy arrays in float64, library primitives (dense solve, QR, eig, lstsq)
used as single steps, no blocking and no fusion.

Modules and the part of the paper each follows:

* ``operators``  -- discretised PDE operators ``A`` (Sec. 3, Example 1 and
  Example 3 operator; constant-coefficient 2-D/3-D convection-diffusion;
  variable-coefficient diffusion in divergence form).
* ``transfer``   -- coarse-to-fine prolongation and fine-to-coarse restriction
  (Sec. 3 "moved to the fine grid with ... prolongation").
* ``projection`` -- Galerkin projection over approximate eigenvectors
  (Sec. 2.2, projection box, steps 0-4).
* ``bicgstab``   -- BiCGStab(ncyc)-Proj(k) with the per-cycle tolerance
  (Sec. 4.1 algorithm box, step 3 a-d).
* ``gmres``      -- GMRES(m)-Proj(k) (Sec. 2.2 algorithm box).
* ``idr``        -- IDR(s)(ncyc)-Proj(k): the Sec. 4.1 box with IDR(s) (the
  biorthogonal variant of van Gijzen and Sonneveld) as the inner solver.
* ``gmresdr``    -- GMRES-DR(m,k) on the coarse grid (Sec. 2.1; phase 1 of
  the Sec. 3 algorithm).
* ``deflation``  -- the fine-grid deflation space built from moved vectors
  (Sec. 2.2 step 1-2, Sec. 3 phase 1).
* ``adjoint``    -- gradient of a least-squares loss through a solve, by an
  adjoint solve with ``A^T`` (extension of the method; not in the paper).
* ``direct``     -- ``x = A^{-1} b`` by a sparse LU factorisation (the plain
  definition every solve converges to; pins full-size solutions).

Functions whose result has no independent pin are marked "parity unpinned"
in their docstring.
"""
