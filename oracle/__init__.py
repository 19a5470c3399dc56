"""FP64 CPU oracle for the two-level DD-alpha-AMG hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library
never calls it and shares no code with it.

It is a plain, slow, numpy implementation of what the method computes,
written from the paper (Heybrock, Rottmann, Georg, Wettig, "Adaptive
algebraic multigrid on SIMD architectures", arXiv:1512.04506):

  dirac   -- Wilson-clover operator D, clover term, block operator B
             (Sec. 2, splitting D = B + Z of Alg. 3; hopping structure of Alg. 7)
  sap     -- minimal-residual block solver and the multiplicative Schwarz
             smoother (Alg. 3, SAP reading)
  coarse  -- aggregates, Gram-Schmidt, restriction R and prolongation
             P = R^dagger (Eq. R, Alg. 5, Alg. 6), Galerkin coarse operator
             D_c = R D P (Eq. cgo), coarse stencil apply, even/odd
             preconditioned coarse GMRES (Alg. 2)
  mg      -- V-cycle (Alg. 1), setup (Alg. 4), outer flexible GMRES and
             the FP64 residual check (Sec. 1)

Every array is complex128 in the canonical layouts of `synth.py`.
Parity pins live in tests/test_oracle_*.py; a function that has none says
"parity unpinned" in its docstring.
"""
from . import dirac, sap, coarse, mg  # noqa: F401
