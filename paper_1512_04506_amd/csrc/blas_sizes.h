// Sizes of the partial-sum workspace that the Krylov multi-dot kernels
// (k_blas.hip) write: one partial per (rhs, vector, chunk of the vector).
// Plain host arithmetic without HIP, shared by the launchers (which refuse
// to launch into a buffer that is too small), the allocation of every such
// buffer, and a CPU test of the allocation rules.
#pragma once
#include <cstddef>

namespace ddamg {

// workgroups per rhs (chunks) of a multi-dot over n elements per rhs
inline int blas_nchunks(size_t n) {
  size_t c = (n + 8191) / 8192;
  if (c < 1) c = 1;
  if (c > 512) c = 512;
  return (int)c;
}

// partial sums written by a multi-dot of nvec vectors over n elements per
// rhs for nrhs rhs (the fused second Gram-Schmidt pass over nvec vectors
// writes nvec + 1 of them per rhs and chunk: the extra one is |w|^2)
inline size_t mdot_part_entries(size_t n, int nvec, int nrhs) {
  return (size_t)(nrhs > 0 ? nrhs : 0) * (size_t)(nvec > 0 ? nvec : 0) * (size_t)blas_nchunks(n);
}

// Krylov workspace of GMRES(m) on vectors of n elements per rhs: the
// widest multi-dot is the Gram-Schmidt of a new vector against all m + 1
// basis vectors of a cycle
inline size_t krylov_part_entries(int m, int nrhs, size_t n) { return mdot_part_entries(n, m + 1, nrhs); }

// normalisation of the ntv fine test vectors of the setup (one norm per
// vector over 12 V elements)
inline size_t setup_norm_part_entries(int ntv, size_t fine_elems) { return mdot_part_entries(fine_elems, 1, ntv); }

}  // namespace ddamg
