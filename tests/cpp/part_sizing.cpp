// Checks the partial-sum workspace rules of the Krylov multi-dot kernels
// (paper_1512_04506_amd/csrc/blas_sizes.h) against the largest call each
// buffer serves, for the lattice shapes of the three workloads and short
// coarse restarts.  Prints one line per case; exit status 1 on a failure.
#include <algorithm>
#include <cstdio>

#include "blas_sizes.h"

using namespace ddamg;

static int fails = 0;

static void check(const char* what, const char* shape, int m, size_t cap, size_t need) {
  const bool ok = need <= cap;
  std::printf("%-5s restart %2d  %-22s need %8zu  cap %8zu  %s\n", shape, m, what, need, cap, ok ? "ok" : "FAIL");
  if (!ok) ++fails;
}

int main() {
  struct Shape {
    const char* name;
    int L[4], b[4], ntv, max_rhs;
  } shapes[] = {
      {"c1", {4, 4, 4, 4}, {2, 2, 2, 2}, 8, 1},
      {"c2", {16, 16, 16, 16}, {4, 4, 4, 4}, 20, 8},
      {"c3", {32, 32, 32, 64}, {4, 4, 4, 4}, 24, 12},
      {"16^3x32", {16, 16, 16, 32}, {4, 4, 4, 4}, 24, 12},
  };
  const int coarse_restarts[] = {1, 5, 30, 64};
  const int outer_restarts[] = {1, 20, 64};
  const int fused_max = 24;  // widest fused second Gram-Schmidt pass
  int old_rule_overflows = 0;
  for (const Shape& s : shapes) {
    size_t V = 1, vb = 1;
    for (int mu = 0; mu < 4; ++mu) {
      V *= s.L[mu];
      vb *= s.b[mu];
    }
    const size_t nblocks = V / vb, nc = 2 * (size_t)s.ntv;
    const size_t fsz = 12 * V, csz = nblocks * nc, osz = (nblocks / 2) * nc;
    const int maxr = std::max(s.max_rhs, s.ntv);
    for (int mc : coarse_restarts) {
      // coarse GMRES: |y_c|, |r| and Gram-Schmidt against up to mc vectors
      const size_t cap = krylov_part_entries(mc, maxr, std::max(osz, csz));
      check("coarse |y_c|", s.name, mc, cap, mdot_part_entries(csz, 1, maxr));
      check("coarse Gram-Schmidt", s.name, mc, cap, mdot_part_entries(osz, mc, maxr));
      // the setup's test-vector norms have their own buffer
      check("setup norms", s.name, mc, setup_norm_part_entries(s.ntv, fsz), mdot_part_entries(fsz, 1, s.ntv));
      // before the fix they shared the coarse buffer
      if (mdot_part_entries(fsz, 1, s.ntv) > cap) ++old_rule_overflows;
    }
    for (int m : outer_restarts) {
      const int nrhs = s.max_rhs;
      const size_t cap = krylov_part_entries(m, nrhs, fsz);
      check("outer first pass", s.name, m, cap, mdot_part_entries(fsz, m, nrhs));
      check("outer fused pass", s.name, m, cap, mdot_part_entries(fsz, std::min(m, fused_max) + 1, nrhs));
      check("outer unfused pass", s.name, m, cap, mdot_part_entries(fsz, m + 1, nrhs));
    }
  }
  // the shared buffer overflowed on c2 and on 16^3x32 (and on c3 at short
  // restarts): the check has teeth
  std::printf("shapes x restarts where a shared coarse buffer would overflow: %d\n", old_rule_overflows);
  if (old_rule_overflows == 0) ++fails;
  return fails ? 1 : 0;
}
