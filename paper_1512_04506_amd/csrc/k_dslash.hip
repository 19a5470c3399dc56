// Wilson-clover operator on site-major structure-of-arrays fields.
//
//   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
//                                         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// (Sec. 1; the hop/clover structure is the one Alg. 7 applies to the columns
// of P).  One thread per (site, rhs): consecutive lanes own consecutive
// sites, so every load of a spinor component, link entry or clover entry is
// a coalesced 64-lane access.  The spin projectors (1 -+ g_mu) reduce each
// hop to a 2-spinor (6 complex) before the SU(3) multiply.  In the chiral
// basis g_mu = [[0, X_mu], [X_mu^dag, 0]] with X_k = -i s_k and X_4 = -1:
//   (1 - g) psi = (h, -X^dag h),  h = psi_up - X psi_dn
//   (1 + g) psi = (h,  X^dag h),  h = psi_up + X psi_dn
// Variants: the full operator, the block operator B (hops leaving the block
// dropped, Alg. 3), and the block-crossing forward/backward hops of one
// direction (the pieces D_ij of Eq. cgo for a neighbour block j).
// Workgroups walk the blocks in lexicographic order (through the XCD
// swizzle), so face neighbours are processed at the same time on the same
// XCD although blocks of opposite parity are far apart in memory.
#include "dirac_device.h"

namespace ddamg {

namespace {

constexpr int TPB = 256;
using namespace dev;

template <typename Tin, typename Tout, typename S, typename Tc, int MODE>
__global__ __launch_bounds__(TPB) void dslash_kernel(cx<Tout>* __restrict__ out, const cx<Tin>* __restrict__ in,
                                                     GaugeView<S> gv, Geom g, int mu_sel, int chi_in, size_t in_rs,
                                                     size_t out_rs, int nrhs) {
  // workgroup = (run of 256 sites, rhs) with the rhs fastest, so the
  // workgroups that read the same links and clover run side by side on one
  // XCD and share its L2
  const int wl = xcd_swizzle(blockIdx.x, gridDim.x);
  const int r = wl % nrhs;
  const int ls = (wl / nrhs) * blockDim.x + threadIdx.x;  // lexicographic-block order
  // the block-crossing pieces only touch one layer of every block: one
  // thread per site of that layer (the output elsewhere is left alone)
  constexpr bool CROSS = MODE == DS_CROSS_FWD || MODE == DS_CROSS_BWD;
  const int per_block = CROSS ? g.vblock / g.bs[mu_sel] : g.vblock;
  if (ls >= g.nblocks * per_block) return;
  const int bl = ls / per_block;
  const int lo = ls - bl * per_block;
  int bc[4];
  bc[0] = bl % g.NB[0];
  bc[1] = (bl / g.NB[0]) % g.NB[1];
  bc[2] = (bl / (g.NB[0] * g.NB[1])) % g.NB[2];
  bc[3] = bl / (g.NB[0] * g.NB[1] * g.NB[2]);
  const int s = block_to_int(g, bc) * g.vblock +
                (CROSS ? face_site(g, mu_sel, MODE == DS_CROSS_FWD ? g.bs[mu_sel] - 1 : 0, lo) : lo);
  const cx<Tin>* ip = in + (size_t)r * in_rs;
  cx<Tout>* op = out + (size_t)r * out_rs;
  const size_t V = g.V;
  const SitePos pos = site_pos(g, s);
  cx<Tc> acc[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[sp][k] = mk((Tc)0, (Tc)0);
  if (MODE == DS_FULL || MODE == DS_BLOCK) {
    cx<Tc> p[4][3];
    load_spinor<Tin, Tc, MODE != DS_FULL>(p, ip, s, V, chi_in, (Tc)1);
    clover_apply<Tc, S>(acc, p, gv, s, V);
  }
  hops_all<Tin, Tc, S, MODE>(acc, ip, gv, g, pos, mu_sel, chi_in);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) op[(size_t)(3 * sp + k) * V + s] = cvt<Tout>(acc[sp][k]);
}

}  // namespace

template <typename Tin, typename Tout, typename S, typename Tc>
void launch_dslash(cx<Tout>* out, const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g, int nrhs, int mode,
                   int mu, int chi_in, size_t in_rstride, size_t out_rstride, hipStream_t st) {
  if (nrhs <= 0) return;
  const size_t nsite = (mode == DS_CROSS_FWD || mode == DS_CROSS_BWD) ? (size_t)g.nblocks * (g.vblock / g.bs[mu])
                                                                      : (size_t)g.V;
  const unsigned grid = (unsigned)((nsite + TPB - 1) / TPB) * (unsigned)nrhs;
  switch (mode) {
    case DS_FULL:
      dslash_kernel<Tin, Tout, S, Tc, DS_FULL><<<grid, TPB, 0, st>>>(out, in, gv, g, mu, chi_in, in_rstride, out_rstride, nrhs);
      break;
    case DS_BLOCK:
      dslash_kernel<Tin, Tout, S, Tc, DS_BLOCK><<<grid, TPB, 0, st>>>(out, in, gv, g, mu, chi_in, in_rstride, out_rstride, nrhs);
      break;
    case DS_CROSS_FWD:
      dslash_kernel<Tin, Tout, S, Tc, DS_CROSS_FWD><<<grid, TPB, 0, st>>>(out, in, gv, g, mu, chi_in, in_rstride,
                                                                          out_rstride, nrhs);
      break;
    default:
      dslash_kernel<Tin, Tout, S, Tc, DS_CROSS_BWD><<<grid, TPB, 0, st>>>(out, in, gv, g, mu, chi_in, in_rstride,
                                                                          out_rstride, nrhs);
      break;
  }
}

#define INST(Tin, Tout, S, Tc)                                                                                   \
  template void launch_dslash<Tin, Tout, S, Tc>(cx<Tout>*, const cx<Tin>*, const GaugeView<S>&, const Geom&, int, \
                                                int, int, int, size_t, size_t, hipStream_t);
INST(double, double, double, double)
INST(float, float, float, float)
INST(float, float, __half, float)
INST(float, double, double, double)
#undef INST

}  // namespace ddamg
