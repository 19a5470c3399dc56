// Wilson-clover operator on site-major structure-of-arrays fields.
//
//   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
//                                         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// (Sec. 1; the hop/clover structure is the one Alg. 7 applies to the columns
// of P).  One thread per (site, group of NR rhs): consecutive lanes own
// consecutive sites, so every load of a spinor component, link entry or
// clover entry is a coalesced 64-lane access, and each link and clover entry
// loaded is used for all NR right-hand sides held in registers.  The spin
// projectors (1 -+ g_mu) reduce each hop to a 2-spinor (6 complex) before the
// SU(3) multiply.  In the chiral basis g_mu = [[0, X_mu], [X_mu^dag, 0]] with
// X_k = -i s_k and X_4 = -1:
//   (1 - g) psi = (h, -X^dag h),  h = psi_up - X psi_dn
//   (1 + g) psi = (h,  X^dag h),  h = psi_up + X psi_dn
// Variants: the full operator, the block operator B (hops leaving the block
// dropped, Alg. 3), and the block-crossing forward/backward hops of one
// direction (the pieces D_ij of Eq. cgo for a neighbour block j).  The input
// of the block and crossing variants may be restricted to one chirality
// (a column of P); the other chirality is then neither loaded nor used.
// Workgroups walk the blocks in lexicographic order (through the XCD
// swizzle), so face neighbours are processed at the same time on the same
// XCD although blocks of opposite parity are far apart in memory.
#include "dirac_device.h"

namespace ddamg {

namespace {

constexpr int TPB = 256;
using namespace dev;

// spinor of one rhs at site s; with chi >= 0 only the spins of that chirality
// are loaded (a uniform branch), the others are zero
template <typename Tin, typename Tc>
__device__ inline void load_spinor_chi(cx<Tc> p[4][3], const cx<Tin>* in, int s, size_t V, int chi) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    const bool keep = chi < 0 || (sp >> 1) == chi;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (keep)
        p[sp][c] = cvt<Tc>(elem(in + (size_t)(3 * sp + c) * V, (unsigned)s));
      else
        p[sp][c] = mk((Tc)0, (Tc)0);
    }
  }
}

// acc[r] += -1/2 sign (1 -+ g_MU) [U_MU(slink) or its adjoint] psi_r(sn) for
// the nr rhs of the group (the slots r >= nr read rhs nr - 1 and are never
// stored), with one load of the link
template <int MU, bool FWD, int NR, typename Tin, typename Tc, typename S>
__device__ inline void hop_group(cx<Tc> acc[NR][4][3], const cx<Tin>* in, size_t rs, int nr, const GaugeView<S>& gv,
                                 int sn, int slink, size_t V, int chi, Tc sign) {
  cx<Tc> U[3][3];
  load_link<Tc, S>(U, gv, MU, slink, V);
  Tc coef = (Tc)-0.5 * sign;
  if constexpr (is_half<S>()) coef *= (Tc)gv.Usc[slink];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    cx<Tc> p[4][3];
    load_spinor_chi<Tin, Tc>(p, in + (size_t)min(r, nr - 1) * rs, sn, V, chi);
    Half2<Tc> h, u;
    project<MU, FWD, Tc>(h, p);
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cx<Tc> t = mk((Tc)0, (Tc)0);
#pragma unroll
        for (int b = 0; b < 3; ++b) t = FWD ? cfma(U[a][b], h.h[sp][b], t) : cfmac(U[b][a], h.h[sp][b], t);
        u.h[sp][a] = t;
      }
    reconstruct<MU, FWD, Tc>(acc[r], u, coef);
  }
}

// acc[r] += A(x) psi_r(x), one chirality block at a time (the clover is
// block diagonal in chirality); a chirality absent from the input is skipped
template <int NR, typename Tin, typename Tc, typename S>
__device__ inline void clover_group(cx<Tc> acc[NR][4][3], const cx<Tin>* in, size_t rs, int nr, const GaugeView<S>& gv,
                                    int s, size_t V, int chi) {
  Tc sc = (Tc)1;
  if constexpr (is_half<S>()) sc = (Tc)gv.Asc[s];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (chi >= 0 && h != chi) continue;
    const stc_t<S>* Ah = gv.A + (size_t)h * CLOVER_PAIRS * V;
    cx<Tc> a[CLOVER_PAIRS];
#pragma unroll
    for (int e = 0; e < CLOVER_PAIRS; ++e) a[e] = ldc<Tc>(Ah + (size_t)e * V, (unsigned)s);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const cx<Tin>* ir = in + (size_t)min(r, nr - 1) * rs;
      cx<Tc> v[6], o[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = cvt<Tc>(elem(ir + (size_t)(6 * h + k) * V, (unsigned)s));
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        o[2 * k] = a[k].r * v[2 * k];
        o[2 * k + 1] = a[k].i * v[2 * k + 1];
      }
      int q = 0;
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
          o[i] = cfma(a[3 + q], v[j], o[i]);
          o[j] = cfmac(a[3 + q], v[i], o[j]);
          ++q;
        }
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[r][2 * h + k / 3][k % 3] = acc[r][2 * h + k / 3][k % 3] + sc * o[k];
    }
  }
}

// the hops of direction MU that MODE selects (see hops_mu in dirac_device.h);
// a hop across the time boundary carries the factor -1
template <int MU, int MODE, int NR, typename Tin, typename Tc, typename S>
__device__ inline void hops_group_mu(cx<Tc> acc[NR][4][3], const cx<Tin>* in, size_t rs, int nr,
                                     const GaugeView<S>& gv, const Geom& g, const SitePos& p, int mu_sel, int chi) {
  const size_t V = g.V;
  const int l = p.lc[MU];
  bool do_f, do_b;
  if (MODE == DS_FULL) {
    do_f = do_b = g.V > 0;  // opaque: keeps every hop in its own branch
  } else if (MODE == DS_BLOCK) {
    do_f = l != g.bs[MU] - 1;
    do_b = l != 0;
  } else if (MODE == DS_CROSS_FWD) {
    do_f = MU == mu_sel && l == g.bs[MU] - 1;
    do_b = false;
  } else {
    do_f = false;
    do_b = MU == mu_sel && l == 0;
  }
  if (do_f) {
    const bool wrap = MU == 3 && l == g.bs[3] - 1 && p.bc[3] == g.NB[3] - 1;
    hop_group<MU, true, NR, Tin, Tc, S>(acc, in, rs, nr, gv, nbr_fwd(g, p, MU), p.S, V, chi, wrap ? (Tc)-1 : (Tc)1);
  }
  if (do_b) {
    const bool wrap = MU == 3 && l == 0 && p.bc[3] == 0;
    const int sb = nbr_bwd(g, p, MU);
    hop_group<MU, false, NR, Tin, Tc, S>(acc, in, rs, nr, gv, sb, sb, V, chi, wrap ? (Tc)-1 : (Tc)1);
  }
}

template <typename Tin, typename Tout, typename S, typename Tc, int MODE, int NR>
__global__ __launch_bounds__(TPB) void dslash_kernel(cx<Tout>* __restrict__ out, const cx<Tin>* __restrict__ in,
                                                     GaugeView<S> gv, Geom g, int mu_sel, int chi_in, size_t in_rs,
                                                     size_t out_rs, int nrhs) {
  // workgroup = (run of 256 sites, group of NR rhs) with the group fastest,
  // so the workgroups that read the same links and clover run side by side
  // on one XCD and share its L2
  const int ngroup = (nrhs + NR - 1) / NR;
  const int wl = xcd_swizzle(blockIdx.x, gridDim.x);
  const int r0 = (wl % ngroup) * NR;
  const int nr = min(NR, nrhs - r0);
  const int ls = (wl / ngroup) * blockDim.x + threadIdx.x;  // lexicographic-block order
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
  const cx<Tin>* ip = in + (size_t)r0 * in_rs;
  cx<Tout>* op = out + (size_t)r0 * out_rs;
  const size_t V = g.V;
  // the full operator takes both chiralities whatever chi_in says
  const int chi = MODE == DS_FULL ? -1 : chi_in;
  const SitePos pos = site_pos(g, s);
  cx<Tc> acc[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[r][sp][k] = mk((Tc)0, (Tc)0);
  if (MODE == DS_FULL || MODE == DS_BLOCK) clover_group<NR, Tin, Tc, S>(acc, ip, in_rs, nr, gv, s, V, chi);
  hops_group_mu<0, MODE, NR, Tin, Tc, S>(acc, ip, in_rs, nr, gv, g, pos, mu_sel, chi);
  asm volatile("" ::: "memory");
  hops_group_mu<1, MODE, NR, Tin, Tc, S>(acc, ip, in_rs, nr, gv, g, pos, mu_sel, chi);
  asm volatile("" ::: "memory");
  hops_group_mu<2, MODE, NR, Tin, Tc, S>(acc, ip, in_rs, nr, gv, g, pos, mu_sel, chi);
  asm volatile("" ::: "memory");
  hops_group_mu<3, MODE, NR, Tin, Tc, S>(acc, ip, in_rs, nr, gv, g, pos, mu_sel, chi);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) break;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) op[(size_t)r * out_rs + (size_t)(3 * sp + k) * V + s] = cvt<Tout>(acc[r][sp][k]);
  }
}

// The full operator with the block's input staged in LDS: workgroup = (one
// block, group of NR rhs), one lane per site.  The block's spinors are read
// once, coalesced, into LDS; a hop to a neighbour inside the block reads it
// there, a hop leaving the block reads the neighbour block in global memory
// (the lanes of a wave on a block face take that branch).  This keeps the
// eight neighbour reads of every site out of the L2.
template <int MU, bool FWD, int NR, typename Tin, typename Tc, typename S>
__device__ inline void hop_staged(cx<Tc> acc[NR][4][3], const cx<Tin>* lds, int vb, int ln, bool inside,
                                  const cx<Tin>* in, size_t rs, int nr, int sn, int slink, Tc sign,
                                  const GaugeView<S>& gv, size_t V) {
  cx<Tc> p[NR][4][3];
  if (inside) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) p[r][sp][c] = cvt<Tc>(lds[(r * 12 + 3 * sp + c) * vb + ln]);
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const cx<Tin>* ir = in + (size_t)min(r, nr - 1) * rs;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) p[r][sp][c] = sign * cvt<Tc>(elem(ir + (size_t)(3 * sp + c) * V, (unsigned)sn));
    }
  }
  hop_spinor_multi<MU, FWD, NR, Tc, S>(acc, p, gv, slink, V);
}

template <int MU, int NR, typename Tin, typename Tc, typename S>
__device__ inline void hops_staged_mu(cx<Tc> acc[NR][4][3], const cx<Tin>* lds, int vb, const cx<Tin>* in, size_t rs,
                                      int nr, const GaugeView<S>& gv, const Geom& g, const SitePos& p) {
  const size_t V = g.V;
  const int l = p.lc[MU];
  const bool live = g.V > 0;  // opaque: each hop stays in its own region
  if (live) {
    const bool inside = l < g.bs[MU] - 1;
    const bool wrap = MU == 3 && !inside && p.bc[3] == g.NB[3] - 1;
    hop_staged<MU, true, NR, Tin, Tc, S>(acc, lds, vb, p.l + g.lstr[MU], inside, in, rs, nr,
                                          inside ? p.S : nbr_fwd(g, p, MU), p.S, wrap ? (Tc)-1 : (Tc)1, gv, V);
  }
  asm volatile("" ::: "memory");
  if (live) {
    const bool inside = l > 0;
    const bool wrap = MU == 3 && !inside && p.bc[3] == 0;
    const int sb = nbr_bwd(g, p, MU);
    hop_staged<MU, false, NR, Tin, Tc, S>(acc, lds, vb, p.l - g.lstr[MU], inside, in, rs, nr, sb, sb,
                                           wrap ? (Tc)-1 : (Tc)1, gv, V);
  }
}

template <typename Tin, typename Tout, typename S, typename Tc, int NR>
__global__ __launch_bounds__(256) void dslash_staged_kernel(cx<Tout>* __restrict__ out, const cx<Tin>* __restrict__ in,
                                                            GaugeView<S> gv, Geom g, size_t in_rs, size_t out_rs,
                                                            int nrhs) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int vb = g.vblock;
  cx<Tin>* lds = reinterpret_cast<cx<Tin>*>(smem_raw);  // [NR][12][vb]
  const int ngroup = (nrhs + NR - 1) / NR;
  const int wl = xcd_swizzle(blockIdx.x, gridDim.x);
  const int r0 = (wl % ngroup) * NR;
  const int nr = min(NR, nrhs - r0);
  const int bl = wl / ngroup;  // lexicographic block order
  int bc[4];
  bc[0] = bl % g.NB[0];
  bc[1] = (bl / g.NB[0]) % g.NB[1];
  bc[2] = (bl / (g.NB[0] * g.NB[1])) % g.NB[2];
  bc[3] = bl / (g.NB[0] * g.NB[1] * g.NB[2]);
  const int ci = block_to_int(g, bc);
  const int l = threadIdx.x;
  const bool act = l < vb;
  const size_t V = g.V;
  const int s = ci * vb + (act ? l : 0);
  const cx<Tin>* ip = in + (size_t)r0 * in_rs;
  if (act) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k)
        lds[(r * 12 + k) * vb + l] = elem(ip + (size_t)min(r, nr - 1) * in_rs + (size_t)k * V, (unsigned)s);
  }
  __syncthreads();
  if (!act) return;
  const SitePos pos = site_pos(g, s);
  cx<Tc> acc[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[r][sp][k] = mk((Tc)0, (Tc)0);
  {
    cx<Tc> p[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) p[r][sp][k] = cvt<Tc>(lds[(r * 12 + 3 * sp + k) * vb + l]);
    clover_apply_multi<NR, Tc, S>(acc, p, gv, s, V);
  }
  hops_staged_mu<0, NR, Tin, Tc, S>(acc, lds, vb, ip, in_rs, nr, gv, g, pos);
  asm volatile("" ::: "memory");
  hops_staged_mu<1, NR, Tin, Tc, S>(acc, lds, vb, ip, in_rs, nr, gv, g, pos);
  asm volatile("" ::: "memory");
  hops_staged_mu<2, NR, Tin, Tc, S>(acc, lds, vb, ip, in_rs, nr, gv, g, pos);
  asm volatile("" ::: "memory");
  hops_staged_mu<3, NR, Tin, Tc, S>(acc, lds, vb, ip, in_rs, nr, gv, g, pos);
  cx<Tout>* op = out + (size_t)r0 * out_rs;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) break;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) op[(size_t)r * out_rs + (size_t)(3 * sp + k) * V + s] = cvt<Tout>(acc[r][sp][k]);
  }
}

// 4^4 blocks, one rhs, FP32 input and arithmetic: the staged operator with
// the x and y faces of the neighbour blocks staged in LDS as well.  In the site-major
// planes a face across x or y is strided (every 4th site, or runs of 4), so
// each read of it pulls whole lines of the neighbour block; read late in
// the workgroup's life those lines have left the L2 and are fetched again.
// Here every lane loads one face site (4 faces x 64 sites = 256 lanes) at
// the start, next to its own site, while the neighbour workgroups stage the
// same lines, and keeps only its projection (1 -+ g_mu) psi, the 2-spinor
// the hop multiplies (half the LDS of the full spinor).  The z and t faces
// are contiguous runs and stay global.
constexpr int HB = 4;                 // block extent
constexpr int HVB = HB * HB * HB * HB;  // sites per block
constexpr int HF = HVB / HB;          // sites per face
constexpr int HD = 2;                 // directions whose faces are staged (x, y)

// local index of face site q (the three other coordinates in increasing
// dimension order) of the face with local coordinate lmu in direction mu
__device__ inline int face_site(int mu, int lmu, int q) {
  int c[4], k = 0;
  for (int d = 0; d < 4; ++d) {
    if (d == mu) {
      c[d] = lmu;
    } else {
      c[d] = (q >> (2 * k)) & 3;
      ++k;
    }
  }
  return c[0] + HB * (c[1] + HB * (c[2] + HB * c[3]));
}
// face index of local coordinates lc across direction mu
__device__ inline int face_index(int mu, const int lc[4]) {
  int q = 0, k = 0;
  for (int d = 0; d < 4; ++d)
    if (d != mu) {
      q |= lc[d] << (2 * k);
      ++k;
    }
  return q;
}

// acc += -1/2 (1 -+ g_mu) [U or U^dag] psi for a neighbour given by its
// projected 2-spinor h (the link at slink, as hop_spinor applies it)
template <int MU, bool FWD, typename Tc, typename S>
__device__ inline void hop_projected(cx<Tc> acc[4][3], const Half2<Tc>& h, const GaugeView<S>& gv, int slink,
                                     size_t V) {
  cx<Tc> U[3][3];
  load_link<Tc, S>(U, gv, MU, slink, V);
  Tc coef = (Tc)-0.5;
  if constexpr (is_half<S>()) coef *= (Tc)gv.Usc[slink];
  Half2<Tc> u;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<Tc> t = mk((Tc)0, (Tc)0);
#pragma unroll
      for (int b = 0; b < 3; ++b) t = FWD ? cfma(U[a][b], h.h[sp][b], t) : cfmac(U[b][a], h.h[sp][b], t);
      u.h[sp][a] = t;
    }
  reconstruct<MU, FWD, Tc>(acc, u, coef);
}

// both hops of direction MU: the neighbour's projected 2-spinor comes from
// the block in LDS (projected here), from the staged face (x and y), or
// from global memory (z and t faces, with the time boundary's sign)
template <int MU, typename Tin, typename Tc, typename S>
__device__ inline void hops_halo_mu(cx<Tc> acc[4][3], const cx<Tin>* lds, const cx<Tc>* halo, const cx<Tin>* in,
                                    const GaugeView<S>& gv, const Geom& g, const SitePos& p) {
  const size_t V = g.V;
  const int l = p.lc[MU];
  const bool live = g.V > 0;  // opaque: each hop stays in its own region
  if (live) {
    Half2<Tc> h;
    if (l < HB - 1 || MU >= HD) {
      cx<Tc> q[4][3];
      if (l < HB - 1) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int c = 0; c < 3; ++c) q[sp][c] = cvt<Tc>(lds[(3 * sp + c) * HVB + p.l + g.lstr[MU]]);
      } else {
        const int sn = nbr_fwd(g, p, MU);
        const Tc sign = MU == 3 && p.bc[3] == g.NB[3] - 1 ? (Tc)-1 : (Tc)1;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int c = 0; c < 3; ++c) q[sp][c] = sign * cvt<Tc>(elem(in + (size_t)(3 * sp + c) * V, (unsigned)sn));
      }
      project<MU, true, Tc>(h, q);
    } else {
      const cx<Tc>* hf = halo + (size_t)(2 * MU) * 6 * HF;
      const int fq = face_index(MU, p.lc);
#pragma unroll
      for (int k = 0; k < 6; ++k) h.h[k / 3][k % 3] = hf[k * HF + fq];
    }
    hop_projected<MU, true, Tc, S>(acc, h, gv, p.S, V);
  }
  asm volatile("" ::: "memory");
  if (live) {
    Half2<Tc> h;
    const int sb = nbr_bwd(g, p, MU);
    if (l > 0 || MU >= HD) {
      cx<Tc> q[4][3];
      if (l > 0) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int c = 0; c < 3; ++c) q[sp][c] = cvt<Tc>(lds[(3 * sp + c) * HVB + p.l - g.lstr[MU]]);
      } else {
        const Tc sign = MU == 3 && p.bc[3] == 0 ? (Tc)-1 : (Tc)1;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int c = 0; c < 3; ++c) q[sp][c] = sign * cvt<Tc>(elem(in + (size_t)(3 * sp + c) * V, (unsigned)sb));
      }
      project<MU, false, Tc>(h, q);
    } else {
      const cx<Tc>* hf = halo + (size_t)(2 * MU + 1) * 6 * HF;
      const int fq = face_index(MU, p.lc);
#pragma unroll
      for (int k = 0; k < 6; ++k) h.h[k / 3][k % 3] = hf[k * HF + fq];
    }
    hop_projected<MU, false, Tc, S>(acc, h, gv, sb, V);
  }
}

template <typename Tin, typename Tout, typename S, typename Tc>
__global__ __launch_bounds__(HVB) void dslash_halo_kernel(cx<Tout>* __restrict__ out, const cx<Tin>* __restrict__ in,
                                                          GaugeView<S> gv, Geom g) {
  __shared__ cx<Tin> lds[12 * HVB];     // the block's spinors [12][256]
  __shared__ cx<Tc> halo[2 * HD * 6 * HF];  // faces x+, x-, y+, y-: projected 2-spinors [2 HD][6][64]
  const int bl = xcd_swizzle(blockIdx.x, gridDim.x);  // lexicographic block order
  int bc[4];
  bc[0] = bl % g.NB[0];
  bc[1] = (bl / g.NB[0]) % g.NB[1];
  bc[2] = (bl / (g.NB[0] * g.NB[1])) % g.NB[2];
  bc[3] = bl / (g.NB[0] * g.NB[1] * g.NB[2]);
  const int ci = block_to_int(g, bc);
  const int l = threadIdx.x;
  const size_t V = g.V;
  const int s = ci * HVB + l;
  // the face site this lane stages: face f = 2 mu + (0 forward, 1 backward),
  // the neighbour block's sites with local coordinate 0 (forward) or 3
#pragma unroll
  for (int k = 0; k < 12; ++k) lds[k * HVB + l] = elem(in + (size_t)k * V, (unsigned)s);
  if (l < 2 * HD * HF) {
    const int f = l / HF, q = l % HF, mu = f >> 1;
    int nc[4] = {bc[0], bc[1], bc[2], bc[3]};
    if ((f & 1) == 0)
      nc[mu] = nc[mu] + 1 == g.NB[mu] ? 0 : nc[mu] + 1;
    else
      nc[mu] = nc[mu] == 0 ? g.NB[mu] - 1 : nc[mu] - 1;
    const int sn = block_to_int(g, nc) * HVB + face_site(mu, (f & 1) == 0 ? 0 : HB - 1, q);
    cx<Tc> ph[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) ph[k / 3][k % 3] = cvt<Tc>(elem(in + (size_t)k * V, (unsigned)sn));
    // the hop that reads this face site needs only its projection:
    // (1 - g_mu) for the forward face, (1 + g_mu) for the backward one
    Half2<Tc> h;
    if (f == 0)
      project<0, true, Tc>(h, ph);
    else if (f == 1)
      project<0, false, Tc>(h, ph);
    else if (f == 2)
      project<1, true, Tc>(h, ph);
    else
      project<1, false, Tc>(h, ph);
#pragma unroll
    for (int k = 0; k < 6; ++k) halo[(f * 6 + k) * HF + q] = h.h[k / 3][k % 3];
  }
  __syncthreads();
  const SitePos pos = site_pos(g, s);
  cx<Tc> acc[1][4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[0][sp][k] = mk((Tc)0, (Tc)0);
  {
    cx<Tc> p[1][4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) p[0][sp][k] = cvt<Tc>(lds[(3 * sp + k) * HVB + l]);
    clover_apply_multi<1, Tc, S>(acc, p, gv, s, V);
  }
  hops_halo_mu<0, Tin, Tc, S>(acc[0], lds, halo, in, gv, g, pos);
  asm volatile("" ::: "memory");
  hops_halo_mu<1, Tin, Tc, S>(acc[0], lds, halo, in, gv, g, pos);
  asm volatile("" ::: "memory");
  hops_halo_mu<2, Tin, Tc, S>(acc[0], lds, halo, in, gv, g, pos);
  asm volatile("" ::: "memory");
  hops_halo_mu<3, Tin, Tc, S>(acc[0], lds, halo, in, gv, g, pos);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[(size_t)(3 * sp + k) * V + s] = cvt<Tout>(acc[0][sp][k]);
}

template <typename Tin, typename Tout, typename S, typename Tc, int NR>
void launch_staged(cx<Tout>* out, const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g, int nrhs, size_t in_rs,
                   size_t out_rs, hipStream_t st) {
  const int threads = ((g.vblock + 63) / 64) * 64;
  const size_t lds = (size_t)NR * 12 * g.vblock * sizeof(cx<Tin>);
  const unsigned grid = (unsigned)g.nblocks * (unsigned)((nrhs + NR - 1) / NR);
  dslash_staged_kernel<Tin, Tout, S, Tc, NR><<<grid, threads, lds, st>>>(out, in, gv, g, in_rs, out_rs, nrhs);
}

template <typename Tin, typename Tout, typename S, typename Tc, int MODE, int NR>
void launch_mode(cx<Tout>* out, const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g, int nrhs, int mu, int chi_in,
                 size_t in_rs, size_t out_rs, size_t nsite, hipStream_t st) {
  const unsigned grid = (unsigned)((nsite + TPB - 1) / TPB) * (unsigned)((nrhs + NR - 1) / NR);
  dslash_kernel<Tin, Tout, S, Tc, MODE, NR><<<grid, TPB, 0, st>>>(out, in, gv, g, mu, chi_in, in_rs, out_rs, nrhs);
}

// rhs per thread: 1 for a lone rhs; otherwise as many as the registers hold
// without spilling (the accumulators of FP64 spinors are twice the size)
template <typename Tin, typename Tout, typename S, typename Tc, int MODE>
void launch_nr(cx<Tout>* out, const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g, int nrhs, int mu, int chi_in,
               size_t in_rs, size_t out_rs, size_t nsite, hipStream_t st) {
  if (nrhs == 1) {
    launch_mode<Tin, Tout, S, Tc, MODE, 1>(out, in, gv, g, nrhs, mu, chi_in, in_rs, out_rs, nsite, st);
  } else if constexpr (sizeof(Tc) == 8) {
    launch_mode<Tin, Tout, S, Tc, MODE, 2>(out, in, gv, g, nrhs, mu, chi_in, in_rs, out_rs, nsite, st);
  } else {
    if (nrhs < 4)
      launch_mode<Tin, Tout, S, Tc, MODE, 2>(out, in, gv, g, nrhs, mu, chi_in, in_rs, out_rs, nsite, st);
    else
      launch_mode<Tin, Tout, S, Tc, MODE, 4>(out, in, gv, g, nrhs, mu, chi_in, in_rs, out_rs, nsite, st);
  }
}

}  // namespace

template <typename Tin, typename Tout, typename S, typename Tc>
void launch_dslash(cx<Tout>* out, const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g, int nrhs, int mode,
                   int mu, int chi_in, size_t in_rstride, size_t out_rstride, hipStream_t st) {
  if (nrhs <= 0) return;
  const size_t nsite = (mode == DS_CROSS_FWD || mode == DS_CROSS_BWD) ? (size_t)g.nblocks * (g.vblock / g.bs[mu])
                                                                      : (size_t)g.V;
  switch (mode) {
    case DS_FULL:
      // blocks of up to 256 sites: the block-staged kernel, one or two rhs per lane
      if (g.vblock <= 256) {
        if (nrhs == 1) {
          // 4^4 blocks, FP32 input and arithmetic: the x and y faces staged as well
          if constexpr (sizeof(Tin) == 4 && sizeof(Tc) == 4) {
            if (g.bs[0] == HB && g.bs[1] == HB && g.bs[2] == HB && g.bs[3] == HB) {
              dslash_halo_kernel<Tin, Tout, S, Tc><<<g.nblocks, HVB, 0, st>>>(out, in, gv, g);
              break;
            }
          }
          launch_staged<Tin, Tout, S, Tc, 1>(out, in, gv, g, nrhs, in_rstride, out_rstride, st);
        }
        else
          launch_staged<Tin, Tout, S, Tc, 2>(out, in, gv, g, nrhs, in_rstride, out_rstride, st);
        break;
      }
      launch_nr<Tin, Tout, S, Tc, DS_FULL>(out, in, gv, g, nrhs, mu, chi_in, in_rstride, out_rstride, nsite, st);
      break;
    case DS_BLOCK:
      launch_nr<Tin, Tout, S, Tc, DS_BLOCK>(out, in, gv, g, nrhs, mu, chi_in, in_rstride, out_rstride, nsite, st);
      break;
    case DS_CROSS_FWD:
      launch_nr<Tin, Tout, S, Tc, DS_CROSS_FWD>(out, in, gv, g, nrhs, mu, chi_in, in_rstride, out_rstride, nsite, st);
      break;
    default:
      launch_nr<Tin, Tout, S, Tc, DS_CROSS_BWD>(out, in, gv, g, nrhs, mu, chi_in, in_rstride, out_rstride, nsite, st);
      break;
  }
}

// The runtime loads a file's code object (device memory for its kernels)
// when one of them is first used; asking for a kernel's attributes does it
// now, so that later applies, including the one that must not allocate,
// find the code resident.
void preload_dslash_code() {
  hipFuncAttributes a;
  (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&dslash_staged_kernel<double, double, double, double, 1>));
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
