// Per-site device helpers of the Wilson-clover operator shared by the
// dslash and SAP kernels: spin projection/reconstruction of the hops, SU(3)
// link loads, the clover block multiply, and one site of D or its pieces.
//
// In the chiral basis g_mu = [[0, X_mu], [X_mu^dag, 0]] with X_k = -i s_k
// (Pauli s_k) and X_4 = -1, so
//   (1 - g) psi = (h, -X^dag h),  h = psi_up - X psi_dn
//   (1 + g) psi = (h,  X^dag h),  h = psi_up + X psi_dn
// and each hop multiplies only the 2-spinor h by the link.
#pragma once
#include "ddamg_internal.h"

namespace ddamg {
namespace dev {

template <typename T>
struct Half2 {
  cx<T> h[2][3];
};

// h = psi_up - X_mu psi_dn (FWD) or psi_up + X_mu psi_dn (BWD)
template <int MU, bool FWD, typename T>
__device__ inline void project(Half2<T>& o, const cx<T> p[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 0) {
      o.h[0][c] = FWD ? p[0][c] + times_i(p[3][c]) : p[0][c] + times_mi(p[3][c]);
      o.h[1][c] = FWD ? p[1][c] + times_i(p[2][c]) : p[1][c] + times_mi(p[2][c]);
    } else if (MU == 1) {
      o.h[0][c] = FWD ? p[0][c] + p[3][c] : p[0][c] - p[3][c];
      o.h[1][c] = FWD ? p[1][c] - p[2][c] : p[1][c] + p[2][c];
    } else if (MU == 2) {
      o.h[0][c] = FWD ? p[0][c] + times_i(p[2][c]) : p[0][c] + times_mi(p[2][c]);
      o.h[1][c] = FWD ? p[1][c] + times_mi(p[3][c]) : p[1][c] + times_i(p[3][c]);
    } else {
      o.h[0][c] = FWD ? p[0][c] + p[2][c] : p[0][c] - p[2][c];
      o.h[1][c] = FWD ? p[1][c] + p[3][c] : p[1][c] - p[3][c];
    }
  }
}

// acc += coef * (h, lower(h)) with lower = -X^dag h (FWD) or X^dag h (BWD)
template <int MU, bool FWD, typename T>
__device__ inline void reconstruct(cx<T> acc[4][3], const Half2<T>& u, T coef) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<T> h0 = u.h[0][c], h1 = u.h[1][c];
    cx<T> l0, l1;
    if (MU == 0) {
      l0 = times_i(h1);
      l1 = times_i(h0);
    } else if (MU == 1) {
      l0 = h1;
      l1 = neg(h0);
    } else if (MU == 2) {
      l0 = times_i(h0);
      l1 = times_mi(h1);
    } else {
      l0 = neg(h0);
      l1 = neg(h1);
    }
    if (FWD) {
      l0 = neg(l0);
      l1 = neg(l1);
    }
    acc[0][c] = acc[0][c] + coef * h0;
    acc[1][c] = acc[1][c] + coef * h1;
    acc[2][c] = acc[2][c] + coef * l0;
    acc[3][c] = acc[3][c] + coef * l1;
  }
}

template <typename Tin, typename Tc, bool CHI = true>
__device__ inline void load_spinor(cx<Tc> p[4][3], const cx<Tin>* in, int s, size_t V, int chi_in, Tc sign) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    const bool keep = !CHI || chi_in < 0 || (sp >> 1) == chi_in;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<Tc> v = cvt<Tc>(elem(in + (size_t)(3 * sp + c) * V, (unsigned)s));
      p[sp][c] = keep ? sign * v : mk((Tc)0, (Tc)0);
    }
  }
}

// link entries as stored (FP16: without the per-site scale, which the hop
// applies once to its 2-spinor result)
template <typename Tc, typename S>
__device__ inline void load_link(cx<Tc> u[3][3], const GaugeView<S>& gv, int mu, int s, size_t V) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) u[a][b] = ldc<Tc>(gv.U + (size_t)(mu * 9 + 3 * a + b) * V, (unsigned)s);
}

// acc += -1/2 (1 -+ g_mu) [U_mu(slink) or U_mu(slink)^dag] p
template <int MU, bool FWD, typename Tc, typename S>
__device__ inline void hop_spinor(cx<Tc> acc[4][3], const cx<Tc> p[4][3], const GaugeView<S>& gv, int slink,
                                  size_t V) {
  Half2<Tc> h, u;
  project<MU, FWD, Tc>(h, p);
  cx<Tc> U[3][3];
  load_link<Tc, S>(U, gv, MU, slink, V);
  Tc coef = (Tc)-0.5;
  if constexpr (is_half<S>()) coef *= (Tc)gv.Usc[slink];
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

// acc[r] += coef (1 -+ g_mu) [U or U^dag] p[r] for NR spinors and a link
// already loaded (entries as stored, coef = -1/2 times the link scale)
template <int MU, bool FWD, int NR, typename Tc>
__device__ inline void hop_spinor_multi_u(cx<Tc> acc[NR][4][3], const cx<Tc> p[NR][4][3], const cx<Tc> U[3][3],
                                          Tc coef) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    Half2<Tc> h, u;
    project<MU, FWD, Tc>(h, p[r]);
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

// The same hop applied to NR spinors with one load of the link.
template <int MU, bool FWD, int NR, typename Tc, typename S>
__device__ inline void hop_spinor_multi(cx<Tc> acc[NR][4][3], const cx<Tc> p[NR][4][3], const GaugeView<S>& gv,
                                        int slink, size_t V) {
  cx<Tc> U[3][3];
  load_link<Tc, S>(U, gv, MU, slink, V);
  Tc coef = (Tc)-0.5;
  if constexpr (is_half<S>()) coef *= (Tc)gv.Usc[slink];
  hop_spinor_multi_u<MU, FWD, NR, Tc>(acc, p, U, coef);
}

template <int MU, bool FWD, typename Tin, typename Tc, typename S, bool CHI>
__device__ inline void hop(cx<Tc> acc[4][3], const cx<Tin>* in, const GaugeView<S>& gv, int sn, int slink, size_t V,
                           int chi_in, Tc sign) {
  cx<Tc> p[4][3];
  load_spinor<Tin, Tc, CHI>(p, in, sn, V, chi_in, sign);
  hop_spinor<MU, FWD, Tc, S>(acc, p, gv, slink, V);
}

// acc += A(x) psi(x) for the two chirality blocks
template <typename Tc, typename S>
__device__ inline void clover_apply(cx<Tc> acc[4][3], const cx<Tc> p[4][3], const GaugeView<S>& gv, int s, size_t V) {
  Tc sc = (Tc)1;
  if constexpr (is_half<S>()) sc = (Tc)gv.Asc[s];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const stc_t<S>* Ah = gv.A + (size_t)h * CLOVER_PAIRS * V;
    cx<Tc> v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = p[2 * h + k / 3][k % 3];
    cx<Tc> o[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<Tc> d = ldc<Tc>(Ah + (size_t)k * V, (unsigned)s);
      o[2 * k] = d.r * v[2 * k];
      o[2 * k + 1] = d.i * v[2 * k + 1];
    }
    int q = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j) {
        const cx<Tc> a = ldc<Tc>(Ah + (size_t)(3 + q) * V, (unsigned)s);
        o[i] = cfma(a, v[j], o[i]);
        o[j] = cfmac(a, v[i], o[j]);
        ++q;
      }
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[2 * h + k / 3][k % 3] = acc[2 * h + k / 3][k % 3] + sc * o[k];
  }
}

// acc[r] += sc A_h p[r] on chirality h for NR spinors, the 18 stored pairs
// of A_h already loaded
template <int NR, typename Tc>
__device__ inline void clover_half_multi(cx<Tc> acc[NR][4][3], const cx<Tc> p[NR][4][3], const cx<Tc> a[CLOVER_PAIRS],
                                         int h, Tc sc) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    cx<Tc> v[6], o[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = p[r][2 * h + k / 3][k % 3];
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

// acc[r] += A(x) p[r] for NR spinors with one load of the clover entries
template <int NR, typename Tc, typename S>
__device__ inline void clover_apply_multi(cx<Tc> acc[NR][4][3], const cx<Tc> p[NR][4][3], const GaugeView<S>& gv,
                                          int s, size_t V) {
  Tc sc = (Tc)1;
  if constexpr (is_half<S>()) sc = (Tc)gv.Asc[s];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const stc_t<S>* Ah = gv.A + (size_t)h * CLOVER_PAIRS * V;
    cx<Tc> a[CLOVER_PAIRS];
#pragma unroll
    for (int e = 0; e < CLOVER_PAIRS; ++e) a[e] = ldc<Tc>(Ah + (size_t)e * V, (unsigned)s);
    clover_half_multi<NR, Tc>(acc, p, a, h, sc);
  }
}

// Position of an internal site: block coordinates, local coordinates and
// the local index, from which neighbours are found without a table.
struct SitePos {
  int S, ci, l;
  int bc[4], lc[4];
};

__device__ inline SitePos site_pos(const Geom& g, int S) {
  SitePos p;
  p.S = S;
  p.ci = S / g.vblock;
  p.l = S - p.ci * g.vblock;
  int_block_coords(g, p.ci, p.bc);
  local_coords(g, p.l, p.lc);
  return p;
}

// internal index of the forward / backward neighbour in direction mu
__device__ inline int nbr_fwd(const Geom& g, const SitePos& p, int mu) {
  if (p.lc[mu] < g.bs[mu] - 1) return p.S + g.lstr[mu];
  int bc[4] = {p.bc[0], p.bc[1], p.bc[2], p.bc[3]};
  bc[mu] = bc[mu] + 1 == g.NB[mu] ? 0 : bc[mu] + 1;
  return block_to_int(g, bc) * g.vblock + p.l - p.lc[mu] * g.lstr[mu];
}
__device__ inline int nbr_bwd(const Geom& g, const SitePos& p, int mu) {
  if (p.lc[mu] > 0) return p.S - g.lstr[mu];
  int bc[4] = {p.bc[0], p.bc[1], p.bc[2], p.bc[3]};
  bc[mu] = bc[mu] == 0 ? g.NB[mu] - 1 : bc[mu] - 1;
  return block_to_int(g, bc) * g.vblock + p.l + (g.bs[mu] - 1) * g.lstr[mu];
}

// hops of direction MU selected by MODE: all (full D), inside the block
// (block operator B), or the block-crossing forward / backward hops of
// direction mu_sel.  A hop across the time boundary carries the factor -1.
template <int MU, typename Tin, typename Tc, typename S, int MODE>
__device__ inline void hops_mu(cx<Tc> acc[4][3], const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g,
                               const SitePos& p, int mu_sel, int chi_in) {
  const size_t V = g.V;
  const int l = p.lc[MU];
  bool do_f, do_b;
  if (MODE == DS_FULL) {
    // true at run time; being opaque to the compiler it keeps each hop in
    // its own branch, so its loads are issued with its arithmetic instead of
    // all being hoisted to the top of the kernel
    do_f = do_b = g.V > 0;
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
    hop<MU, true, Tin, Tc, S, MODE != DS_FULL>(acc, in, gv, nbr_fwd(g, p, MU), p.S, V, chi_in, wrap ? (Tc)-1 : (Tc)1);
  }
  if (do_b) {
    const bool wrap = MU == 3 && l == 0 && p.bc[3] == 0;
    const int sb = nbr_bwd(g, p, MU);
    hop<MU, false, Tin, Tc, S, MODE != DS_FULL>(acc, in, gv, sb, sb, V, chi_in, wrap ? (Tc)-1 : (Tc)1);
  }
}

// All four directions, one after the other.  The empty asm statements with a
// memory clobber keep the compiler from hoisting the loads of later
// directions above the arithmetic of earlier ones, which would keep all
// eight neighbours live at once and overflow the register file.
template <typename Tin, typename Tc, typename S, int MODE>
__device__ inline void hops_all(cx<Tc> acc[4][3], const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g,
                                const SitePos& p, int mu_sel, int chi_in) {
  hops_mu<0, Tin, Tc, S, MODE>(acc, in, gv, g, p, mu_sel, chi_in);
  asm volatile("" ::: "memory");
  hops_mu<1, Tin, Tc, S, MODE>(acc, in, gv, g, p, mu_sel, chi_in);
  asm volatile("" ::: "memory");
  hops_mu<2, Tin, Tc, S, MODE>(acc, in, gv, g, p, mu_sel, chi_in);
  asm volatile("" ::: "memory");
  hops_mu<3, Tin, Tc, S, MODE>(acc, in, gv, g, p, mu_sel, chi_in);
}

}  // namespace dev
}  // namespace ddamg
