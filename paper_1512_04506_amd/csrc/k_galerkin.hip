// Block-crossing couplings of the coarse operator, Eq. (cgo):
//
//   (D_c)_{b, b+mu}[i][j] = w_i^{b dag} D_{b, b+mu} w_j^{b+mu}
//     = -1/2 s sum_{x in F} < w_i(x), (1 - g_mu) U_mu(x) w_j(x + mu) >
//
// where F is the last layer of block b in direction mu (its sites are the
// only ones with a forward neighbour in block b + mu) and s = -1 for the hop
// across the time boundary.  With the forward spin projection
// P_mu psi = psi_up - X_mu psi_dn (the 2-spinor a hop multiplies by the link)
// and the reconstruction R u = (u, -X_mu^dag u), (1 - g_mu) v = R P_mu v and
// <w, R u> = <P_mu w, u>, so each term is a 6-component inner product
//
//   < P_mu w_i(x), U_mu(x) P_mu w_j(x + mu) >.
//
// A basis vector lives on one chirality, so P_mu w is two of its spins
// multiplied by phases +-1, +-i: exact copies of stored values.  Per block
// and direction this is a complex contraction of 2 ntv rows by 2 ntv
// columns over 6 |F| terms, which runs on the matrix cores, one wave per
// (row chirality, column chirality) quadrant: FP32 32x32x2 MFMA, or FP64
// 16x16x4 MFMA on four 16x16 tiles.  Chunks of face sites (8 in FP32, 4 in
// FP64) are staged through LDS; the loads of the next chunk are issued
// before the matrix products of the current one.
#include <type_traits>

#include "galerkin.h"

namespace ddamg {

namespace {

typedef float gc_v16 __attribute__((ext_vector_type(16)));
typedef double gc_v4d __attribute__((ext_vector_type(4)));
template <typename T>
struct GcShape {
  static constexpr int CS = sizeof(T) == 8 ? 4 : 8;  // face sites per chunk
  static constexpr int ROWS = 6 * CS;                 // contraction terms per chunk
  static constexpr int NQ = CS / 2;                   // (spin, chirality, vector) entries per thread and chunk
};
constexpr int GC_LD = 33;  // padded row length in LDS

// P_mu w for w of chirality ch: component sg of the 2-spinor is
// phase * w_spin.  ch = 0: (w_0, w_1).  ch = 1: -X_mu (w_2, w_3), i.e.
// mu = 0: i (w_3, w_2); mu = 1: (w_3, -w_2); mu = 2: (i w_2, -i w_3);
// mu = 3: (w_2, w_3).
__device__ inline void proj_spin(int mu, int ch, int sg, int& spin, float& pr, float& pi) {
  if (ch == 0) {
    spin = sg;
    pr = 1.f;
    pi = 0.f;
  } else if (mu == 0) {
    spin = 3 - sg;
    pr = 0.f;
    pi = 1.f;
  } else if (mu == 1) {
    spin = 3 - sg;
    pr = sg ? -1.f : 1.f;
    pi = 0.f;
  } else if (mu == 2) {
    spin = 2 + sg;
    pr = 0.f;
    pi = sg ? -1.f : 1.f;
  } else {
    spin = 2 + sg;
    pr = 1.f;
    pi = 0.f;
  }
}

__device__ inline int sel4(const int a[4], int mu) { return mu == 0 ? a[0] : mu == 1 ? a[1] : mu == 2 ? a[2] : a[3]; }

// two waves per SIMD (the FP64 instance would otherwise take 280 registers)
template <typename T, typename S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void galerkin_cross_kernel(cx<T>* __restrict__ Dc, BasisView<S> bv,
                                                             GaugeView<T> gv, Geom g) {
  constexpr int GC_CS = GcShape<T>::CS, GC_ROWS = GcShape<T>::ROWS, GC_NQ = GcShape<T>::NQ;
  __shared__ cx<T> Ps[2][GC_ROWS][GC_LD];  // [row chirality][term][row vector]
  __shared__ cx<T> Qs[2][GC_ROWS][GC_LD];  // [column chirality][term][column vector]
  // blocks in lexicographic order (through the XCD swizzle): the neighbour
  // blocks read here are processed at about the same time on the same XCD
  const int bl = xcd_swizzle(blockIdx.x, gridDim.x);
  int bc[4];
  bc[0] = bl % g.NB[0];
  bc[1] = (bl / g.NB[0]) % g.NB[1];
  bc[2] = (bl / (g.NB[0] * g.NB[1])) % g.NB[2];
  bc[3] = bl / (g.NB[0] * g.NB[1] * g.NB[2]);
  const int ci = block_to_int(g, bc);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int h = w >> 1, hp = w & 1;      // this wave's output tile
  const int al = lane & 31, kk = lane >> 5;
  const int xl = t % GC_CS, rest = t / GC_CS;  // staging: face site and entry
  const int ntv = g.ntv, nc = g.nc;
  const size_t V = g.V, nn = (size_t)nc * nc;

  // raw values of one chunk: the basis at x (rows) and at x + mu (columns)
  // for GC_NQ (spin, chirality, vector) entries, and the link at x
  cx<T> praw[GC_NQ][3], qraw[GC_NQ][3], uraw[3][3];
  T psc[GC_NQ], qsc[GC_NQ];
  auto nsites_of = [&](int mu) { return g.vblock / sel4(g.bs, mu); };
  auto fetch = [&](int mu, int f0) {
    const int bsm = sel4(g.bs, mu);
    int nb[4] = {bc[0], bc[1], bc[2], bc[3]};
    for (int d = 0; d < 4; ++d)
      if (d == mu) nb[d] = nb[d] + 1 == g.NB[d] ? 0 : nb[d] + 1;
    const int cn = block_to_int(g, nb);
    const int f = min(f0 + xl, nsites_of(mu) - 1);
    const int lx = face_site(g, mu, bsm - 1, f);
    const unsigned x = (unsigned)(ci * g.vblock + lx);
    const unsigned y = (unsigned)(cn * g.vblock + lx - (bsm - 1) * sel4(g.lstr, mu));
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) uraw[a][b] = ldc<T>(gv.U + (size_t)(mu * 9 + 3 * a + b) * V, x);
#pragma unroll
    for (int q = 0; q < GC_NQ; ++q) {
      const int r2 = rest + (256 / GC_CS) * q;
      const int sg = r2 & 1, ch = (r2 >> 1) & 1, av = min(r2 >> 2, ntv - 1);
      int spin;
      float pr, pi;
      proj_spin(mu, ch, sg, spin, pr, pi);
      const stc_t<S>* wb = bv.W + (size_t)(av * 12 + 3 * spin) * V;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        praw[q][c] = ldc<T>(wb + (size_t)c * V, x);
        qraw[q][c] = ldc<T>(wb + (size_t)c * V, y);
      }
      if constexpr (is_half<S>()) {
        psc[q] = bv.Wsc[(size_t)av * V + x];
        qsc[q] = bv.Wsc[(size_t)av * V + y];
      } else {
        psc[q] = qsc[q] = (T)1;
      }
    }
  };
  auto store = [&](int mu, int f0) {
    const bool fin = f0 + xl < nsites_of(mu);
#pragma unroll
    for (int q = 0; q < GC_NQ; ++q) {
      const int r2 = rest + (256 / GC_CS) * q;
      const int sg = r2 & 1, ch = (r2 >> 1) & 1, av = r2 >> 2;
      int spin;
      float pr, pi;
      proj_spin(mu, ch, sg, spin, pr, pi);
      const bool ok = fin && av < ntv;
      const T tr = (T)pr, ti = (T)pi;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> pv = psc[q] * praw[q][c];
        cx<T> u = mk((T)0, (T)0);
#pragma unroll
        for (int b = 0; b < 3; ++b) u = cfma(uraw[c][b], qraw[q][b], u);
        u = qsc[q] * u;
        const int row = xl * 6 + sg * 3 + c;
        Ps[ch][row][av] = ok ? mk(tr * pv.r - ti * pv.i, tr * pv.i + ti * pv.r) : mk((T)0, (T)0);
        Qs[ch][row][av] = ok ? mk(tr * u.r - ti * u.i, tr * u.i + ti * u.r) : mk((T)0, (T)0);
      }
    }
  };

  // FP32: one 32x32 tile per wave; FP64: four 16x16 tiles [ti][tj]
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int NACC = F64 ? 4 : 1;
  using Acc = typename std::conditional<F64, gc_v4d, gc_v16>::type;
  constexpr int AV = F64 ? 4 : 16;
  Acc RR[NACC], II[NACC], RI[NACC], IR[NACC];
#pragma unroll
  for (int u = 0; u < NACC; ++u)
#pragma unroll
    for (int v = 0; v < AV; ++v) RR[u][v] = II[u][v] = RI[u][v] = IR[u][v] = (T)0;
  int mu = 0, f0 = 0;
  fetch(0, 0);
  for (;;) {
    __syncthreads();  // the previous chunk has been consumed
    store(mu, f0);
    int nmu = mu, nf0 = f0 + GC_CS;
    if (nf0 >= nsites_of(mu)) {
      nmu = mu + 1;
      nf0 = 0;
    }
    if (nmu < 4) fetch(nmu, nf0);
    __syncthreads();
    if constexpr (F64) {
      const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
      for (int k0 = 0; k0 < GC_ROWS; k0 += 4) {
        cx<T> pv[2], qv[2];
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2) {
          pv[t2] = Ps[h][k0 + k4][16 * t2 + i16];
          qv[t2] = Qs[hp][k0 + k4][16 * t2 + i16];
        }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) {
            Acc* const acc[4] = {&RR[2 * ti + tj], &II[2 * ti + tj], &RI[2 * ti + tj], &IR[2 * ti + tj]};
            *acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[ti].r, qv[tj].r, *acc[0], 0, 0, 0);
            *acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[ti].i, qv[tj].i, *acc[1], 0, 0, 0);
            *acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[ti].r, qv[tj].i, *acc[2], 0, 0, 0);
            *acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[ti].i, qv[tj].r, *acc[3], 0, 0, 0);
          }
      }
    } else {
#pragma unroll
      for (int tt = 0; tt < GC_ROWS / 2; ++tt) {
        const cx<T> pv = Ps[h][2 * tt + kk][al];
        const cx<T> qv = Qs[hp][2 * tt + kk][al];
        RR[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv.r, qv.r, RR[0], 0, 0, 0);
        II[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv.i, qv.i, II[0], 0, 0, 0);
        RI[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv.r, qv.i, RI[0], 0, 0, 0);
        IR[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv.i, qv.r, IR[0], 0, 0, 0);
      }
    }
    if (nmu != mu) {
      // slot 1 + 2 mu done: sum conj(p) q = (RR + II, RI - IR)
      const T coef = (mu == 3 && bc[3] == g.NB[3] - 1) ? (T)0.5 : (T)-0.5;
      cx<T>* out = Dc + ((size_t)ci * 9 + 1 + 2 * mu) * nn + h * ntv;
#pragma unroll
      for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int v = 0; v < AV; ++v) {
          // FP32 32x32 result: row 8 (v / 4) + 4 kk + v % 4, column lane % 32;
          // FP64 16x16 result: row lane / 16 + 4 v, column lane % 16
          const int ai = F64 ? 16 * (u >> 1) + (lane >> 4) + 4 * v : 8 * (v / 4) + 4 * kk + (v % 4);
          const int aj = F64 ? 16 * (u & 1) + (lane & 15) : al;
          if (ai < ntv && aj < ntv)
            out[(size_t)(hp * ntv + aj) * nc + ai] = mk(coef * (RR[u][v] + II[u][v]), coef * (RI[u][v] - IR[u][v]));
          RR[u][v] = II[u][v] = RI[u][v] = IR[u][v] = (T)0;
        }
      if (nmu == 4) break;
    }
    mu = nmu;
    f0 = nf0;
  }
}

}  // namespace

template <typename T, typename S>
void launch_galerkin_cross(cx<T>* Dc, const BasisView<S>& bv, const GaugeView<T>& gv, const Geom& g, hipStream_t st) {
  galerkin_cross_kernel<T, S><<<g.nblocks, 256, 0, st>>>(Dc, bv, gv, g);
}

template void launch_galerkin_cross<float, float>(cx<float>*, const BasisView<float>&, const GaugeView<float>&,
                                                  const Geom&, hipStream_t);
template void launch_galerkin_cross<float, __half>(cx<float>*, const BasisView<__half>&, const GaugeView<float>&,
                                                   const Geom&, hipStream_t);
template void launch_galerkin_cross<double, double>(cx<double>*, const BasisView<double>&, const GaugeView<double>&,
                                                    const Geom&, hipStream_t);

}  // namespace ddamg
