// Gauge-covariant network that proposes test vectors for the adaptive
// setup (the random start of Alg. 4 replaced by a learned map), trained on
// the device: layer applies, their transposes (input gradients), weight
// gradients, the span loss against a target aggregate basis (Sec. 2
// aggregates, Alg. 5 basis) with its gradient, and Adam.
//
// Fields are FP32 complex in the internal layout [channel][12][V].  A
// layer's weights are [C_out][C_in][18] complex: k = 0 multiplies phi,
// k = 1 g5 phi, and hop h = 2 mu + s (s = 0 forward, 1 backward) has
// k = 2 + 2h for T_h phi and k = 3 + 2h for g_mu T_h phi, with the parallel
// transports T_mu,+ phi(x) = U_mu(x) phi(x + mu) and T_mu,- phi(x) =
// U_mu(x - mu)^dag phi(x - mu) under the boundary conditions of D.  Between
// layers every channel passes the gate phi / sqrt(1 + |phi(x)|^2 / 12); the
// kernels apply it when they load a hidden layer's stored pre-gate output.
#include <cmath>

#include "dirac_device.h"

namespace ddamg {

namespace {

using namespace dev;
constexpr int NTPB = 256;
constexpr int NFEAT = 18;

// g_mu p in the chiral basis: a signed / phased permutation of the spins
template <int MU>
__device__ inline void gamma_mul(cx<float> o[4][3], const cx<float> p[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 0) {
      o[0][c] = times_mi(p[3][c]);
      o[1][c] = times_mi(p[2][c]);
      o[2][c] = times_i(p[1][c]);
      o[3][c] = times_i(p[0][c]);
    } else if (MU == 1) {
      o[0][c] = neg(p[3][c]);
      o[1][c] = p[2][c];
      o[2][c] = p[1][c];
      o[3][c] = neg(p[0][c]);
    } else if (MU == 2) {
      o[0][c] = times_mi(p[2][c]);
      o[1][c] = times_i(p[3][c]);
      o[2][c] = times_i(p[0][c]);
      o[3][c] = times_mi(p[1][c]);
    } else {
      o[0][c] = neg(p[2][c]);
      o[1][c] = neg(p[3][c]);
      o[2][c] = neg(p[0][c]);
      o[3][c] = neg(p[1][c]);
    }
  }
}

// spinor of one channel (plane base f = channel * 12 V) at internal site s,
// times sign; GATE: the stored value is a pre-gate activation, apply the gate
template <bool GATE>
__device__ inline void load_in(cx<float> p[4][3], const cx<float>* f, int s, size_t V, float sign) {
  float n = 0.f;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p[sp][c] = elem(f + (size_t)(3 * sp + c) * V, (unsigned)s);
      n += p[sp][c].r * p[sp][c].r + p[sp][c].i * p[sp][c].i;
    }
  float sc = sign;
  if (GATE) sc *= 1.f / sqrtf(1.f + n * (1.f / 12.f));
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[sp][c] = sc * p[sp][c];
}

// t = U p (FWD) or U^dag p on the colour index of every spin
template <bool FWD>
__device__ inline void transport(cx<float> t[4][3], const cx<float> p[4][3], const cx<float> U[3][3]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<float> acc = mk(0.f, 0.f);
#pragma unroll
      for (int b = 0; b < 3; ++b) acc = FWD ? cfma(U[a][b], p[sp][b], acc) : cfmac(U[b][a], p[sp][b], acc);
      t[sp][a] = acc;
    }
}

// the transported neighbour of hop (MU, FWD) of channel plane f at site p
template <int MU, bool FWD, bool GATE>
__device__ inline void hop_feature(cx<float> t[4][3], const cx<float>* f, const SitePos& p, const Geom& g,
                                   const GaugeView<float>& gv, size_t V) {
  cx<float> ph[4][3], U[3][3];
  if (FWD) {
    const int sn = nbr_fwd(g, p, MU);
    const bool wrap = MU == 3 && p.lc[3] == g.bs[3] - 1 && p.bc[3] == g.NB[3] - 1;
    load_in<GATE>(ph, f, sn, V, wrap ? -1.f : 1.f);
    load_link<float, float>(U, gv, MU, p.S, V);
  } else {
    const int sb = nbr_bwd(g, p, MU);
    const bool wrap = MU == 3 && p.lc[3] == 0 && p.bc[3] == 0;
    load_in<GATE>(ph, f, sb, V, wrap ? -1.f : 1.f);
    load_link<float, float>(U, gv, MU, sb, V);
  }
  transport<FWD>(t, ph, U);
}

template <int OG>
__device__ inline void mix_hop(cx<float> acc[OG][4][3], const cx<float> t[4][3], const cx<float> gt[4][3],
                               const cx<float>* const w[OG], int k) {
#pragma unroll
  for (int q = 0; q < OG; ++q) {
    const cx<float> cw = w[q][k], dw = w[q][k + 1];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[q][sp][c] = cfma(dw, gt[sp][c], cfma(cw, t[sp][c], acc[q][sp][c]));
  }
}

// hop (MU, FWD) of every input channel for the OG outputs: the link, the
// neighbour index and its boundary sign are loaded once, then each channel's
// neighbour spinor is transported and mixed in (the link loads dominated the
// traffic when they were repeated for every input channel)
template <int MU, bool FWD, int OG, bool GATE>
__device__ inline void layer_hop_all(cx<float> acc[OG][4][3], const cx<float>* in, int cin,
                                     const cx<float>* const w0[OG], const SitePos& p, const Geom& g,
                                     const GaugeView<float>& gv, size_t V) {
  cx<float> U[3][3];
  int sn;
  float sign;
  if (FWD) {
    sn = nbr_fwd(g, p, MU);
    sign = MU == 3 && p.lc[3] == g.bs[3] - 1 && p.bc[3] == g.NB[3] - 1 ? -1.f : 1.f;
    load_link<float, float>(U, gv, MU, p.S, V);
  } else {
    sn = nbr_bwd(g, p, MU);
    sign = MU == 3 && p.lc[3] == 0 && p.bc[3] == 0 ? -1.f : 1.f;
    load_link<float, float>(U, gv, MU, sn, V);
  }
  const int k = 2 + 2 * (2 * MU + (FWD ? 0 : 1));
  for (int j = 0; j < cin; ++j) {
    cx<float> ph[4][3], t[4][3], gt[4][3];
    load_in<GATE>(ph, in + (size_t)j * 12 * V, sn, V, sign);
    transport<FWD>(t, ph, U);
    gamma_mul<MU>(gt, t);
    const cx<float>* w[OG];
#pragma unroll
    for (int q = 0; q < OG; ++q) w[q] = w0[q] + (size_t)j * NFEAT;
    mix_hop<OG>(acc, t, gt, w, k);
  }
  asm volatile("" ::: "memory");
}

// out[i] = sum_jk W[i][j][k] F_k(in_j) for the OG output channels
// i0 .. i0 + OG - 1 of this workgroup (blockIdx.y); one thread per site.
// GATE_IN: the input planes hold pre-gate activations (gate applied on load).
// GATE_BWD: the result is the gradient with respect to the gate's output of
// the channels whose pre-gate values are in pre; store instead the gradient
// with respect to those pre-gate values (the gate's backward).
template <int OG, bool GATE_IN, bool GATE_BWD>
__global__ __launch_bounds__(NTPB) __attribute__((amdgpu_waves_per_eu(3))) void net_layer_kernel(cx<float>* __restrict__ out, const cx<float>* __restrict__ in,
                                                         const cx<float>* __restrict__ W, int cin, int cout,
                                                         GaugeView<float> gv, Geom g,
                                                         const cx<float>* __restrict__ pre) {
  const int s = blockIdx.x * NTPB + threadIdx.x;
  if (s >= g.V) return;
  const int i0 = blockIdx.y * OG;
  const size_t V = g.V;
  const SitePos p = site_pos(g, s);
  cx<float> acc[OG][4][3];
#pragma unroll
  for (int q = 0; q < OG; ++q)
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[q][sp][c] = mk(0.f, 0.f);
  // weights of the OG outputs for input channel 0; channel j is j * NFEAT on
  const cx<float>* w0[OG];
#pragma unroll
  for (int q = 0; q < OG; ++q) w0[q] = W + (size_t)min(i0 + q, cout - 1) * cin * NFEAT;
  for (int j = 0; j < cin; ++j) {
    cx<float> ph[4][3];
    load_in<GATE_IN>(ph, in + (size_t)j * 12 * V, s, V, 1.f);
    // a phi + b g5 phi, g5 = diag(-1, -1, +1, +1)
#pragma unroll
    for (int q = 0; q < OG; ++q) {
      const cx<float> a = w0[q][(size_t)j * NFEAT], b = w0[q][(size_t)j * NFEAT + 1];
      const cx<float> lo = a - b, hi = a + b;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[q][sp][c] = cfma(sp < 2 ? lo : hi, ph[sp][c], acc[q][sp][c]);
    }
  }
  layer_hop_all<0, true, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<0, false, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<1, true, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<1, false, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<2, true, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<2, false, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<3, true, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
  layer_hop_all<3, false, OG, GATE_IN>(acc, in, cin, w0, p, g, gv, V);
#pragma unroll
  for (int q = 0; q < OG; ++q) {
    const int i = i0 + q;
    if (i >= cout) break;
    if (GATE_BWD) {
      // gradient through psi -> psi g(n), n = |psi|^2 / 12, g = (1 + n)^(-1/2):
      // g gam + (rho g'(n) / 6) psi with rho = Re <psi, gam>, g' = -g^3 / 2
      cx<float> ps[4][3];
      float n = 0.f, rho = 0.f;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ps[sp][c] = elem(pre + ((size_t)i * 12 + 3 * sp + c) * V, (unsigned)s);
          n += ps[sp][c].r * ps[sp][c].r + ps[sp][c].i * ps[sp][c].i;
          rho += ps[sp][c].r * acc[q][sp][c].r + ps[sp][c].i * acc[q][sp][c].i;
        }
      const float gg = 1.f / sqrtf(1.f + n * (1.f / 12.f));
      const float cr = rho * (-0.5f * gg * gg * gg) * (1.f / 6.f);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[q][sp][c] = gg * acc[q][sp][c] + cr * ps[sp][c];
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) out[((size_t)i * 12 + 3 * sp + c) * V + s] = acc[q][sp][c];
  }
}

// Wb[j][i][k]: the weights of the transposed layer (input gradients):
// conj(W[i][j][k]) with the hop direction reversed (T_mu,s^dag = T_mu,-s;
// g5 and g_mu are Hermitian and commute with the transports)
__global__ void net_transpose_kernel(cx<float>* Wb, const cx<float>* W, int cin, int cout) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cin * cout * NFEAT) return;
  const int k = e % NFEAT, i = (e / NFEAT) % cout, j = e / (NFEAT * cout);
  int ks = k;
  if (k >= 2) {
    const int h = (k - 2) >> 1, t = (k - 2) & 1;
    ks = 2 + 2 * (h ^ 1) + t;
  }
  Wb[((size_t)j * cout + i) * NFEAT + k] = conj(W[((size_t)i * cin + j) * NFEAT + ks]);
}

__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// <a, b> summed over spin and colour
__device__ inline cx<float> sdot(const cx<float> a[4][3], const cx<float> b[4][3]) {
  cx<float> s = mk(0.f, 0.f);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) s = cfmac(a[sp][c], b[sp][c], s);
  return s;
}

template <int MU, int OG, bool GATE>
__device__ inline void wgrad_hops(cx<float> acc[OG][NFEAT], const cx<float>* f, const cx<float> gm[OG][4][3],
                                  const SitePos& p, const Geom& g, const GaugeView<float>& gv, size_t V) {
  cx<float> t[4][3], gt[4][3];
  hop_feature<MU, true, GATE>(t, f, p, g, gv, V);
  gamma_mul<MU>(gt, t);
#pragma unroll
  for (int q = 0; q < OG; ++q) {
    acc[q][2 + 4 * MU] = acc[q][2 + 4 * MU] + sdot(t, gm[q]);
    acc[q][3 + 4 * MU] = acc[q][3 + 4 * MU] + sdot(gt, gm[q]);
  }
  asm volatile("" ::: "memory");
  hop_feature<MU, false, GATE>(t, f, p, g, gv, V);
  gamma_mul<MU>(gt, t);
#pragma unroll
  for (int q = 0; q < OG; ++q) {
    acc[q][4 + 4 * MU] = acc[q][4 + 4 * MU] + sdot(t, gm[q]);
    acc[q][5 + 4 * MU] = acc[q][5 + 4 * MU] + sdot(gt, gm[q]);
  }
  asm volatile("" ::: "memory");
}

// Partial weight gradients Gamma_w[i][j][k] = sum_x <F_k(in_j)(x), gam_i(x)>
// over the sites of one chunk (blockIdx.x, spt sites per thread), for the
// input channel j and the OG output channels of job blockIdx.y:
// part[(chunk * cout + i) * cin + j][k] (FP64).
template <int OG, bool GATE_IN>
__global__ __launch_bounds__(NTPB) void net_wgrad_kernel(cx<double>* __restrict__ part,
                                                         const cx<float>* __restrict__ in,
                                                         const cx<float>* __restrict__ gam, int cin, int cout,
                                                         GaugeView<float> gv, Geom g, int spt) {
  __shared__ cx<float> red[NTPB / 64][OG * NFEAT];
  const int ngroup = (cout + OG - 1) / OG;
  const int j = blockIdx.y / ngroup, i0 = (blockIdx.y % ngroup) * OG;
  const size_t V = g.V;
  const cx<float>* f = in + (size_t)j * 12 * V;
  cx<float> acc[OG][NFEAT];
#pragma unroll
  for (int q = 0; q < OG; ++q)
#pragma unroll
    for (int k = 0; k < NFEAT; ++k) acc[q][k] = mk(0.f, 0.f);
  const int base = blockIdx.x * spt * NTPB;
  for (int it = 0; it < spt; ++it) {
    const int s = base + it * NTPB + threadIdx.x;
    if (s >= g.V) break;
    const SitePos p = site_pos(g, s);
    cx<float> gm[OG][4][3];
#pragma unroll
    for (int q = 0; q < OG; ++q) {
      const int i = min(i0 + q, cout - 1);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) gm[q][sp][c] = elem(gam + ((size_t)i * 12 + 3 * sp + c) * V, (unsigned)s);
    }
    {
      cx<float> ph[4][3], g5[4][3];
      load_in<GATE_IN>(ph, f, s, V, 1.f);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) g5[sp][c] = sp < 2 ? neg(ph[sp][c]) : ph[sp][c];
#pragma unroll
      for (int q = 0; q < OG; ++q) {
        acc[q][0] = acc[q][0] + sdot(ph, gm[q]);
        acc[q][1] = acc[q][1] + sdot(g5, gm[q]);
      }
    }
    wgrad_hops<0, OG, GATE_IN>(acc, f, gm, p, g, gv, V);
    wgrad_hops<1, OG, GATE_IN>(acc, f, gm, p, g, gv, V);
    wgrad_hops<2, OG, GATE_IN>(acc, f, gm, p, g, gv, V);
    wgrad_hops<3, OG, GATE_IN>(acc, f, gm, p, g, gv, V);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < OG; ++q)
#pragma unroll
    for (int k = 0; k < NFEAT; ++k) {
      const float re = wave_sum_f(acc[q][k].r), im = wave_sum_f(acc[q][k].i);
      if (lane == 0) red[wid][q * NFEAT + k] = mk(re, im);
    }
  __syncthreads();
  for (int e = threadIdx.x; e < OG * NFEAT; e += NTPB) {
    const int q = e / NFEAT, k = e % NFEAT;
    if (i0 + q >= cout) continue;
    cx<double> sum = mk(0.0, 0.0);
    for (int w = 0; w < NTPB / 64; ++w) sum = sum + cvt<double>(red[w][e]);
    part[(((size_t)blockIdx.x * cout + i0 + q) * cin + j) * NFEAT + k] = sum;
  }
}

// grad[e] = 2 sum_chunk part[chunk][e] (dL/dRe w + i dL/dIm w from the
// Wirtinger sums), summed in a fixed order
__global__ void net_wgrad_final_kernel(cx<float>* grad, const cx<double>* part, size_t n, int nchunk) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  cx<double> s = mk(0.0, 0.0);
  for (int c = 0; c < nchunk; ++c) s = s + part[(size_t)c * n + e];
  grad[e] = cvt<float>(2.0 * s);
}

// Span loss of the proposal X against the target basis T on one aggregate
// per workgroup (blockIdx.x = 2 ci + h), N_tv <= 32:
//   G = X^H X, C = X^H T, Z = G^-1 C (Cholesky, FP64),
//   loss_agg = ||T||^2 - Re tr(C^H Z),
//   gam = -scale (T - X Z) Z^H on the aggregate's components.
// Rows of the aggregate: r = 6 l + q, l the site in the block, q = 3 spin'
// + colour with spin = 2 h + spin'.  status is set to 1 if G is not
// positive definite.
constexpr int SL_CHUNK = 32;  // rows staged per pass
__global__ __launch_bounds__(256) void net_span_loss_kernel(cx<float>* __restrict__ gam, double* __restrict__ loss_agg,
                                                            const cx<float>* __restrict__ X,
                                                            const cx<float>* __restrict__ T, Geom g, int ntv,
                                                            double scale, int* status) {
  __shared__ cx<double> Gs[32][33], Cs[32][33], Zs[32][33];
  __shared__ cx<float> xs[SL_CHUNK][32], ts[SL_CHUNK][32];
  __shared__ double tn[32];
  __shared__ int bad;
  const int ci = blockIdx.x >> 1, h = blockIdx.x & 1;
  const size_t V = g.V;
  const int vb = g.vblock, nrow = 6 * vb;
  const int t = threadIdx.x;
  const int np = ntv * ntv;
  if (t == 0) bad = 0;
  // element (row r, vector a) of a field F
  auto at = [&](const cx<float>* F, int r, int a) -> cx<float> {
    const int l = r / 6, q = r - 6 * (r / 6);
    return F[((size_t)a * 12 + 6 * h + q) * V + (size_t)ci * vb + l];
  };
  cx<double> gacc[4], cacc[4];  // pairs t, t + 256, ... (np <= 1024)
  double tacc = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) gacc[u] = cacc[u] = mk(0.0, 0.0);
  for (int r0 = 0; r0 < nrow; r0 += SL_CHUNK) {
    __syncthreads();
    for (int e = t; e < SL_CHUNK * ntv; e += 256) {
      const int rr = e % SL_CHUNK, a = e / SL_CHUNK;
      const int r = r0 + rr;
      xs[rr][a] = r < nrow ? at(X, r, a) : mk(0.f, 0.f);
      ts[rr][a] = r < nrow ? at(T, r, a) : mk(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int pi = t + 256 * u;
      if (pi < np) {
        const int a = pi / ntv, b = pi % ntv;
        for (int rr = 0; rr < SL_CHUNK; ++rr) {
          const cx<double> xa = cvt<double>(xs[rr][a]);
          gacc[u] = cfmac(xa, cvt<double>(xs[rr][b]), gacc[u]);
          cacc[u] = cfmac(xa, cvt<double>(ts[rr][b]), cacc[u]);
        }
      }
    }
    if (t < ntv)
      for (int rr = 0; rr < SL_CHUNK; ++rr) {
        const cx<float> v = ts[rr][t];
        tacc += (double)v.r * v.r + (double)v.i * v.i;
      }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int pi = t + 256 * u;
    if (pi < np) {
      Gs[pi / ntv][pi % ntv] = gacc[u];
      Cs[pi / ntv][pi % ntv] = cacc[u];
    }
  }
  if (t < ntv) tn[t] = tacc;
  __syncthreads();
  // Cholesky G = L L^H in place (lower triangle), one thread
  if (t == 0) {
    for (int k = 0; k < ntv; ++k) {
      double d = Gs[k][k].r;
      for (int m = 0; m < k; ++m) d -= Gs[k][m].r * Gs[k][m].r + Gs[k][m].i * Gs[k][m].i;
      if (!(d > 0.0)) {
        bad = 1;
        break;
      }
      const double lk = sqrt(d);
      Gs[k][k] = mk(lk, 0.0);
      for (int i = k + 1; i < ntv; ++i) {
        cx<double> v = Gs[i][k];
        for (int m = 0; m < k; ++m) v = v - Gs[i][m] * conj(Gs[k][m]);
        Gs[i][k] = (1.0 / lk) * v;
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (t == 0) {
      atomicExch(status, 1);
      loss_agg[blockIdx.x] = 0.0;
    }
    return;
  }
  // Z[:, b] = G^-1 C[:, b] by forward and back substitution, one column per thread
  if (t < ntv) {
    const int b = t;
    cx<double> y[32];
    for (int i = 0; i < ntv; ++i) {
      cx<double> v = Cs[i][b];
      for (int m = 0; m < i; ++m) v = v - Gs[i][m] * y[m];
      y[i] = (1.0 / Gs[i][i].r) * v;
    }
    for (int i = ntv - 1; i >= 0; --i) {
      cx<double> v = y[i];
      for (int m = i + 1; m < ntv; ++m) v = v - conj(Gs[m][i]) * Zs[m][b];
      Zs[i][b] = (1.0 / Gs[i][i].r) * v;
    }
  }
  __syncthreads();
  if (t == 0) {
    double tr = 0.0, tt = 0.0;
    for (int a = 0; a < ntv; ++a) {
      tt += tn[a];
      for (int b = 0; b < ntv; ++b) tr += Cs[a][b].r * Zs[a][b].r + Cs[a][b].i * Zs[a][b].i;
    }
    loss_agg[blockIdx.x] = tt - tr;
  }
  // gradient rows: v = T_r - X_r Z, gam_r = -scale v Z^H
  for (int r = t; r < nrow; r += 256) {
    cx<double> v[32];
    for (int b = 0; b < ntv; ++b) {
      cx<double> s = cvt<double>(at(T, r, b));
      for (int c = 0; c < ntv; ++c) s = s - cvt<double>(at(X, r, c)) * Zs[c][b];
      v[b] = s;
    }
    const int l = r / 6, q = r - 6 * l;
    for (int a = 0; a < ntv; ++a) {
      cx<double> s = mk(0.0, 0.0);
      for (int b = 0; b < ntv; ++b) s = s + v[b] * conj(Zs[a][b]);
      gam[((size_t)a * 12 + 6 * h + q) * V + (size_t)ci * vb + l] = cvt<float>(-scale * s);
    }
  }
}

// out = scale * sum in[i], summed in a fixed order
__global__ void sum_kernel(double* out, const double* in, int n, double scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += in[i];
  *out = scale * s;
}

// Adam on the real and imaginary parts (n reals), bias corrections c1, c2
__global__ void adam_kernel(float* w, float* m, float* v, const float* grad, size_t n, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gr = grad[e];
  const float mm = b1 * m[e] + (1.f - b1) * gr;
  const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
  m[e] = mm;
  v[e] = vv;
  w[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

constexpr int NET_OG = 4;          // output channels per thread in the layer kernel
constexpr int NET_WOG = 2;         // in the weight-gradient kernel

void launch_net_layer(cx<float>* out, const cx<float>* in, const cx<float>* W, int cin, int cout, bool gate_in,
                      const cx<float>* gate_bwd_pre, const GaugeView<float>& gv, const Geom& g, hipStream_t st) {
  const dim3 grid(cdiv(g.V, NTPB), cdiv(cout, NET_OG));
  if (gate_bwd_pre)
    net_layer_kernel<NET_OG, false, true><<<grid, NTPB, 0, st>>>(out, in, W, cin, cout, gv, g, gate_bwd_pre);
  else if (gate_in)
    net_layer_kernel<NET_OG, true, false><<<grid, NTPB, 0, st>>>(out, in, W, cin, cout, gv, g, nullptr);
  else
    net_layer_kernel<NET_OG, false, false><<<grid, NTPB, 0, st>>>(out, in, W, cin, cout, gv, g, nullptr);
}

void launch_net_transpose(cx<float>* Wb, const cx<float>* W, int cin, int cout, hipStream_t st) {
  const int n = cin * cout * NFEAT;
  net_transpose_kernel<<<cdiv(n, 256), 256, 0, st>>>(Wb, W, cin, cout);
}

int net_wgrad_chunks(const Geom& g) { return (int)cdiv(g.V, (size_t)NTPB * NET_WGRAD_SPT); }

void launch_net_wgrad(cx<float>* grad, cx<double>* part, const cx<float>* in, bool gate_in, const cx<float>* gam,
                      int cin, int cout, const GaugeView<float>& gv, const Geom& g, hipStream_t st) {
  const int nchunk = net_wgrad_chunks(g);
  const dim3 grid(nchunk, cin * cdiv(cout, NET_WOG));
  if (gate_in)
    net_wgrad_kernel<NET_WOG, true><<<grid, NTPB, 0, st>>>(part, in, gam, cin, cout, gv, g, NET_WGRAD_SPT);
  else
    net_wgrad_kernel<NET_WOG, false><<<grid, NTPB, 0, st>>>(part, in, gam, cin, cout, gv, g, NET_WGRAD_SPT);
  const size_t n = (size_t)cout * cin * NFEAT;
  net_wgrad_final_kernel<<<cdiv(n, 256), 256, 0, st>>>(grad, part, n, nchunk);
}

void launch_net_span_loss(cx<float>* gam, double* loss_agg, double* loss, const cx<float>* X, const cx<float>* T,
                          const Geom& g, int ntv, int* status, hipStream_t st) {
  const int nagg = 2 * g.nblocks;
  const double scale = 1.0 / ((double)nagg * ntv);
  net_span_loss_kernel<<<nagg, 256, 0, st>>>(gam, loss_agg, X, T, g, ntv, scale, status);
  sum_kernel<<<1, 64, 0, st>>>(loss, loss_agg, nagg, scale);
}

void launch_adam(float* w, float* m, float* v, const float* grad, size_t n, float lr, int64_t step, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)step)));
  adam_kernel<<<cdiv(n, 256), 256, 0, st>>>(w, m, v, grad, n, lr, b1, b2, c1, c2, eps);
}

}  // namespace ddamg
