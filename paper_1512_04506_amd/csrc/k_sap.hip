// Fused SAP colour phase (Alg. 3, multiplicative Schwarz reading).
//
// One workgroup per (block of the given colour, rhs); one thread per site of
// the block.  The workgroup
//   1. forms the residual r = y - D x on its sites (neighbour values from
//      the other colour come from global memory and are not written in this
//      phase, so there is no race),
//   2. runs n_mr minimal-residual steps on B e = r, where B is D restricted
//      to the block (hops leaving the block dropped): the current residual
//      rho lives in registers and is exchanged between sites through LDS,
//      the two inner products of each step are workgroup reductions,
//   3. adds the correction e to x on its own sites.
// Blocks of one colour never touch each other, so one launch per colour is
// one Schwarz half-sweep.
#include "dirac_device.h"

namespace ddamg {

namespace {

using namespace dev;

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// in-block hop of direction MU using rho of the neighbouring site from LDS
template <int MU, typename T, typename S>
__device__ inline void block_hops(cx<T> acc[4][3], const cx<T>* lds, int vb, int l, const int lc[4], const int lstr[4],
                                  const Geom& g, int s, const int c[4], const GaugeView<S>& gv, size_t V) {
  cx<T> p[4][3];
  if (lc[MU] < g.bs[MU] - 1) {
    int ln = l + lstr[MU];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) p[sp][k] = lds[(3 * sp + k) * vb + ln];
    hop_spinor<MU, true, T, S>(acc, p, gv, s, V);
  }
  if (lc[MU] > 0) {
    int ln = l - lstr[MU];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) p[sp][k] = lds[(3 * sp + k) * vb + ln];
    int e[4] = {c[0], c[1], c[2], c[3]};
    e[MU] -= 1;  // inside the block: no wrap
    hop_spinor<MU, false, T, S>(acc, p, gv, site_index(g, e), V);
  }
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void sap_phase_kernel(cx<T>* __restrict__ x, const cx<T>* __restrict__ y,
                                                        GaugeView<S> gv, Geom g, const int* __restrict__ colour_blocks,
                                                        int colour, int n_mr, size_t rs) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int vb = g.vblock;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);          // [12][vb]
  T* red = reinterpret_cast<T*>(lds + 12 * vb);               // [nwaves][3]
  const int nwaves = (blockDim.x + 63) / 64;
  const int b = colour_blocks[colour * (g.nblocks / 2) + blockIdx.x];
  const int r = blockIdx.y;
  const int l = threadIdx.x;
  const bool act = l < vb;
  const size_t V = g.V;
  x += (size_t)r * rs;
  y += (size_t)r * rs;

  int c[4] = {0, 0, 0, 0}, lc[4] = {0, 0, 0, 0};
  int s = 0;
  const int lstr[4] = {1, g.bs[0], g.bs[0] * g.bs[1], g.bs[0] * g.bs[1] * g.bs[2]};
  cx<T> rho[4][3], e[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rho[sp][k] = mk((T)0, (T)0);
      e[sp][k] = mk((T)0, (T)0);
    }
  if (act) {
    s = block_site(g, b, l, c);
    int t = l;
    lc[0] = t % g.bs[0]; t /= g.bs[0];
    lc[1] = t % g.bs[1]; t /= g.bs[1];
    lc[2] = t % g.bs[2];
    lc[3] = t / g.bs[2];
    // residual r = y - D x with the current x (global memory)
    cx<T> acc[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[sp][k] = mk((T)0, (T)0);
    cx<T> p[4][3];
    load_spinor<T, T>(p, x, s, V, -1, (T)1);
    clover_apply<T, S>(acc, p, gv, s, V);
    hops_mu<0, T, T, S, DS_FULL>(acc, x, gv, g, c, s, 0, -1);
    hops_mu<1, T, T, S, DS_FULL>(acc, x, gv, g, c, s, 0, -1);
    hops_mu<2, T, T, S, DS_FULL>(acc, x, gv, g, c, s, 0, -1);
    hops_mu<3, T, T, S, DS_FULL>(acc, x, gv, g, c, s, 0, -1);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) rho[sp][k] = y[(size_t)(3 * sp + k) * V + s] - acc[sp][k];
  }

  for (int it = 0; it < n_mr; ++it) {
    if (act) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) lds[(3 * sp + k) * vb + l] = rho[sp][k];
    }
    __syncthreads();
    cx<T> q[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) q[sp][k] = mk((T)0, (T)0);
    T qr_re = 0, qr_im = 0, qq = 0;
    if (act) {
      clover_apply<T, S>(q, rho, gv, s, V);
      block_hops<0, T, S>(q, lds, vb, l, lc, lstr, g, s, c, gv, V);
      block_hops<1, T, S>(q, lds, vb, l, lc, lstr, g, s, c, gv, V);
      block_hops<2, T, S>(q, lds, vb, l, lc, lstr, g, s, c, gv, V);
      block_hops<3, T, S>(q, lds, vb, l, lc, lstr, g, s, c, gv, V);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          cx<T> t = cmulc(q[sp][k], rho[sp][k]);
          qr_re += t.r;
          qr_im += t.i;
          qq += q[sp][k].r * q[sp][k].r + q[sp][k].i * q[sp][k].i;
        }
    }
    qr_re = wave_sum(qr_re);
    qr_im = wave_sum(qr_im);
    qq = wave_sum(qq);
    const int w = l >> 6;
    if ((l & 63) == 0) {
      red[3 * w + 0] = qr_re;
      red[3 * w + 1] = qr_im;
      red[3 * w + 2] = qq;
    }
    __syncthreads();
    T a_re = 0, a_im = 0, n2 = 0;
    for (int k = 0; k < nwaves; ++k) {
      a_re += red[3 * k + 0];
      a_im += red[3 * k + 1];
      n2 += red[3 * k + 2];
    }
    cx<T> alpha = n2 > (T)0 ? mk(a_re / n2, a_im / n2) : mk((T)0, (T)0);
    if (act) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          e[sp][k] = e[sp][k] + alpha * rho[sp][k];
          rho[sp][k] = rho[sp][k] - alpha * q[sp][k];
        }
    }
  }
  if (act) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        size_t i = (size_t)(3 * sp + k) * V + s;
        x[i] = x[i] + e[sp][k];
      }
  }
}

}  // namespace

template <typename T, typename S>
void launch_sap_phase(cx<T>* x, const cx<T>* y, const GaugeView<S>& gv, const Geom& g, const int* colour_blocks,
                      int colour, int n_mr, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  int threads = ((g.vblock + 63) / 64) * 64;
  int nwaves = threads / 64;
  size_t lds = (size_t)12 * g.vblock * sizeof(cx<T>) + (size_t)3 * nwaves * sizeof(T);
  dim3 grid(g.nblocks / 2, nrhs);
  sap_phase_kernel<T, S><<<grid, threads, lds, st>>>(x, y, gv, g, colour_blocks, colour, n_mr, (size_t)12 * g.V);
}

template void launch_sap_phase<double, double>(cx<double>*, const cx<double>*, const GaugeView<double>&, const Geom&,
                                               const int*, int, int, int, hipStream_t);
template void launch_sap_phase<float, float>(cx<float>*, const cx<float>*, const GaugeView<float>&, const Geom&,
                                             const int*, int, int, int, hipStream_t);
template void launch_sap_phase<float, __half>(cx<float>*, const cx<float>*, const GaugeView<__half>&, const Geom&,
                                              const int*, int, int, int, hipStream_t);

}  // namespace ddamg
