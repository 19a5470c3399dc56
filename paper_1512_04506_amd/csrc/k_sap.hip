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

// in-block hops of direction MU using rho of the neighbouring sites from LDS
template <int MU, typename T, typename S>
__device__ inline void block_hops(cx<T> acc[4][3], const cx<T>* lds, int vb, const SitePos& p, const Geom& g,
                                  const GaugeView<S>& gv, size_t V) {
  cx<T> q[4][3];
  if (p.lc[MU] < g.bs[MU] - 1) {
    const int ln = p.l + g.lstr[MU];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) q[sp][k] = lds[(3 * sp + k) * vb + ln];
    hop_spinor<MU, true, T, S>(acc, q, gv, p.S, V);
  }
  if (p.lc[MU] > 0) {
    const int ln = p.l - g.lstr[MU];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) q[sp][k] = lds[(3 * sp + k) * vb + ln];
    hop_spinor<MU, false, T, S>(acc, q, gv, p.S - g.lstr[MU], V);
  }
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void sap_phase_kernel(cx<T>* __restrict__ x, const cx<T>* __restrict__ y,
                                                        GaugeView<S> gv, Geom g, int colour, int n_mr, size_t rs) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int vb = g.vblock;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);          // [12][vb]
  T* red = reinterpret_cast<T*>(lds + 12 * vb);               // [nwaves][3]
  const int nwaves = (blockDim.x + 63) / 64;
  // blocks of one colour are contiguous; the swizzle gives each XCD one
  // contiguous run of them (a compact lattice region and its halo)
  const int ci = colour * g.neven + xcd_swizzle(blockIdx.x, gridDim.x);
  const int r = blockIdx.y;
  const int l = threadIdx.x;
  const bool act = l < vb;
  const size_t V = g.V;
  x += (size_t)r * rs;
  y += (size_t)r * rs;

  const int s = ci * vb + (act ? l : 0);
  const SitePos pos = site_pos(g, s);
  cx<T> rho[4][3], e[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rho[sp][k] = mk((T)0, (T)0);
      e[sp][k] = mk((T)0, (T)0);
    }
  if (act) {
    // residual r = y - D x with the current x (global memory)
    cx<T> acc[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[sp][k] = mk((T)0, (T)0);
    cx<T> p[4][3];
    load_spinor<T, T, false>(p, x, s, V, -1, (T)1);
    clover_apply<T, S>(acc, p, gv, s, V);
    hops_all<T, T, S, DS_FULL>(acc, x, gv, g, pos, 0, -1);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) rho[sp][k] = y[(size_t)(3 * sp + k) * V + s] - acc[sp][k];
  }

  for (int it = 0; it < n_mr; ++it) {
    // Launder the link/clover pointers: the loads of B below are the same in
    // every MR step, and hoisting them out of the loop would pin ~200 values
    // in registers for the whole kernel.
    GaugeView<S> gvi = gv;
    asm volatile("" : "+s"(gvi.U), "+s"(gvi.A));
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
      clover_apply<T, S>(q, rho, gvi, s, V);
      block_hops<0, T, S>(q, lds, vb, pos, g, gvi, V);
      block_hops<1, T, S>(q, lds, vb, pos, g, gvi, V);
      block_hops<2, T, S>(q, lds, vb, pos, g, gvi, V);
      block_hops<3, T, S>(q, lds, vb, pos, g, gvi, V);
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
void launch_sap_phase(cx<T>* x, const cx<T>* y, const GaugeView<S>& gv, const Geom& g, int colour, int n_mr, int nrhs,
                      hipStream_t st) {
  if (nrhs <= 0) return;
  int threads = ((g.vblock + 63) / 64) * 64;
  int nwaves = threads / 64;
  size_t lds = (size_t)12 * g.vblock * sizeof(cx<T>) + (size_t)3 * nwaves * sizeof(T);
  dim3 grid(g.nblocks / 2, nrhs);
  sap_phase_kernel<T, S><<<grid, threads, lds, st>>>(x, y, gv, g, colour, n_mr, (size_t)12 * g.V);
}

template void launch_sap_phase<double, double>(cx<double>*, const cx<double>*, const GaugeView<double>&, const Geom&,
                                               int, int, int, hipStream_t);
template void launch_sap_phase<float, float>(cx<float>*, const cx<float>*, const GaugeView<float>&, const Geom&,
                                             int, int, int, hipStream_t);
template void launch_sap_phase<float, __half>(cx<float>*, const cx<float>*, const GaugeView<__half>&, const Geom&,
                                              int, int, int, hipStream_t);

}  // namespace ddamg
