// Fused SAP colour phase (Alg. 3, multiplicative Schwarz reading).
//
// One workgroup per (block of the given colour, rhs); one thread per site of
// the block.  The workgroup
//   1. forms the residual r = y - D x on its sites (the block's x staged in
//      LDS; neighbour values from the other colour come from global memory
//      and are not written in this phase, so there is no race),
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

// Sum over the 64 lanes of a wave by DPP lane moves (no LDS round trips):
// quad sums, then row sums (lanes 15, 31, 47, 63), then the row broadcasts;
// lane 63 ends with the total.
template <int CTRL, int ROWS>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename T>
__device__ inline T wave_sum63(T v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Gauge-field loads of the smoother.  GaugeLd<S, false> reads the planes
// with global loads (a 64-bit address per load and lane); GaugeLd<S, true>
// reads them with buffer loads, one descriptor per link direction and per
// clover chirality, the plane's offset in a scalar register and the site's
// byte offset shared by all loads of a site: no vector instruction per load
// for its address.  A descriptor covers at most 2^31 bytes (checked by the
// launcher) and returns zeros beyond its range instead of faulting.
template <typename S, bool BUF>
struct GaugeLd;

template <typename S>
struct GaugeLd<S, false> {
  GaugeView<S> gv;
  size_t V;
  __device__ GaugeLd(const GaugeView<S>& g, size_t v) : gv(g), V(v) {}
  __device__ void launder() {
    int zero = 0;
    asm volatile("" : "+s"(zero));
    gv.U += zero;
    gv.A += zero;
  }
  template <int MU, typename Tc>
  __device__ void link(cx<Tc> u[3][3], int s) const {
    load_link<Tc, S>(u, gv, MU, s, V);
  }
  template <typename Tc>
  __device__ void clover(cx<Tc> a[CLOVER_PAIRS], int h, int s) const {
    const stc_t<S>* Ah = gv.A + (size_t)h * CLOVER_PAIRS * V;
#pragma unroll
    for (int e = 0; e < CLOVER_PAIRS; ++e) a[e] = ldc<Tc>(Ah + (size_t)e * V, (unsigned)s);
  }
  __device__ float link_scale(int s) const { return gv.Usc[s]; }
  __device__ float clover_scale(int s) const { return gv.Asc[s]; }
};

constexpr int BUF_WORD3 = 0x00020000;  // CDNA buffer descriptor word 3: 32-bit dword format

template <typename X>
__device__ inline X buf_ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  X x;
  if constexpr (sizeof(X) == 4) {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
    __builtin_memcpy(&x, &v, 4);
  } else if constexpr (sizeof(X) == 8) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    __builtin_memcpy(&x, &v, 8);
  } else {
    static_assert(sizeof(X) == 16, "complex entry of 4, 8 or 16 bytes");
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
    __builtin_memcpy(&x, &v, 16);
  }
  return x;
}

template <typename Tc, typename X>
__device__ inline cx<Tc> to_cx(const X& v) {
  if constexpr (std::is_same<X, __half2>::value) {
    const float2 f = __half22float2(v);
    return mk((Tc)f.x, (Tc)f.y);
  } else {
    return mk((Tc)v.r, (Tc)v.i);
  }
}

template <typename S>
struct GaugeLd<S, true> {
  using E = stc_t<S>;
  __amdgpu_buffer_rsrc_t U[4], A[2];
  const float* Usc;
  const float* Asc;
  unsigned plane;  // bytes of one component plane, V entries
  __device__ GaugeLd(const GaugeView<S>& g, size_t V) : Usc(g.Usc), Asc(g.Asc), plane((unsigned)(V * sizeof(E))) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
      U[mu] = __builtin_amdgcn_make_buffer_rsrc((void*)(g.U + (size_t)mu * 9 * V), (short)0, (int)(9 * plane),
                                                BUF_WORD3);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      A[h] = __builtin_amdgcn_make_buffer_rsrc((void*)(g.A + (size_t)h * CLOVER_PAIRS * V), (short)0,
                                               (int)(CLOVER_PAIRS * plane), BUF_WORD3);
  }
  __device__ void launder() { asm volatile("" : "+s"(plane)); }
  template <int MU, typename Tc>
  __device__ void link(cx<Tc> u[3][3], int s) const {
    const unsigned vo = (unsigned)s * (unsigned)sizeof(E);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) u[a][b] = to_cx<Tc>(buf_ld<E>(U[MU], vo, (unsigned)(3 * a + b) * plane));
  }
  template <typename Tc>
  __device__ void clover(cx<Tc> a[CLOVER_PAIRS], int h, int s) const {
    const unsigned vo = (unsigned)s * (unsigned)sizeof(E);
#pragma unroll
    for (int e = 0; e < CLOVER_PAIRS; ++e) a[e] = to_cx<Tc>(buf_ld<E>(h ? A[1] : A[0], vo, (unsigned)e * plane));
  }
  __device__ float link_scale(int s) const { return elem(Usc, (unsigned)s); }
  __device__ float clover_scale(int s) const { return elem(Asc, (unsigned)s); }
};

// Block shape: B4 > 0 is a block of B4^4 sites known at compile time (LDS
// offsets of the neighbours become instruction immediates), B4 = 0 the
// shape of the geometry.
template <int B4>
struct Blk {
  __device__ static int vb(const Geom& g) {
    if constexpr (B4 > 0) return B4 * B4 * B4 * B4;
    else return g.vblock;
  }
  template <int MU>
  __device__ static int bs(const Geom& g) {
    if constexpr (B4 > 0) return B4;
    else return g.bs[MU];
  }
  template <int MU>
  __device__ static int lstr(const Geom& g) {
    if constexpr (B4 > 0) return MU == 0 ? 1 : MU == 1 ? B4 : MU == 2 ? B4 * B4 : B4 * B4 * B4;
    else return g.lstr[MU];
  }
};

// hop of direction MU (forward or backward) for NR spinors, link at slink
template <int MU, bool FWD, int NR, typename T, typename S, typename GL>
__device__ inline void sap_hop(cx<T> acc[NR][4][3], const cx<T> q[NR][4][3], const GL& gl, int slink) {
  cx<T> U[3][3];
  gl.template link<MU, T>(U, slink);
  T coef = (T)-0.5;
  if constexpr (is_half<S>()) coef *= (T)gl.link_scale(slink);
  hop_spinor_multi_u<MU, FWD, NR, T>(acc, q, U, coef);
}

// acc[r] += A(s) p[r] for NR spinors
template <int NR, typename T, typename S, typename GL>
__device__ inline void sap_clover(cx<T> acc[NR][4][3], const cx<T> p[NR][4][3], const GL& gl, int s) {
  T sc = (T)1;
  if constexpr (is_half<S>()) sc = (T)gl.clover_scale(s);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    cx<T> a[CLOVER_PAIRS];
    gl.template clover<T>(a, h, s);
    clover_half_multi<NR, T>(acc, p, a, h, sc);
  }
}

// in-block hops of direction MU for NR residual vectors from LDS
template <int MU, int NR, int B4, typename T, typename S, typename GL>
__device__ inline void block_hops(cx<T> acc[NR][4][3], const cx<T>* lds, const SitePos& p, const Geom& g,
                                  const GL& gl) {
  const int vb = Blk<B4>::vb(g);
  const int ls = Blk<B4>::template lstr<MU>(g);
  cx<T> q[NR][4][3];
  if (p.lc[MU] < Blk<B4>::template bs<MU>(g) - 1) {
    const int ln = p.l + ls;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) q[r][sp][k] = lds[(r * 12 + 3 * sp + k) * vb + ln];
    sap_hop<MU, true, NR, T, S>(acc, q, gl, p.S);
  }
  if (p.lc[MU] > 0) {
    const int ln = p.l - ls;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) q[r][sp][k] = lds[(r * 12 + 3 * sp + k) * vb + ln];
    sap_hop<MU, false, NR, T, S>(acc, q, gl, p.S - ls);
  }
}

// hops of the full operator for NR vectors whose in-block values are staged
// in LDS: a neighbour inside the block is read there, one across the face
// from global memory (the other colour's blocks, not written in this phase)
template <int MU, int NR, int B4, typename T, typename S, typename GL>
__device__ inline void staged_hops(cx<T> acc[NR][4][3], const cx<T>* lds, const cx<T>* x, size_t rs, int nr,
                                   const SitePos& p, const Geom& g, const GL& gl, size_t V) {
  const int vb = Blk<B4>::vb(g);
  const int ls = Blk<B4>::template lstr<MU>(g);
  const bool live = g.V > 0;  // opaque: keeps each hop's loads with its arithmetic
  cx<T> q[NR][4][3];
  if (live) {
    const bool inside = p.lc[MU] < Blk<B4>::template bs<MU>(g) - 1;
    if (inside) {
      const int ln = p.l + ls;
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) q[r][sp][k] = lds[(r * 12 + 3 * sp + k) * vb + ln];
    } else {
      const int sn = nbr_fwd(g, p, MU);
      const bool wrap = MU == 3 && p.bc[3] == g.NB[3] - 1;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        load_spinor<T, T, false>(q[r], x + (size_t)min(r, nr - 1) * rs, sn, V, -1, wrap ? (T)-1 : (T)1);
    }
    sap_hop<MU, true, NR, T, S>(acc, q, gl, p.S);
  }
  asm volatile("" ::: "memory");
  if (live) {
    const bool inside = p.lc[MU] > 0;
    const int sb = nbr_bwd(g, p, MU);
    if (inside) {
      const int ln = p.l - ls;
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) q[r][sp][k] = lds[(r * 12 + 3 * sp + k) * vb + ln];
    } else {
      const bool wrap = MU == 3 && p.bc[3] == 0;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        load_spinor<T, T, false>(q[r], x + (size_t)min(r, nr - 1) * rs, sb, V, -1, wrap ? (T)-1 : (T)1);
    }
    sap_hop<MU, false, NR, T, S>(acc, q, gl, sb);
  }
}

// At least two waves per SIMD: the FP64 instance would otherwise take 262
// registers and run one wave per SIMD (the FP32 ones are below 256 anyway).
// B4 = 4: blocks of 4^4 sites and gauge planes read through buffer
// descriptors; B4 = 0: any block shape, global loads.
template <typename T, typename S, int NR, int B4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sap_phase_kernel(
    cx<T>* __restrict__ x, const cx<T>* __restrict__ y, GaugeView<S> gv, Geom g, int colour, int n_mr, size_t rs,
    int nrhs) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int vb = Blk<B4>::vb(g);
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);          // [NR][12][vb]
  T* red = reinterpret_cast<T*>(lds + NR * 12 * vb);          // [nwaves][3 NR]
  const int nwaves = (blockDim.x + 63) / 64;
  // Workgroup = (block of the colour, group of NR rhs), rhs group fastest so
  // that the workgroups sharing a block's links and clover run side by side.
  // Blocks of one colour are contiguous; the swizzle gives each XCD one
  // contiguous run of them (a compact lattice region and its halo, and the
  // links read by all rhs groups of those blocks stay in that XCD's L2).
  const int ngroup = (nrhs + NR - 1) / NR;
  const int wl = xcd_swizzle(blockIdx.x, gridDim.x);
  const int ci = colour * g.neven + wl / ngroup;
  const int r0 = (wl % ngroup) * NR;
  const int nr = min(NR, nrhs - r0);  // rhs handled by this workgroup
  const int l = threadIdx.x;
  const bool act = l < vb;
  const size_t V = g.V;
  x += (size_t)r0 * rs;
  y += (size_t)r0 * rs;
  GaugeLd<S, (B4 > 0)> gl(gv, V);

  const int s = ci * vb + (act ? l : 0);
  const SitePos pos = site_pos(g, s);
  cx<T> rho[NR][4][3], e[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        rho[r][sp][k] = mk((T)0, (T)0);
        e[r][sp][k] = mk((T)0, (T)0);
      }
  // residual r = y - D x with the current x: the block's x is staged in LDS
  // (the buffer the MR steps use later) for the in-block hops, the halo from
  // the other colour comes from global memory; a missing second rhs repeats
  // the first and is never stored
  if (act) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k)
        lds[(r * 12 + k) * vb + l] = elem(x + (size_t)min(r, nr - 1) * rs + (size_t)k * V, (unsigned)s);
  }
  __syncthreads();
  if (act) {
    cx<T> acc[NR][4][3], p[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          acc[r][sp][k] = mk((T)0, (T)0);
          p[r][sp][k] = lds[(r * 12 + 3 * sp + k) * vb + l];
        }
    sap_clover<NR, T, S>(acc, p, gl, s);
    staged_hops<0, NR, B4, T, S>(acc, lds, x, rs, nr, pos, g, gl, V);
    asm volatile("" ::: "memory");
    staged_hops<1, NR, B4, T, S>(acc, lds, x, rs, nr, pos, g, gl, V);
    asm volatile("" ::: "memory");
    staged_hops<2, NR, B4, T, S>(acc, lds, x, rs, nr, pos, g, gl, V);
    asm volatile("" ::: "memory");
    staged_hops<3, NR, B4, T, S>(acc, lds, x, rs, nr, pos, g, gl, V);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          rho[r][sp][k] = elem(y + (size_t)min(r, nr - 1) * rs + (size_t)(3 * sp + k) * V, (unsigned)s) - acc[r][sp][k];
  }

  __syncthreads();  // every lane is done reading the staged x
  for (int it = 0; it < n_mr; ++it) {
    // Launder the gauge loader: the loads of B below are the same in every
    // MR step, and hoisting them out of the loop would pin them in registers
    // for the whole kernel.
    auto gli = gl;
    gli.launder();
    if (act) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) lds[(r * 12 + 3 * sp + k) * vb + l] = rho[r][sp][k];
    }
    __syncthreads();
    cx<T> q[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) q[r][sp][k] = mk((T)0, (T)0);
    T dots[NR][3];
#pragma unroll
    for (int r = 0; r < NR; ++r) dots[r][0] = dots[r][1] = dots[r][2] = (T)0;
    if (act) {
      sap_clover<NR, T, S>(q, rho, gli, s);
      block_hops<0, NR, B4, T, S>(q, lds, pos, g, gli);
      block_hops<1, NR, B4, T, S>(q, lds, pos, g, gli);
      block_hops<2, NR, B4, T, S>(q, lds, pos, g, gli);
      block_hops<3, NR, B4, T, S>(q, lds, pos, g, gli);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const cx<T> t = cmulc(q[r][sp][k], rho[r][sp][k]);
            dots[r][0] += t.r;
            dots[r][1] += t.i;
            dots[r][2] += q[r][sp][k].r * q[r][sp][k].r + q[r][sp][k].i * q[r][sp][k].i;
          }
    }
    const int w = l >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T v = wave_sum63(dots[r][c]);
        if ((l & 63) == 63) red[w * 3 * NR + 3 * r + c] = v;
      }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T a_re = 0, a_im = 0, n2 = 0;
      for (int k = 0; k < nwaves; ++k) {
        a_re += red[k * 3 * NR + 3 * r + 0];
        a_im += red[k * 3 * NR + 3 * r + 1];
        n2 += red[k * 3 * NR + 3 * r + 2];
      }
      const T inv = n2 > (T)0 ? (T)1 / n2 : (T)0;
      const cx<T> alpha = mk(a_re * inv, a_im * inv);
      if (act) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            e[r][sp][k] = e[r][sp][k] + alpha * rho[r][sp][k];
            rho[r][sp][k] = rho[r][sp][k] - alpha * q[r][sp][k];
          }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) break;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const size_t i = (size_t)r * rs + (size_t)(3 * sp + k) * V + s;
          x[i] = x[i] + e[r][sp][k];
        }
    }
  }
}

}  // namespace

template <typename T, typename S, int NR>
static void launch_sap_nr(cx<T>* x, const cx<T>* y, const GaugeView<S>& gv, const Geom& g, int colour, int n_mr,
                          int nrhs, hipStream_t st) {
  const int threads = ((g.vblock + 63) / 64) * 64;
  const int nwaves = threads / 64;
  const size_t rs = (size_t)12 * g.V;
  const size_t lds = (size_t)NR * 12 * g.vblock * sizeof(cx<T>) + (size_t)3 * NR * nwaves * sizeof(T);
  const int grid = g.nblocks / 2 * ((nrhs + NR - 1) / NR);
  // 4^4 blocks take the specialised kernel when every buffer descriptor
  // (9 link planes of a direction, 18 clover planes of a chirality) stays
  // below 2^31 bytes
  const bool b4 = g.bs[0] == 4 && g.bs[1] == 4 && g.bs[2] == 4 && g.bs[3] == 4;
  const bool fits = (double)CLOVER_PAIRS * (double)g.V * sizeof(stc_t<S>) < 2147483648.0;
  if (b4 && fits)
    sap_phase_kernel<T, S, NR, 4><<<grid, threads, lds, st>>>(x, y, gv, g, colour, n_mr, rs, nrhs);
  else
    sap_phase_kernel<T, S, NR, 0><<<grid, threads, lds, st>>>(x, y, gv, g, colour, n_mr, rs, nrhs);
}

template <typename T, typename S>
void launch_sap_phase(cx<T>* x, const cx<T>* y, const GaugeView<S>& gv, const Geom& g, int colour, int n_mr, int nrhs,
                      hipStream_t st) {
  if (nrhs <= 0) return;
  // FP32 arithmetic on blocks of other shapes: two right-hand sides per
  // thread share every link and clover load.  With 4^4 blocks one rhs per
  // thread: 127 registers, four waves per SIMD instead of two, which hides
  // the LDS and barrier waits of the MR steps better than the shared loads
  // save (measured on 32^3x64 with 12 rhs: 4.87 ms against 5.45 ms per
  // launch).  FP64 keeps one per thread to fit the register file.
  const bool b4 = g.bs[0] == 4 && g.bs[1] == 4 && g.bs[2] == 4 && g.bs[3] == 4;
  if constexpr (sizeof(T) == 4) {
    if (nrhs > 1 && !b4) {
      launch_sap_nr<T, S, 2>(x, y, gv, g, colour, n_mr, nrhs, st);
      return;
    }
  }
  launch_sap_nr<T, S, 1>(x, y, gv, g, colour, n_mr, nrhs, st);
}

template void launch_sap_phase<double, double>(cx<double>*, const cx<double>*, const GaugeView<double>&, const Geom&,
                                               int, int, int, hipStream_t);
template void launch_sap_phase<float, float>(cx<float>*, const cx<float>*, const GaugeView<float>&, const Geom&,
                                             int, int, int, hipStream_t);
template void launch_sap_phase<float, __half>(cx<float>*, const cx<float>*, const GaugeView<__half>&, const Geom&,
                                              int, int, int, hipStream_t);

}  // namespace ddamg
