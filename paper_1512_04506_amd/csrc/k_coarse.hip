// Coarse-grid kernels: restriction y_c = R y (Eq. R), prolongation
// x = P x_c with P = R^dag (Alg. 2), the 9-slot coarse stencil D_c
// (Eq. cgo), dense per-site block products (D_ee^{-1}), the backward
// couplings from the forward ones (Eq. dagger), FP16 quantisation of D_c
// and the inversion of the even self-coupling blocks for the even/odd coarse
// solve.
//
// Coarse vectors are [rhs][coarse site][2 ntv] complex with coarse sites in
// the internal order (even parity first).  D_c is [site][slot][col][row]
// (column-major 2ntv x 2ntv blocks) so that the lanes of a wave, one per row,
// read consecutive addresses for every column.
#include "ddamg_internal.h"

namespace ddamg {

namespace {

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ----------------------------------------------------------- restriction
// One workgroup per block, one lane per site of the block (its sites are
// contiguous in the block-major layout, so every load is coalesced).  For a
// tile of RT right-hand sides (kept in registers) and AT test vectors at a
// time each lane forms the 6-component partial products of its site for
// both chiralities; the 64 lanes of a wave are then summed by a butterfly
// reduce-scatter (63 shuffle-adds for 32 values) and the waves through LDS.
// Register tiles: RT right-hand sides x AT test vectors per pass, NV real
// partial sums per lane (smaller in FP64 to stay within the register file).
template <typename T>
struct RTile {
  static constexpr int RT = sizeof(T) == 8 ? 2 : 4;
  static constexpr int AT = sizeof(T) == 8 ? 1 : 2;
  static constexpr int NV = AT * 2 * RT * 2;
};

// One halving step of the butterfly, unrolled at compile time so that every
// register index is static: lanes with bit HALF set keep the upper half of
// their values and receive the partner's upper half, the others the lower.
template <int HALF, int NV, typename T>
__device__ inline void rs_step(T v[NV], int lane) {
  const bool up = (lane & HALF) != 0;
#pragma unroll
  for (int j = 0; j < HALF; ++j) {
    const T send = up ? v[j] : v[j + HALF];
    const T keep = up ? v[j + HALF] : v[j];
    v[j] = keep + __shfl_xor(send, HALF, 64);
  }
  if constexpr (HALF > 1) rs_step<HALF / 2, NV, T>(v, lane);
}

// v[0..NV-1] (NV a power of two <= 32): after the call lane i holds the sum
// over the 64 lanes of v[i % NV] (full sums over the lane bits >= NV first,
// then a reduce-scatter over the lower bits)
template <int NV, typename T>
__device__ inline T reduce_scatter(T v[NV], int lane) {
#pragma unroll
  for (int o = 32; o >= NV; o >>= 1)
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += __shfl_xor(v[j], o, 64);
  rs_step<NV / 2, NV, T>(v, lane);
  return v[0];
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void restrict_kernel(cx<T>* __restrict__ out, size_t ostr_r, size_t ostr_b,
                                                       const cx<T>* __restrict__ y, size_t ystr, BasisView<S> bv,
                                                       Geom g, int nrhs, int face_mu) {
  constexpr int RT = RTile<T>::RT, AT = RTile<T>::AT, NV = RTile<T>::NV;
  constexpr int MAXAT = 32 / AT;  // ntv <= 32
  __shared__ T red[4][MAXAT][NV];
  const int ci = blockIdx.x;
  const int l = threadIdx.x;
  const int lane = l & 63, w = l >> 6;
  const int nw = blockDim.x >> 6;
  const bool act = l < g.vblock;
  const size_t V = g.V;
  const size_t site = (size_t)ci * g.vblock + (act ? l : 0);
  const int nat = (g.ntv + AT - 1) / AT;
  bool onface = true;  // face_mu >= 0: only the last layer in direction face_mu holds data
  if (face_mu >= 0) {
    int lc[4];
    local_coords(g, act ? l : 0, lc);
    onface = lc[face_mu] == g.bs[face_mu] - 1;
  }
  for (int r0 = 0; r0 < nrhs; r0 += RT) {
    const int nr = min(RT, nrhs - r0);
    // Every load below is unconditional (clamped to valid addresses and
    // masked by a factor instead): a load guarded by a value that is itself
    // loaded would serialise the memory accesses of the whole loop.
    cx<T> yv[RT][12];
#pragma unroll
    for (int j = 0; j < RT; ++j) {
      const bool m = act && j < nr && onface;
      const size_t r = (size_t)min(r0 + j, nrhs - 1);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<T> v = y[r * ystr + (size_t)k * V + site];
        yv[j][k] = m ? v : mk((T)0, (T)0);  // a select: the other layers may hold stale values
      }
    }
    // no barrier inside this loop: each wave parks its reduced values per
    // test-vector tile and runs ahead
    for (int at = 0; at < nat; ++at) {
      const int a0 = at * AT;
      T v[NV];
#pragma unroll
      for (int q = 0; q < AT; ++q) {
        const int a = min(a0 + q, g.ntv - 1);
        T sc = (act && a0 + q < g.ntv) ? (T)1 : (T)0;
        if constexpr (is_half<S>()) sc *= (T)bv.Wsc[(size_t)a * V + site];
        cx<T> wv[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) wv[k] = sc * ldc<T>(bv.W, ((size_t)a * 12 + k) * V + site);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int j = 0; j < RT; ++j) {
            cx<T> acc = mk((T)0, (T)0);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc = acc + cmulc(wv[6 * h + k], yv[j][6 * h + k]);
            const int idx = ((q * 2 + h) * RT + j) * 2;
            v[idx] = acc.r;
            v[idx + 1] = acc.i;
          }
      }
      const T mine = reduce_scatter<NV, T>(v, lane);
      if (lane < NV) red[w][at][lane] = mine;
    }
    __syncthreads();
    for (int e = l; e < nat * NV; e += blockDim.x) {
      const int at = e / NV, idx = e % NV;
      T t = (T)0;
      for (int k = 0; k < nw; ++k) t += red[k][at][idx];
      // idx = ((q * 2 + h) * RT + j) * 2 + part
      const int part = idx & 1, j = (idx >> 1) % RT, h = (idx / (2 * RT)) & 1, q = idx / (4 * RT);
      const int a = at * AT + q;
      if (a < g.ntv && j < nr) {
        T* o = reinterpret_cast<T*>(out + (size_t)(r0 + j) * ostr_r + (size_t)ci * ostr_b + h * g.ntv + a);
        o[part] = t;
      }
    }
    __syncthreads();
  }
}

// Restriction on the FP32 matrix cores, for many right-hand sides: per
// block and chirality h, C (ntv x 32 rhs) = W_h^H Y_h is a GEMM over the rows
// (site, spin-colour of chirality h).  v_mfma_f32_32x32x2f32 takes A[i][k]
// in lane i + 32 k and B[k][j] in lane j + 32 k and leaves C[i][j] in lane
// j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.  The sites along k
// cannot be spread over the lanes, so chunks of RM_CS sites are first read
// with coalesced site-contiguous loads into LDS (basis scaled to FP32, rows
// (site, component)), then fed to the MFMAs from there.  The complex
// product takes four real GEMMs: conj(W) Y = (Wr Yr + Wi Yi) + i (Wr Yi -
// Wi Yr).  Waves 2h and 2h+1 take the two halves of each chunk's rows of
// chirality h and are summed through LDS at the end.
typedef float mf_v16 __attribute__((ext_vector_type(16)));
constexpr int RM_CS = 8;                  // sites per chunk
constexpr int RM_ROWS = RM_CS * 6;        // rows per chirality and chunk
constexpr int RM_LD = 33;                 // padded row length (float2) in LDS
constexpr int RESTRICT_MFMA_MIN_RHS = 16;  // fewer rhs: the VALU kernel (an MFMA tile holds 32)

template <typename S>
__global__ __launch_bounds__(256) void restrict_mfma_kernel(cx<float>* __restrict__ out, size_t ostr_r, size_t ostr_b,
                                                            const cx<float>* __restrict__ y, size_t ystr,
                                                            BasisView<S> bv, Geom g, int nrhs, int face_mu) {
  __shared__ float2 Ws[2][RM_ROWS][RM_LD];  // [h][row][a]
  __shared__ float2 Ys[2][RM_ROWS][RM_LD];  // [h][row][rhs]
  // [h][re, im][register][lane] of the upper-half waves, in the basis
  // staging area once the chunks are done (three workgroups fit a CU)
  static_assert(sizeof(float) * 2 * 2 * 16 * 64 <= sizeof(float2) * 2 * RM_ROWS * RM_LD, "reduction area");
  auto red = reinterpret_cast<float(*)[2][16][64]>(&Ws[0][0][0]);
  const int ci = blockIdx.x;
  const int col0 = blockIdx.y * 32;
  const int l = threadIdx.x, lane = l & 63, w = l >> 6;
  const int h = w >> 1, kh = w & 1;
  const int ntv = g.ntv;
  const int ncol = min(32, nrhs - col0);
  const size_t V = g.V;
  const size_t base = (size_t)ci * g.vblock;
  const int nsites = face_mu < 0 ? g.vblock : g.vblock / g.bs[face_mu];
  // padding columns stay zero
  for (int e = l; e < 2 * RM_ROWS * RM_LD; e += 256) {
    (&Ws[0][0][0])[e] = make_float2(0.f, 0.f);
    (&Ys[0][0][0])[e] = make_float2(0.f, 0.f);
  }
  mf_v16 RR, II, RI, IR;
#pragma unroll
  for (int v = 0; v < 16; ++v) RR[v] = II[v] = RI[v] = IR[v] = 0.f;
  const int a = lane & 31, kk = lane >> 5;
  // staging: lane (site xl of the chunk, test vector / rhs index idx) loads
  // all 12 components of its basis vector and of its rhs at that site (the
  // scale once); lanes 8 apart in idx, consecutive in xl, so each load is
  // 8-site runs
  static_assert(RM_CS * 32 == 256, "one (site, index) pair per lane");
  const int xl = l % RM_CS, idx = l / RM_CS;
  const bool wok = idx < ntv, yok = idx < ncol;
  const int ia = min(idx, ntv - 1), ir = min(idx, ncol - 1);
  stc_t<S> wraw[12];
  cx<float> yraw[12];
  float sraw = 1.f;
  auto fetch = [&](int f0) {
    const int f = min(f0 + xl, nsites - 1);
    const unsigned x = (unsigned)(base + (face_mu < 0 ? f : face_site(g, face_mu, g.bs[face_mu] - 1, f)));
    const stc_t<S>* wb = bv.W + (size_t)ia * 12 * V;
    const cx<float>* yb = y + (size_t)(col0 + ir) * ystr;
#pragma unroll
    for (int comp = 0; comp < 12; ++comp) {
      wraw[comp] = elem(wb + (size_t)comp * V, x);
      yraw[comp] = elem(yb + (size_t)comp * V, x);
    }
    if constexpr (is_half<S>()) sraw = elem(bv.Wsc + (size_t)ia * V, x);
  };
  fetch(0);
  for (int f0 = 0; f0 < nsites; f0 += RM_CS) {
    __syncthreads();  // previous chunk consumed (and the zero fill done)
    {
      const bool fin = f0 + xl < nsites;
#pragma unroll
      for (int comp = 0; comp < 12; ++comp) {
        const cx<float> wv = ldc<float>(&wraw[comp], (size_t)0);
        Ws[comp / 6][xl * 6 + comp % 6][idx] =
            (fin && wok) ? make_float2(sraw * wv.r, sraw * wv.i) : make_float2(0.f, 0.f);
        Ys[comp / 6][xl * 6 + comp % 6][idx] = (fin && yok) ? make_float2(yraw[comp].r, yraw[comp].i) : make_float2(0.f, 0.f);
      }
    }
    if (f0 + RM_CS < nsites) fetch(f0 + RM_CS);
    __syncthreads();
    // rows 2t, 2t+1 of chirality h; this wave takes half of the chunk
#pragma unroll
    for (int t = kh * (RM_ROWS / 4); t < (kh + 1) * (RM_ROWS / 4); ++t) {
      const float2 wv = Ws[h][2 * t + kk][a];
      const float2 yv = Ys[h][2 * t + kk][a];
      RR = __builtin_amdgcn_mfma_f32_32x32x2f32(wv.x, yv.x, RR, 0, 0, 0);
      II = __builtin_amdgcn_mfma_f32_32x32x2f32(wv.y, yv.y, II, 0, 0, 0);
      RI = __builtin_amdgcn_mfma_f32_32x32x2f32(wv.x, yv.y, RI, 0, 0, 0);
      IR = __builtin_amdgcn_mfma_f32_32x32x2f32(wv.y, yv.x, IR, 0, 0, 0);
    }
  }
  __syncthreads();  // every wave is done with the staging area
  if (kh == 1) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      red[h][0][v][lane] = RR[v] + II[v];
      red[h][1][v][lane] = RI[v] - IR[v];
    }
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ai = 8 * (v / 4) + 4 * kk + (v % 4);
      const int r = lane & 31;
      if (ai < ntv && r < ncol)
        out[(size_t)(col0 + r) * ostr_r + (size_t)ci * ostr_b + h * ntv + ai] =
            mk(RR[v] + II[v] + red[h][0][v][lane], RI[v] - IR[v] + red[h][1][v][lane]);
    }
  }
}

// The FP64 restriction of many rhs on the FP64 matrix cores (16x16x4
// MFMA).  Workgroup = (block, 32 rhs); wave = (chirality h, tile of 16 test
// vectors), each over both 16-rhs tiles and every staged chunk, so no
// partial sums cross waves.  Chunks of RD_CS sites (rows: site x component
// of chirality h) are staged in LDS as in the FP32 kernel, the next chunk's
// loads in flight during the products.
typedef double rd_v4 __attribute__((ext_vector_type(4)));
constexpr int RD_CS = 4;
constexpr int RD_ROWS = RD_CS * 6;
constexpr int RESTRICT_MFMA64_MIN_RHS = 4;

__global__ __launch_bounds__(256) void restrict_mfma64_kernel(cx<double>* __restrict__ out, size_t ostr_r,
                                                              size_t ostr_b, const cx<double>* __restrict__ y,
                                                              size_t ystr, BasisView<double> bv, Geom g, int nrhs,
                                                              int face_mu) {
  __shared__ cx<double> Ws[2][RD_ROWS][RM_LD];  // [h][row][a]
  __shared__ cx<double> Ys[2][RD_ROWS][RM_LD];  // [h][row][rhs]
  const int ci = blockIdx.x;
  const int col0 = blockIdx.y * 32;
  const int l = threadIdx.x, lane = l & 63, w = l >> 6;
  const int h = w >> 1, ti = w & 1;
  const int ntv = g.ntv;
  const int ncol = min(32, nrhs - col0);
  const size_t V = g.V;
  const size_t base = (size_t)ci * g.vblock;
  const int nsites = face_mu < 0 ? g.vblock : g.vblock / g.bs[face_mu];
  rd_v4 RR[2], II[2], RI[2], IR[2];
#pragma unroll
  for (int tj = 0; tj < 2; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) RR[tj][v] = II[tj][v] = RI[tj][v] = IR[tj][v] = 0.0;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int nW = 12 * ntv * RD_CS, nY = 12 * ncol * RD_CS;
  constexpr int NQ = (12 * 32 * RD_CS + 255) / 256;
  cx<double> wraw[NQ], yraw[NQ];
  auto fetch = [&](int f0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = l + 256 * q;
      const int xl = e % RD_CS, rest = e / RD_CS, comp = rest % 12, idx = rest / 12;
      const int f = min(f0 + xl, nsites - 1);
      const size_t x = base + (face_mu < 0 ? f : face_site(g, face_mu, g.bs[face_mu] - 1, f));
      const int ia = min(idx, ntv - 1), ir = min(idx, ncol - 1);
      wraw[q] = bv.W[((size_t)ia * 12 + comp) * V + x];
      yraw[q] = y[(size_t)(col0 + ir) * ystr + (size_t)comp * V + x];
    }
  };
  fetch(0);
  for (int f0 = 0; f0 < nsites; f0 += RD_CS) {
    __syncthreads();  // previous chunk consumed
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = l + 256 * q;
      const int xl = e % RD_CS, rest = e / RD_CS, comp = rest % 12, idx = rest / 12;
      const bool fin = f0 + xl < nsites;
      if (idx < 32) {
        Ws[comp / 6][xl * 6 + comp % 6][idx] = (fin && e < nW) ? wraw[q] : mk(0.0, 0.0);
        Ys[comp / 6][xl * 6 + comp % 6][idx] = (fin && e < nY) ? yraw[q] : mk(0.0, 0.0);
      }
    }
    if (f0 + RD_CS < nsites) fetch(f0 + RD_CS);
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < RD_ROWS; k0 += 4) {
      const cx<double> wv = Ws[h][k0 + k4][16 * ti + i16];
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        const cx<double> yv = Ys[h][k0 + k4][16 * tj + i16];
        RR[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv.r, yv.r, RR[tj], 0, 0, 0);
        II[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv.i, yv.i, II[tj], 0, 0, 0);
        RI[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv.r, yv.i, RI[tj], 0, 0, 0);
        IR[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv.i, yv.r, IR[tj], 0, 0, 0);
      }
    }
  }
  // conj(w) y = (RR + II, RI - IR); result row lane / 16 + 4 v, column lane % 16
#pragma unroll
  for (int tj = 0; tj < 2; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * ti + k4 + 4 * v, r = 16 * tj + i16;
      if (a < ntv && r < ncol)
        out[(size_t)(col0 + r) * ostr_r + (size_t)ci * ostr_b + h * ntv + a] =
            mk(RR[tj][v] + II[tj][v], RI[tj][v] - IR[tj][v]);
    }
}

// ---------------------------------------------------------- prolongation
// x[r](site, k) = sum_a W_a(site, k) x_c[r](block, h(k), a).  Workgroup =
// (block, group of KP spin-colour components of one chirality h), the group
// fastest so that the workgroups of a block (which share its scales) run
// side by side on one XCD; one lane per site.  Each basis entry is loaded
// once per pass of PT rhs and feeds them all; the block's coarse vectors of
// chirality h sit in LDS and each broadcast read feeds the KP components
// (three in FP32; one in FP64, for the register file).
constexpr int PT = 12;  // rhs per pass of the prolongation
template <typename T>
constexpr int prolong_kp() { return sizeof(T) == 8 ? 1 : 3; }

template <typename T, typename S>
__global__ __launch_bounds__(256) void prolong_kernel(cx<T>* __restrict__ x, size_t xstr, const cx<T>* __restrict__ xc,
                                                      size_t cstr, BasisView<S> bv, Geom g, int nrhs) {
  constexpr int KP = prolong_kp<T>(), NG = 12 / KP;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  cx<T>* xl = reinterpret_cast<cx<T>*>(smem_raw);  // [nrhs][ntv] of chirality h
  const int wl = xcd_swizzle(blockIdx.x, gridDim.x);
  const int ci = wl / NG, k0 = (wl % NG) * KP, h = k0 / 6;
  const int l = threadIdx.x;
  const int ntv = g.ntv;
  const size_t V = g.V;
  for (int e = l; e < nrhs * ntv; e += blockDim.x) {
    const int r = e / ntv, a = e % ntv;
    xl[e] = xc[(size_t)r * cstr + (size_t)ci * g.nc + h * ntv + a];
  }
  __syncthreads();
  if (l >= g.vblock) return;
  const unsigned site = (unsigned)(ci * g.vblock + l);
  for (int r0 = 0; r0 < nrhs; r0 += PT) {
    const int nr = min(PT, nrhs - r0);
    cx<T> acc[PT][KP];
#pragma unroll
    for (int j = 0; j < PT; ++j)
#pragma unroll
      for (int q = 0; q < KP; ++q) acc[j][q] = mk((T)0, (T)0);
#pragma unroll 2
    for (int a = 0; a < ntv; ++a) {
      T sc = (T)1;
      if constexpr (is_half<S>()) sc = (T)elem(bv.Wsc + (size_t)a * V, site);
      cx<T> wv[KP];
#pragma unroll
      for (int q = 0; q < KP; ++q) wv[q] = sc * ldc<T>(bv.W + ((size_t)a * 12 + k0 + q) * V, site);
#pragma unroll
      for (int j = 0; j < PT; ++j) {
        if (j < nr) {
          const cx<T> c = xl[(r0 + j) * ntv + a];
#pragma unroll
          for (int q = 0; q < KP; ++q) acc[j][q] = acc[j][q] + wv[q] * c;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PT; ++j)
      if (j < nr)
#pragma unroll
        for (int q = 0; q < KP; ++q) x[(size_t)(r0 + j) * xstr + (size_t)(k0 + q) * V + site] = acc[j][q];
  }
}

// ------------------------------------------------------------ D_c stencil
// One workgroup per (output coarse site, group of RB right-hand sides).
// Thread (row group, cg) accumulates RP consecutive rows over the columns
// col = cg (mod CG) of every slot, so each input value read from LDS (a
// broadcast) feeds RP rows; each slot's input vectors are staged in LDS,
// and the CG partial sums of a row are combined through LDS at the end.
// RP = 2 for few rhs (the D_c stream), 1 for 12 rhs (the partial sums of
// two rows would cost occupancy).
//   out = add + cs D_self xs + cn sum_{slot>0} D_slot xn(nbr)
// With Dmat != nullptr the kernel instead computes out = Dmat[k] x[k] for
// dense column-major per-site matrices (the even-site D_ee^{-1}).
template <typename T, typename S, int RB, int RP>
__global__ __launch_bounds__(256) void coarse_stencil_kernel(cx<T>* __restrict__ out, size_t ostr, int out_first,
                                                             const cx<T>* __restrict__ add, size_t astr,
                                                             const cx<T>* __restrict__ xs, size_t xsstr, int xs_first,
                                                             T cs, const cx<T>* __restrict__ xn, size_t xnstr,
                                                             int xn_first, T cn, CoarseView<S> cv,
                                                             const cx<T>* __restrict__ Dmat, int nc, int CG,
                                                             int nrhs, const int* gate) {
  if (gate && *gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  cx<T>* xl = reinterpret_cast<cx<T>*>(smem_raw);  // [nc][RB], later [CG][nc][RB]
  const int ci = out_first + blockIdx.x;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const int t = threadIdx.x;
  const int ngr = nc / RP;  // nc = 2 ntv is even
  const int rg = t % ngr, cg = t / ngr;
  const bool act = cg < CG;
  const int row = RP * rg;
  const size_t nn = (size_t)nc * nc;
  cx<T> acc[RP][RB];
#pragma unroll
  for (int q = 0; q < RP; ++q)
#pragma unroll
    for (int j = 0; j < RB; ++j) acc[q][j] = mk((T)0, (T)0);
  const int s_beg = Dmat ? 0 : (cs != (T)0 ? 0 : 1);
  const int s_end = Dmat ? 1 : (cn != (T)0 ? 9 : 1);
  for (int slot = s_beg; slot < s_end; ++slot) {
    const int nb = slot == 0 ? ci : cv.nbr[ci * 9 + slot];
    const cx<T>* xv = slot == 0 ? xs + (size_t)(nb - xs_first) * nc : xn + (size_t)(nb - xn_first) * nc;
    const size_t xstr = slot == 0 ? xsstr : xnstr;
    T coef = slot == 0 ? cs : cn;
    if (Dmat) coef = (T)1;
    if constexpr (is_half<S>()) {
      if (!Dmat) coef *= (T)cv.Dsc[ci * 9 + slot];
    }
    __syncthreads();
    for (int e = t; e < nc * nr; e += blockDim.x) {
      const int col = e / nr, j = e % nr;
      xl[col * RB + j] = xv[(size_t)(r0 + j) * xstr + col];
    }
    __syncthreads();
    if (act) {
      for (int col = cg; col < nc; col += CG) {
        cx<T> d[RP];
        if (Dmat) {
          const cx<T>* Mk = Dmat + (size_t)(ci - out_first) * nn + (size_t)col * nc + row;
#pragma unroll
          for (int q = 0; q < RP; ++q) d[q] = Mk[q];
        } else {
          const size_t base = ((size_t)ci * 9 + slot) * nn + (size_t)col * nc + row;
#pragma unroll
          for (int q = 0; q < RP; ++q) d[q] = coef * ldc<T>(cv.D, base + q);
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          if (j < nr) {
            const cx<T> xj = xl[col * RB + j];
#pragma unroll
            for (int q = 0; q < RP; ++q) acc[q][j] = acc[q][j] + d[q] * xj;
          }
        }
      }
    }
  }
  __syncthreads();
  if (act)
#pragma unroll
    for (int q = 0; q < RP; ++q)
#pragma unroll
      for (int j = 0; j < RB; ++j) xl[((size_t)cg * nc + row + q) * RB + j] = acc[q][j];
  __syncthreads();
  for (int e = t; e < nc * nr; e += blockDim.x) {
    const int rw = e / nr, j = e % nr;
    cx<T> sum = add ? add[(size_t)(r0 + j) * astr + (size_t)(ci - out_first) * nc + rw] : mk((T)0, (T)0);
    for (int k = 0; k < CG; ++k) sum = sum + xl[((size_t)k * nc + rw) * RB + j];
    out[(size_t)(r0 + j) * ostr + (size_t)(ci - out_first) * nc + rw] = sum;
  }
}

// The same stencil (without Dmat) for many rhs in FP32 on the matrix cores:
// 16x16x4 MFMA with a tile of 16 rows of D_c per wave, up to 16 rhs as the
// columns and the components of the neighbour as K.  The A operand (16
// consecutive rows of one column of a column-major slot block) and the B
// operand (4 components of 16 rhs of the neighbour vector, an L2-resident
// read) come straight from memory; the slot's factor (and FP16 scale) is
// applied to B.  At 12 rhs the FP32 multiply-adds per byte of D_c are above
// what the vector ALUs sustain at HBM rate; on the matrix cores the stencil
// streams D_c.  The workgroup is one coarse site and 16 rhs, one wave per
// row tile.
typedef float cm_v4 __attribute__((ext_vector_type(4)));
constexpr int CM_RHS = 16;

template <typename S>
__global__ __launch_bounds__(256) void coarse_mfma_kernel(cx<float>* __restrict__ out, size_t ostr, int out_first,
                                                          const cx<float>* __restrict__ add, size_t astr,
                                                          const cx<float>* __restrict__ xs, size_t xsstr,
                                                          int xs_first, float cs, const cx<float>* __restrict__ xn,
                                                          size_t xnstr, int xn_first, float cn, CoarseView<S> cv,
                                                          int nc, int nrhs, const int* gate) {
  if (gate && *gate == 0) return;
  const int ci = out_first + blockIdx.x;
  const int r0 = blockIdx.y * CM_RHS;
  const int nr = min(CM_RHS, nrhs - r0);
  const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int arow = min(rt * 16 + li, nc - 1);  // A: row li of the tile (clamped)
  const int bj = min(li, nr - 1);               // B: rhs li (clamped)
  const size_t nn = (size_t)nc * nc;
  cm_v4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
  const int s_beg = cs != 0.f ? 0 : 1;
  const int s_end = cn != 0.f ? 9 : 1;
  for (int slot = s_beg; slot < s_end; ++slot) {
    const int nb = slot == 0 ? ci : cv.nbr[ci * 9 + slot];
    const cx<float>* xv = slot == 0 ? xs + (size_t)(nb - xs_first) * nc + (size_t)(r0 + bj) * xsstr
                                    : xn + (size_t)(nb - xn_first) * nc + (size_t)(r0 + bj) * xnstr;
    float coef = slot == 0 ? cs : cn;
    if constexpr (is_half<S>()) coef *= cv.Dsc[ci * 9 + slot];
    const stc_t<S>* Dp = cv.D + ((size_t)ci * 9 + slot) * nn + arow;
#pragma unroll 4
    for (int k0 = 0; k0 < nc; k0 += 4) {
      const int k = k0 + lk;
      const bool kin = k < nc;
      const int kc = kin ? k : nc - 1;
      const cx<float> a = ldc<float>(Dp, (size_t)kc * nc);
      const cx<float> xb = xv[kc];
      const float br = kin ? coef * xb.r : 0.f, bi = kin ? coef * xb.i : 0.f;
      accr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r, br, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.i, bi, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r, bi, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.i, br, acci, 0, 0, 0);
    }
  }
  // lane: rows 4 lk + v of the tile, rhs li
  if (li < nr) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rt * 16 + 4 * lk + v;
      if (row < nc) {
        cx<float> o = mk(accr[v], acci[v]);
        if (add) o = o + add[(size_t)(r0 + li) * astr + (size_t)(ci - out_first) * nc + row];
        out[(size_t)(r0 + li) * ostr + (size_t)(ci - out_first) * nc + row] = o;
      }
    }
  }
}

// The same stencil for many rhs when D_c is stored in FP16: on the f16
// matrix cores (v_mfma_f32_16x16x16_f16), which take D_c as it is stored.
// The FP32 input vectors are split into two FP16 parts per element, x s =
// hi + lo 2^-11 with hi = f16(x s) and lo = f16((x s - hi) 2^11), where s
// is a power of two per rhs that brings the largest |coef D_scale x| over
// the nine neighbour vectors of the workgroup into [1/2, 1): the two
// products then carry the input to within 2^-22 of its largest element,
// the FP32 accumulation is exact to FP32 rounding, and the matrix cores
// are no longer the bound (16 K per instruction instead of 4).  Complex
// arithmetic in real form: Yr = Ar Xr - Ai Xi, Yi = Ai Xr + Ar Xi, every
// loaded D_c element feeding eight MFMAs (two parts, four real products).
// Workgroup = one coarse site and 16 rhs, one wave per 16-row tile; lane
// layout of the instruction: A[l % 16][4 (l / 16) + i], B[4 (l / 16) + i]
// [l % 16], D[4 (l / 16) + v][l % 16].
typedef _Float16 cm_h4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void coarse_mfma16_kernel(cx<float>* __restrict__ out, size_t ostr, int out_first,
                                                            const cx<float>* __restrict__ add, size_t astr,
                                                            const cx<float>* __restrict__ xs, size_t xsstr,
                                                            int xs_first, float cs, const cx<float>* __restrict__ xn,
                                                            size_t xnstr, int xn_first, float cn,
                                                            CoarseView<__half> cv, int nc, int nrhs,
                                                            const int* gate) {
  if (gate && *gate == 0) return;
  __shared__ int smax[CM_RHS];
  const int ci = out_first + blockIdx.x;
  const int r0 = blockIdx.y * CM_RHS;
  const int nr = min(CM_RHS, nrhs - r0);
  const int t = threadIdx.x;
  const int lane = t & 63, rt = t >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const size_t nn = (size_t)nc * nc;
  const int s_beg = cs != 0.f ? 0 : 1;
  const int s_end = cn != 0.f ? 9 : 1;
  auto slot_vec = [&](int slot) -> const cx<float>* {
    const int nb = slot == 0 ? ci : cv.nbr[ci * 9 + slot];
    return slot == 0 ? xs + (size_t)(nb - xs_first) * nc : xn + (size_t)(nb - xn_first) * nc;
  };
  auto slot_str = [&](int slot) -> size_t { return slot == 0 ? xsstr : xnstr; };
  auto slot_coef = [&](int slot) -> float { return (slot == 0 ? cs : cn) * cv.Dsc[ci * 9 + slot]; };
  // per-rhs largest |coef D_scale x| over the inputs of this workgroup
  if (t < CM_RHS) smax[t] = 0;
  __syncthreads();
  for (int slot = s_beg; slot < s_end; ++slot) {
    const cx<float>* xv = slot_vec(slot);
    const size_t xstr = slot_str(slot);
    const float ca = fabsf(slot_coef(slot));
    for (int e = t; e < nc * nr; e += blockDim.x) {
      const int j = e / nc, k = e - j * nc;
      const cx<float> v = xv[(size_t)(r0 + j) * xstr + k];
      const float m = ca * fmaxf(fabsf(v.r), fabsf(v.i));
      atomicMax(&smax[j], __float_as_int(m));  // non-negative floats order as their bit patterns
    }
  }
  __syncthreads();
  // this lane's rhs (B column li) and its scale
  const int bj = min(li, nr - 1);
  int ex = 0;
  const float mx = __int_as_float(smax[bj]);
  if (mx > 0.f) (void)frexpf(mx, &ex);
  const float sc = ldexpf(1.f, -ex);
  const int arow = min(rt * 16 + li, nc - 1);
  cm_v4 ar_h = {0.f, 0.f, 0.f, 0.f}, ai_h = ar_h, ar_l = ar_h, ai_l = ar_h;
  for (int slot = s_beg; slot < s_end; ++slot) {
    const cx<float>* xv = slot_vec(slot) + (size_t)(r0 + bj) * slot_str(slot);
    const float coef = slot_coef(slot) * sc;
    const __half2* Dp = cv.D + ((size_t)ci * 9 + slot) * nn + arow;
    for (int k0 = 0; k0 < nc; k0 += 16) {
      cm_h4 a_r, a_i, a_mi, xr_h, xi_h, xr_l, xi_l;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + 4 * lg + i;
        const bool kin = k < nc;
        const int kc = kin ? k : nc - 1;
        const __half2 a = Dp[(size_t)kc * nc];
        a_r[i] = (_Float16)__low2half(a);
        a_i[i] = (_Float16)__high2half(a);
        a_mi[i] = -a_i[i];
        const cx<float> x = xv[kc];
        const float br = kin ? coef * x.r : 0.f, bi = kin ? coef * x.i : 0.f;
        xr_h[i] = (_Float16)br;
        xi_h[i] = (_Float16)bi;
        xr_l[i] = (_Float16)((br - (float)xr_h[i]) * 2048.f);
        xi_l[i] = (_Float16)((bi - (float)xi_h[i]) * 2048.f);
      }
      ar_h = __builtin_amdgcn_mfma_f32_16x16x16f16(a_r, xr_h, ar_h, 0, 0, 0);
      ar_h = __builtin_amdgcn_mfma_f32_16x16x16f16(a_mi, xi_h, ar_h, 0, 0, 0);
      ai_h = __builtin_amdgcn_mfma_f32_16x16x16f16(a_i, xr_h, ai_h, 0, 0, 0);
      ai_h = __builtin_amdgcn_mfma_f32_16x16x16f16(a_r, xi_h, ai_h, 0, 0, 0);
      ar_l = __builtin_amdgcn_mfma_f32_16x16x16f16(a_r, xr_l, ar_l, 0, 0, 0);
      ar_l = __builtin_amdgcn_mfma_f32_16x16x16f16(a_mi, xi_l, ar_l, 0, 0, 0);
      ai_l = __builtin_amdgcn_mfma_f32_16x16x16f16(a_i, xr_l, ai_l, 0, 0, 0);
      ai_l = __builtin_amdgcn_mfma_f32_16x16x16f16(a_r, xi_l, ai_l, 0, 0, 0);
    }
  }
  // lane: rows 4 lg + v of the tile, rhs li
  const float inv = 1.f / sc;
  if (li < nr) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rt * 16 + 4 * lg + v;
      if (row < nc) {
        cx<float> o = mk((ar_h[v] + ar_l[v] * (1.f / 2048.f)) * inv, (ai_h[v] + ai_l[v] * (1.f / 2048.f)) * inv);
        if (add) o = o + add[(size_t)(r0 + li) * astr + (size_t)(ci - out_first) * nc + row];
        out[(size_t)(r0 + li) * ostr + (size_t)(ci - out_first) * nc + row] = o;
      }
    }
  }
}

// ------------------------------------------------------ Eq. (dagger) fill
// backward block of the neighbour j = i + mu:
//   D[j][2+2mu](row, col) = s_row s_col conj(D[i][1+2mu](col, row)),
// s = -1 on left-handed (row < ntv), +1 on right-handed components.
template <typename T>
__global__ void dagger_fill_kernel(cx<T>* Dc, const int* nbr, int nc, int ntv) {
  const int ci = blockIdx.x;
  const int mu = blockIdx.y;
  const int j = nbr[ci * 9 + 1 + 2 * mu];
  const size_t nn = (size_t)nc * nc;
  const cx<T>* fwd = Dc + ((size_t)ci * 9 + 1 + 2 * mu) * nn;
  cx<T>* bwd = Dc + ((size_t)j * 9 + 2 + 2 * mu) * nn;
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int col = e / nc, row = e % nc;
    const T sgn = ((row < ntv) == (col < ntv)) ? (T)1 : (T)-1;
    bwd[(size_t)col * nc + row] = sgn * conj(fwd[(size_t)row * nc + col]);
  }
}

// ------------------------------------------------------ D_c quantisation
template <typename T, typename S>
__global__ __launch_bounds__(256) void quantize_coarse_kernel(stc_t<S>* Dq, float* Dsc, const cx<T>* Dc, int nc) {
  const size_t nn = (size_t)nc * nc;
  const size_t base = (size_t)blockIdx.x * nn;
  if constexpr (is_half<S>()) {
    __shared__ float red[4];
    float m = 0.f;
    for (size_t e = threadIdx.x; e < nn; e += blockDim.x) {
      cx<T> v = Dc[base + e];
      m = fmaxf(m, fmaxf(fabsf((float)v.r), fabsf((float)v.i)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    if (threadIdx.x == 0) Dsc[blockIdx.x] = m;
    const double inv = m > 0.f ? 1.0 / (double)m : 0.0;
    for (size_t e = threadIdx.x; e < nn; e += blockDim.x) {
      cx<T> v = Dc[base + e];
      Dq[base + e] = __floats2half2_rn((float)(v.r * inv), (float)(v.i * inv));
    }
  } else {
    for (size_t e = threadIdx.x; e < nn; e += blockDim.x) stc_store(Dq, base + e, cvt<double>(Dc[base + e]));
  }
}

// ------------------------------------ inversion of the even self blocks
// In-place Gauss-Jordan with partial (row) pivoting in FP64 LDS, one
// workgroup per even coarse site; the inverse is stored column-major in T.
template <typename T, typename S>
__global__ __launch_bounds__(256) void invert_even_kernel(cx<T>* Dinv, CoarseView<S> cv, int nc, int* status) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  cx<double>* M = reinterpret_cast<cx<double>*>(smem_raw);  // row-major nc x nc
  cx<double>* colk = M + (size_t)nc * nc;                    // column k before elimination
  int* perm = reinterpret_cast<int*>(colk + nc);
  __shared__ int piv_row;
  __shared__ int singular;
  const int ci = blockIdx.x;  // even sites are internal indices [0, neven)
  const size_t nn = (size_t)nc * nc;
  double sc = 1.0;
  if constexpr (is_half<S>()) sc = (double)cv.Dsc[ci * 9];
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int col = e / nc, row = e % nc;
    M[row * nc + col] = sc * ldc<double>(cv.D, (size_t)ci * 9 * nn + e);
  }
  if (threadIdx.x == 0) singular = 0;
  __syncthreads();
  for (int k = 0; k < nc; ++k) {
    if (threadIdx.x < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + threadIdx.x; i < nc; i += 64) {
        cx<double> v = M[i * nc + k];
        double a = v.r * v.r + v.i * v.i;
        if (a > best) { best = a; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (threadIdx.x == 0) {
        piv_row = bi;
        perm[k] = bi;
        if (!(best > 0.0)) singular = 1;
      }
    }
    __syncthreads();
    if (singular) break;
    const int p = piv_row;
    if (p != k)
      for (int j = threadIdx.x; j < nc; j += blockDim.x) {
        cx<double> t = M[k * nc + j];
        M[k * nc + j] = M[p * nc + j];
        M[p * nc + j] = t;
      }
    __syncthreads();
    const cx<double> pv = M[k * nc + k];
    const double pn = pv.r * pv.r + pv.i * pv.i;
    const cx<double> ipv = mk(pv.r / pn, -pv.i / pn);
    __syncthreads();
    // scale the pivot row (the pivot entry becomes 1/pv)
    for (int j = threadIdx.x; j < nc; j += blockDim.x) M[k * nc + j] = (j == k ? mk(1.0, 0.0) : M[k * nc + j]) * ipv;
    __syncthreads();
    for (int i = threadIdx.x; i < nc; i += blockDim.x) colk[i] = M[i * nc + k];
    __syncthreads();
    // eliminate column k from the other rows
    for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
      const int i = e / nc, j = e % nc;
      if (i == k) continue;
      const cx<double> f = colk[i];
      const cx<double> rk = M[k * nc + j];
      M[i * nc + j] = (j == k ? mk(0.0, 0.0) : M[i * nc + j]) - f * rk;
    }
    __syncthreads();
  }
  if (singular) {
    if (threadIdx.x == 0) atomicExch(status, 1);
    return;
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = nc - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        cx<double> t = M[i * nc + k];
        M[i * nc + k] = M[i * nc + p];
        M[i * nc + p] = t;
      }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int col = e / nc, row = e % nc;
    Dinv[(size_t)ci * nn + e] = cvt<T>(M[row * nc + col]);
  }
}

// ------------------------------------------------------ layout conversion
template <typename S>
__global__ void export_coarse_kernel(cx<double>* out, CoarseView<S> cv, Geom g) {
  const int ci = blockIdx.x, slot = blockIdx.y;
  const int nc = g.nc;
  int bc[4];
  int_block_coords(g, ci, bc);
  const int b = lex_block(g, bc);
  const size_t nn = (size_t)nc * nc;
  double sc = 1.0;
  if constexpr (is_half<S>()) sc = (double)cv.Dsc[ci * 9 + slot];
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int col = e / nc, row = e % nc;
    out[((size_t)b * 9 + slot) * nn + (size_t)row * nc + col] = sc * ldc<double>(cv.D, ((size_t)ci * 9 + slot) * nn + e);
  }
}

// D_c from the exported layout (block lexicographic, row-major blocks) into
// the internal one (internal block order, column-major blocks)
template <typename T>
__global__ void coarse_import_kernel(cx<T>* D, const cx<double>* in, Geom g) {
  const int ci = blockIdx.x, slot = blockIdx.y;
  const int nc = g.nc;
  int bc[4];
  int_block_coords(g, ci, bc);
  const int b = lex_block(g, bc);
  const size_t nn = (size_t)nc * nc;
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int col = e / nc, row = e % nc;
    D[((size_t)ci * 9 + slot) * nn + e] = cvt<T>(in[((size_t)b * 9 + slot) * nn + (size_t)row * nc + col]);
  }
}

__device__ inline int lex_to_int_block(const Geom& g, int b) {
  int bc[4];
  bc[0] = b % g.NB[0]; b /= g.NB[0];
  bc[1] = b % g.NB[1]; b /= g.NB[1];
  bc[2] = b % g.NB[2];
  bc[3] = b / g.NB[2];
  return block_to_int(g, bc);
}

template <typename T>
__global__ void coarse_to_internal_kernel(cx<T>* out, const cx<double>* canon, Geom g, int nrhs) {
  const int nb = g.nblocks, nc = g.nc;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrhs * nb * nc) return;
  const int k = (int)(idx % nc);
  const size_t rb = idx / nc;
  const int b = (int)(rb % nb);
  const size_t r = rb / nb;
  out[(r * nb + lex_to_int_block(g, b)) * nc + k] = cvt<T>(canon[idx]);
}

template <typename T>
__global__ void coarse_to_canonical_kernel(cx<double>* canon, const cx<T>* in, Geom g, int nrhs) {
  const int nb = g.nblocks, nc = g.nc;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrhs * nb * nc) return;
  const int k = (int)(idx % nc);
  const size_t rb = idx / nc;
  const int b = (int)(rb % nb);
  const size_t r = rb / nb;
  canon[idx] = cvt<double>(in[(r * nb + lex_to_int_block(g, b)) * nc + k]);
}

}  // namespace

template <typename T, typename S>
void launch_restrict(cx<T>* out, size_t ostr_r, size_t ostr_b, const cx<T>* y, size_t ystr, const BasisView<S>& bv,
                     const Geom& g, int nrhs, hipStream_t st, int face_mu) {
  if (nrhs <= 0) return;
  if constexpr (std::is_same<T, float>::value) {
    if (nrhs >= RESTRICT_MFMA_MIN_RHS) {
      dim3 grid(g.nblocks, (nrhs + 31) / 32);
      restrict_mfma_kernel<S><<<grid, 256, 0, st>>>(out, ostr_r, ostr_b, y, ystr, bv, g, nrhs, face_mu);
      return;
    }
  } else if constexpr (std::is_same<S, double>::value) {
    if (nrhs >= RESTRICT_MFMA64_MIN_RHS && g.ntv <= 32) {
      dim3 grid(g.nblocks, (nrhs + 31) / 32);
      restrict_mfma64_kernel<<<grid, 256, 0, st>>>(out, ostr_r, ostr_b, y, ystr, bv, g, nrhs, face_mu);
      return;
    }
  }
  const int threads = ((g.vblock + 63) / 64) * 64;
  restrict_kernel<T, S><<<g.nblocks, threads, 0, st>>>(out, ostr_r, ostr_b, y, ystr, bv, g, nrhs, face_mu);
}

template <typename T, typename S>
void launch_prolong(cx<T>* x, size_t xstr, const cx<T>* xc, size_t cstr, const BasisView<S>& bv, const Geom& g,
                    int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  const int threads = ((g.vblock + 63) / 64) * 64;
  const size_t lds = (size_t)nrhs * g.ntv * sizeof(cx<T>);
  prolong_kernel<T, S><<<g.nblocks * (12 / prolong_kp<T>()), threads, lds, st>>>(x, xstr, xc, cstr, bv, g, nrhs);
}

namespace {
template <typename T, typename S>
void stencil_launch(cx<T>* out, size_t ostr, int out_first, int nout, const cx<T>* add, size_t astr,
                    const cx<T>* xs, size_t xsstr, int xs_first, T cs, const cx<T>* xn, size_t xnstr, int xn_first,
                    T cn, const CoarseView<S>& cv, const cx<T>* Dmat, int nc, int nrhs, hipStream_t st,
                    const int* gate) {
  if (nrhs <= 0 || nout <= 0) return;
  // CG column groups of nc / RP row groups (at most 256 threads), fewer if
  // the CG partial sums of RB rhs would not fit 64 KB of LDS
  auto cg_for = [&](int rb, int rp) {
    const int cg = std::max(1, 256 * rp / nc);
    const int cap = (int)(65536 / ((size_t)nc * rb * sizeof(cx<T>)));
    return std::max(1, std::min(cg, cap));
  };
  if (nrhs == 1) {
    const int CG = cg_for(1, 2);
    coarse_stencil_kernel<T, S, 1, 2><<<dim3(nout, 1), CG * (nc / 2), (size_t)CG * nc * sizeof(cx<T>), st>>>(
        out, ostr, out_first, add, astr, xs, xsstr, xs_first, cs, xn, xnstr, xn_first, cn, cv, Dmat, nc, CG, nrhs, gate);
  } else if (nrhs <= 4) {
    const int CG = cg_for(4, 2);
    coarse_stencil_kernel<T, S, 4, 2><<<dim3(nout, 1), CG * (nc / 2), (size_t)CG * nc * 4 * sizeof(cx<T>), st>>>(
        out, ostr, out_first, add, astr, xs, xsstr, xs_first, cs, xn, xnstr, xn_first, cn, cv, Dmat, nc, CG, nrhs, gate);
  } else {
    if constexpr (std::is_same<T, float>::value) {
      // many rhs in FP32: matrix cores (a wave per 16-row tile, at most 4)
      if (!Dmat && nc <= 64) {
        const int tiles = (nc + 15) / 16;
        const dim3 grid(nout, (nrhs + CM_RHS - 1) / CM_RHS);
        if constexpr (is_half<S>())
          coarse_mfma16_kernel<<<grid, 64 * tiles, 0, st>>>(out, ostr, out_first, add, astr, xs, xsstr, xs_first,
                                                            cs, xn, xnstr, xn_first, cn, cv, nc, nrhs, gate);
        else
          coarse_mfma_kernel<S><<<grid, 64 * tiles, 0, st>>>(out, ostr, out_first, add, astr, xs, xsstr, xs_first,
                                                             cs, xn, xnstr, xn_first, cn, cv, nc, nrhs, gate);
        return;
      }
    }
    const int CG = cg_for(12, 1);
    coarse_stencil_kernel<T, S, 12, 1><<<dim3(nout, (nrhs + 11) / 12), CG * nc, (size_t)CG * nc * 12 * sizeof(cx<T>), st>>>(
        out, ostr, out_first, add, astr, xs, xsstr, xs_first, cs, xn, xnstr, xn_first, cn, cv, Dmat, nc, CG, nrhs, gate);
  }
}
}  // namespace

template <typename T, typename S>
void launch_coarse_stencil(cx<T>* out, size_t ostr, int out_first, int nout, const cx<T>* add, size_t astr,
                           const cx<T>* xs, size_t xsstr, int xs_first, T cs, const cx<T>* xn, size_t xnstr,
                           int xn_first, T cn, const CoarseView<S>& cv, const Geom& g, int nrhs, hipStream_t st,
                           const int* gate) {
  stencil_launch<T, S>(out, ostr, out_first, nout, add, astr, xs, xsstr, xs_first, cs, xn, xnstr, xn_first, cn, cv,
                       nullptr, g.nc, nrhs, st, gate);
}

template <typename T>
void launch_block_matvec(cx<T>* out, size_t ostr, const cx<T>* M, const cx<T>* x, size_t xstr, int nsites, int nc,
                         int nrhs, hipStream_t st, const int* gate) {
  CoarseView<T> none{nullptr, nullptr, nullptr};
  stencil_launch<T, T>(out, ostr, 0, nsites, nullptr, 0, x, xstr, 0, (T)1, nullptr, 0, 0, (T)0, none, M, nc, nrhs, st,
                       gate);
}

template <typename T>
void launch_dagger_fill(cx<T>* Dc, const int* nbr, const Geom& g, hipStream_t st) {
  dagger_fill_kernel<T><<<dim3(g.nblocks, 4), 256, 0, st>>>(Dc, nbr, g.nc, g.ntv);
}

template <typename T, typename S>
void launch_quantize_coarse(stc_t<S>* Dq, float* Dsc, const cx<T>* Dc, const Geom& g, hipStream_t st) {
  quantize_coarse_kernel<T, S><<<g.nblocks * 9, 256, 0, st>>>(Dq, Dsc, Dc, g.nc);
}

template <typename T, typename S>
void launch_invert_even_blocks(cx<T>* Dinv, const CoarseView<S>& cv, const Geom& g, int* status, hipStream_t st) {
  size_t lds = (size_t)(g.nc * g.nc + g.nc) * sizeof(cx<double>) + (size_t)g.nc * sizeof(int);
  invert_even_kernel<T, S><<<g.neven, 256, lds, st>>>(Dinv, cv, g.nc, status);
}

template <typename T, typename S>
void launch_export_coarse(cx<double>* out, const CoarseView<S>& cv, const Geom& g, hipStream_t st) {
  export_coarse_kernel<S><<<dim3(g.nblocks, 9), 256, 0, st>>>(out, cv, g);
}

template <typename T>
void launch_coarse_import(cx<T>* D, const cx<double>* in, const Geom& g, hipStream_t st) {
  coarse_import_kernel<T><<<dim3(g.nblocks, 9), 256, 0, st>>>(D, in, g);
}

template <typename T>
void launch_coarse_to_internal(cx<T>* out, const cx<double>* canon, const Geom& g, int nrhs, hipStream_t st) {
  size_t n = (size_t)nrhs * g.nblocks * g.nc;
  if (n) coarse_to_internal_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, canon, g, nrhs);
}
template <typename T>
void launch_coarse_to_canonical(cx<double>* canon, const cx<T>* in, const Geom& g, int nrhs, hipStream_t st) {
  size_t n = (size_t)nrhs * g.nblocks * g.nc;
  if (n) coarse_to_canonical_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(canon, in, g, nrhs);
}

#define INST_TS(T, S)                                                                                               \
  template void launch_restrict<T, S>(cx<T>*, size_t, size_t, const cx<T>*, size_t, const BasisView<S>&,            \
                                      const Geom&, int, hipStream_t, int);                                           \
  template void launch_prolong<T, S>(cx<T>*, size_t, const cx<T>*, size_t, const BasisView<S>&, const Geom&, int,    \
                                     hipStream_t);                                                                   \
  template void launch_coarse_stencil<T, S>(cx<T>*, size_t, int, int, const cx<T>*, size_t, const cx<T>*, size_t,    \
                                            int, T, const cx<T>*, size_t, int, T, const CoarseView<S>&, const Geom&, \
                                            int, hipStream_t, const int*);                                           \
  template void launch_quantize_coarse<T, S>(stc_t<S>*, float*, const cx<T>*, const Geom&, hipStream_t);             \
  template void launch_invert_even_blocks<T, S>(cx<T>*, const CoarseView<S>&, const Geom&, int*, hipStream_t);       \
  template void launch_export_coarse<T, S>(cx<double>*, const CoarseView<S>&, const Geom&, hipStream_t);
INST_TS(double, double)
INST_TS(float, float)
INST_TS(float, __half)
#undef INST_TS

#define INST_T(T)                                                                                                   \
  template void launch_block_matvec<T>(cx<T>*, size_t, const cx<T>*, const cx<T>*, size_t, int, int, int,            \
                                       hipStream_t, const int*);                                                     \
  template void launch_dagger_fill<T>(cx<T>*, const int*, const Geom&, hipStream_t);                                 \
  template void launch_coarse_import<T>(cx<T>*, const cx<double>*, const Geom&, hipStream_t);                        \
  template void launch_coarse_to_internal<T>(cx<T>*, const cx<double>*, const Geom&, int, hipStream_t);              \
  template void launch_coarse_to_canonical<T>(cx<double>*, const cx<T>*, const Geom&, int, hipStream_t);
INST_T(double)
INST_T(float)
#undef INST_T

}  // namespace ddamg
