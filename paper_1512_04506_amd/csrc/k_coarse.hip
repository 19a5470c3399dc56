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
// One wave per (block, chirality h, test vector a); lanes stride over the
// block's sites; up to RC right-hand sides accumulate per basis load.
constexpr int RC = 8;

template <typename T, typename S>
__global__ __launch_bounds__(64) void restrict_kernel(cx<T>* __restrict__ out, size_t ostr_r, size_t ostr_b,
                                                      const cx<T>* __restrict__ y, size_t ystr, BasisView<S> bv,
                                                      Geom g, const int* __restrict__ b2i, int nrhs) {
  const int b = blockIdx.x;
  const int h = blockIdx.y / g.ntv;
  const int a = blockIdx.y % g.ntv;
  const int lane = threadIdx.x;
  const size_t V = g.V;
  const int ci = b2i[b];
  for (int r0 = 0; r0 < nrhs; r0 += RC) {
    const int nr = min(RC, nrhs - r0);
    cx<T> acc[RC];
#pragma unroll
    for (int j = 0; j < RC; ++j) acc[j] = mk((T)0, (T)0);
    for (int l = lane; l < g.vblock; l += 64) {
      int c[4];
      const int s = block_site(g, b, l, c);
      T sc = (T)1;
      if constexpr (is_half<S>()) sc = (T)bv.Wsc[(size_t)a * V + s];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int comp = 6 * h + k;
        cx<T> w = sc * ldc<T>(bv.W, ((size_t)a * 12 + comp) * V + s);
#pragma unroll
        for (int j = 0; j < RC; ++j)
          if (j < nr) acc[j] = acc[j] + cmulc(w, y[(size_t)(r0 + j) * ystr + (size_t)comp * V + s]);
      }
    }
#pragma unroll
    for (int j = 0; j < RC; ++j) {
      T re = wave_sum(acc[j].r), im = wave_sum(acc[j].i);
      if (lane == 0 && j < nr) out[(size_t)(r0 + j) * ostr_r + (size_t)ci * ostr_b + h * g.ntv + a] = mk(re, im);
    }
  }
}

// ---------------------------------------------------------- prolongation
// One thread per (site, rhs): x(site) = sum_a W_a(site) x_c[block, h, a].
template <typename T, typename S>
__global__ __launch_bounds__(256) void prolong_kernel(cx<T>* __restrict__ x, size_t xstr, const cx<T>* __restrict__ xc,
                                                      size_t cstr, BasisView<S> bv, Geom g,
                                                      const int* __restrict__ b2i) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int r = blockIdx.y;
  const size_t V = g.V;
  int c[4];
  site_coords(g, s, c);
  const int ci = b2i[block_of(g, c)];
  const cx<T>* xp = xc + (size_t)r * cstr + (size_t)ci * g.nc;
  cx<T> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk((T)0, (T)0);
  for (int a = 0; a < g.ntv; ++a) {
    T sc = (T)1;
    if constexpr (is_half<S>()) sc = (T)bv.Wsc[(size_t)a * V + s];
    const cx<T> xl = sc * xp[a], xr = sc * xp[g.ntv + a];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      cx<T> w = ldc<T>(bv.W, ((size_t)a * 12 + k) * V + s);
      acc[k] = acc[k] + w * (k < 6 ? xl : xr);
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) x[(size_t)r * xstr + (size_t)k * V + s] = acc[k];
}

// ------------------------------------------------------------ D_c stencil
// One wave per (output coarse site, group of RB right-hand sides); lane =
// row.  out = add + cs D_self xs + cn sum_{slot>0} D_slot xn(nbr).
template <typename T, typename S, int RB>
__global__ __launch_bounds__(64) void coarse_stencil_kernel(cx<T>* __restrict__ out, size_t ostr, int out_first,
                                                            const cx<T>* __restrict__ add, size_t astr,
                                                            const cx<T>* __restrict__ xs, size_t xsstr, int xs_first,
                                                            T cs, const cx<T>* __restrict__ xn, size_t xnstr,
                                                            int xn_first, T cn, CoarseView<S> cv, int nc, int nrhs) {
  const int ci = out_first + blockIdx.x;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const int lane = threadIdx.x;
  const size_t nn = (size_t)nc * nc;
  for (int row0 = 0; row0 < nc; row0 += 64) {
    const int row = row0 + lane;
    if (row >= nc) break;
    cx<T> acc[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      acc[j] = mk((T)0, (T)0);
      if (add && j < nr) acc[j] = add[(size_t)(r0 + j) * astr + (size_t)(ci - out_first) * nc + row];
    }
    for (int slot = (cs != (T)0 ? 0 : 1); slot < (cn != (T)0 ? 9 : 1); ++slot) {
      const int nb = slot == 0 ? ci : cv.nbr[ci * 9 + slot];
      const cx<T>* xv = slot == 0 ? xs + (size_t)(nb - xs_first) * nc : xn + (size_t)(nb - xn_first) * nc;
      const size_t xstr = slot == 0 ? xsstr : xnstr;
      T coef = slot == 0 ? cs : cn;
      if constexpr (is_half<S>()) coef *= (T)cv.Dsc[ci * 9 + slot];
      const size_t base = ((size_t)ci * 9 + slot) * nn + row;
      for (int col = 0; col < nc; ++col) {
        const cx<T> d = coef * ldc<T>(cv.D, base + (size_t)col * nc);
#pragma unroll
        for (int j = 0; j < RB; ++j)
          if (j < nr) acc[j] = acc[j] + d * xv[(size_t)(r0 + j) * xstr + col];
      }
    }
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < nr) out[(size_t)(r0 + j) * ostr + (size_t)(ci - out_first) * nc + row] = acc[j];
  }
}

// out[k] = M[k] x[k], M column-major nc x nc per site
template <typename T, int RB>
__global__ __launch_bounds__(64) void block_matvec_kernel(cx<T>* __restrict__ out, size_t ostr,
                                                          const cx<T>* __restrict__ M, const cx<T>* __restrict__ x,
                                                          size_t xstr, int nc, int nrhs) {
  const int k = blockIdx.x;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const int lane = threadIdx.x;
  for (int row0 = 0; row0 < nc; row0 += 64) {
    const int row = row0 + lane;
    if (row >= nc) break;
    cx<T> acc[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) acc[j] = mk((T)0, (T)0);
    const cx<T>* Mk = M + (size_t)k * nc * nc + row;
    const cx<T>* xk = x + (size_t)k * nc;
    for (int col = 0; col < nc; ++col) {
      cx<T> m = Mk[(size_t)col * nc];
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < nr) acc[j] = acc[j] + m * xk[(size_t)(r0 + j) * xstr + col];
    }
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < nr) out[(size_t)(r0 + j) * ostr + (size_t)k * nc + row] = acc[j];
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
__global__ void export_coarse_kernel(cx<double>* out, CoarseView<S> cv, int nc, const int* i2b) {
  const int ci = blockIdx.x, slot = blockIdx.y;
  const int b = i2b[ci];
  const size_t nn = (size_t)nc * nc;
  double sc = 1.0;
  if constexpr (is_half<S>()) sc = (double)cv.Dsc[ci * 9 + slot];
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int col = e / nc, row = e % nc;
    out[((size_t)b * 9 + slot) * nn + (size_t)row * nc + col] = sc * ldc<double>(cv.D, ((size_t)ci * 9 + slot) * nn + e);
  }
}

template <typename T>
__global__ void coarse_to_internal_kernel(cx<T>* out, const cx<double>* canon, int nb, int nc, const int* b2i, int nrhs) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrhs * nb * nc) return;
  const int k = (int)(idx % nc);
  const size_t rb = idx / nc;
  const int b = (int)(rb % nb);
  const int r = (int)(rb / nb);
  out[((size_t)r * nb + b2i[b]) * nc + k] = cvt<T>(canon[idx]);
}

template <typename T>
__global__ void coarse_to_canonical_kernel(cx<double>* canon, const cx<T>* in, int nb, int nc, const int* b2i,
                                           int nrhs) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrhs * nb * nc) return;
  const int k = (int)(idx % nc);
  const size_t rb = idx / nc;
  const int b = (int)(rb % nb);
  const int r = (int)(rb / nb);
  canon[idx] = cvt<double>(in[((size_t)r * nb + b2i[b]) * nc + k]);
}

}  // namespace

template <typename T, typename S>
void launch_restrict(cx<T>* out, size_t ostr_r, size_t ostr_b, const cx<T>* y, size_t ystr, const BasisView<S>& bv,
                     const Geom& g, const int* b2i, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  dim3 grid(g.nblocks, 2 * g.ntv);
  restrict_kernel<T, S><<<grid, 64, 0, st>>>(out, ostr_r, ostr_b, y, ystr, bv, g, b2i, nrhs);
}

template <typename T, typename S>
void launch_prolong(cx<T>* x, size_t xstr, const cx<T>* xc, size_t cstr, const BasisView<S>& bv, const Geom& g,
                    const int* b2i, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  dim3 grid((g.V + 255) / 256, nrhs);
  prolong_kernel<T, S><<<grid, 256, 0, st>>>(x, xstr, xc, cstr, bv, g, b2i);
}

template <typename T, typename S>
void launch_coarse_stencil(cx<T>* out, size_t ostr, int out_first, int nout, const cx<T>* add, size_t astr,
                           const cx<T>* xs, size_t xsstr, int xs_first, T cs, const cx<T>* xn, size_t xnstr,
                           int xn_first, T cn, const CoarseView<S>& cv, const Geom& g, int nrhs, hipStream_t st) {
  if (nrhs <= 0 || nout <= 0) return;
  if (nrhs == 1) {
    dim3 grid(nout, 1);
    coarse_stencil_kernel<T, S, 1><<<grid, 64, 0, st>>>(out, ostr, out_first, add, astr, xs, xsstr, xs_first, cs, xn,
                                                        xnstr, xn_first, cn, cv, g.nc, nrhs);
  } else {
    dim3 grid(nout, (nrhs + 11) / 12);
    coarse_stencil_kernel<T, S, 12><<<grid, 64, 0, st>>>(out, ostr, out_first, add, astr, xs, xsstr, xs_first, cs, xn,
                                                         xnstr, xn_first, cn, cv, g.nc, nrhs);
  }
}

template <typename T>
void launch_block_matvec(cx<T>* out, size_t ostr, const cx<T>* M, const cx<T>* x, size_t xstr, int nsites, int nc,
                         int nrhs, hipStream_t st) {
  if (nrhs <= 0 || nsites <= 0) return;
  if (nrhs == 1) {
    block_matvec_kernel<T, 1><<<dim3(nsites, 1), 64, 0, st>>>(out, ostr, M, x, xstr, nc, nrhs);
  } else {
    block_matvec_kernel<T, 12><<<dim3(nsites, (nrhs + 11) / 12), 64, 0, st>>>(out, ostr, M, x, xstr, nc, nrhs);
  }
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
void launch_export_coarse(cx<double>* out, const CoarseView<S>& cv, const Geom& g, const int* i2b, hipStream_t st) {
  export_coarse_kernel<S><<<dim3(g.nblocks, 9), 256, 0, st>>>(out, cv, g.nc, i2b);
}

template <typename T>
void launch_coarse_to_internal(cx<T>* out, const cx<double>* canon, const Geom& g, const int* b2i, int nrhs,
                               hipStream_t st) {
  size_t n = (size_t)nrhs * g.nblocks * g.nc;
  if (n) coarse_to_internal_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, canon, g.nblocks, g.nc, b2i, nrhs);
}
template <typename T>
void launch_coarse_to_canonical(cx<double>* canon, const cx<T>* in, const Geom& g, const int* b2i, int nrhs,
                                hipStream_t st) {
  size_t n = (size_t)nrhs * g.nblocks * g.nc;
  if (n) coarse_to_canonical_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(canon, in, g.nblocks, g.nc, b2i, nrhs);
}

#define INST_TS(T, S)                                                                                               \
  template void launch_restrict<T, S>(cx<T>*, size_t, size_t, const cx<T>*, size_t, const BasisView<S>&,            \
                                      const Geom&, const int*, int, hipStream_t);                                    \
  template void launch_prolong<T, S>(cx<T>*, size_t, const cx<T>*, size_t, const BasisView<S>&, const Geom&,         \
                                     const int*, int, hipStream_t);                                                  \
  template void launch_coarse_stencil<T, S>(cx<T>*, size_t, int, int, const cx<T>*, size_t, const cx<T>*, size_t,    \
                                            int, T, const cx<T>*, size_t, int, T, const CoarseView<S>&, const Geom&, \
                                            int, hipStream_t);                                                       \
  template void launch_quantize_coarse<T, S>(stc_t<S>*, float*, const cx<T>*, const Geom&, hipStream_t);             \
  template void launch_invert_even_blocks<T, S>(cx<T>*, const CoarseView<S>&, const Geom&, int*, hipStream_t);       \
  template void launch_export_coarse<T, S>(cx<double>*, const CoarseView<S>&, const Geom&, const int*, hipStream_t);
INST_TS(double, double)
INST_TS(float, float)
INST_TS(float, __half)
#undef INST_TS

#define INST_T(T)                                                                                                   \
  template void launch_block_matvec<T>(cx<T>*, size_t, const cx<T>*, const cx<T>*, size_t, int, int, int,            \
                                       hipStream_t);                                                                 \
  template void launch_dagger_fill<T>(cx<T>*, const int*, const Geom&, hipStream_t);                                 \
  template void launch_coarse_to_internal<T>(cx<T>*, const cx<double>*, const Geom&, const int*, int, hipStream_t);  \
  template void launch_coarse_to_canonical<T>(cx<double>*, const cx<T>*, const Geom&, const int*, int, hipStream_t);
INST_T(double)
INST_T(float)
#undef INST_T

}  // namespace ddamg
