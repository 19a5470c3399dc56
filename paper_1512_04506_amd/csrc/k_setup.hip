// Setup kernels of Alg. 5: orthonormalisation of the test vectors on every
// aggregate (Gram-Schmidt on the rows of R_i^h) and the storage formats of
// the resulting basis.
//
// The paper uses classical block Gram-Schmidt for fewer global sums and
// better cache reuse.  Here each aggregate (block, chirality h: 6 V_block
// rows, ntv columns) is one workgroup running CholQR2 in FP64: the Gram
// matrix X^H X, its Cholesky factor (positive real diagonal) and X <- X T^{-1};
// doing it twice restores orthogonality to rounding.  The result is the
// unique Q of X = Q T with positive diag(T), i.e. the basis Gram-Schmidt
// produces.
#include "ddamg_internal.h"

namespace ddamg {

namespace {

constexpr int QR_THREADS = 256;
constexpr int MAX_NTV = 32;
constexpr int TI = 2;                       // Gram tile: TI test vectors (rows of G)
constexpr int TJ = 4;                       //            x TJ test vectors (columns)
constexpr int GNV = TI * TJ * 2;            // real partial sums per lane and tile

template <int HALF, typename T>
__device__ inline void rs_step(T v[GNV], int lane) {
  const bool up = (lane & HALF) != 0;
#pragma unroll
  for (int j = 0; j < HALF; ++j) {
    const T send = up ? v[j] : v[j + HALF];
    const T keep = up ? v[j + HALF] : v[j];
    v[j] = keep + __shfl_xor(send, HALF, 64);
  }
  if constexpr (HALF > 1) rs_step<HALF / 2, T>(v, lane);
}

// lane i (i < GNV) ends with the sum over the 64 lanes of v[i]
template <typename T>
__device__ inline T reduce_scatter(T v[GNV], int lane) {
#pragma unroll
  for (int o = 32; o >= GNV; o >>= 1)
#pragma unroll
    for (int j = 0; j < GNV; ++j) v[j] += __shfl_xor(v[j], o, 64);
  rs_step<GNV / 2, T>(v, lane);
  return v[0];
}

// One workgroup per aggregate (internal block ci, chirality h); one lane per
// site of the block, which owns the aggregate's 6 rows of that site (spins
// of chirality h x colours).  Per CholQR pass:
//   G = X^H X: tiles of TI x TJ entries, each lane summing its 6 rows, the
//              64 lanes by a shuffle butterfly and the waves through LDS;
//   G = T^H T: Cholesky (real positive diagonal) and T^{-1} by one thread;
//   X <- X T^{-1}: each lane updates its own rows (coalesced in-place).
__global__ __launch_bounds__(QR_THREADS) void aggregate_qr_kernel(cx<double>* W, Geom g, int* status) {
  __shared__ cx<double> G[MAX_NTV][MAX_NTV];
  __shared__ cx<double> Ti[MAX_NTV][MAX_NTV];  // T^{-1}, upper triangular
  __shared__ double red[QR_THREADS / 64][MAX_NTV / TI][GNV];
  __shared__ int fail;
  const int ci = blockIdx.x >> 1;  // internal block: its sites are ci * vblock + [0, vblock)
  const int h = blockIdx.x & 1;
  const int n = g.ntv;
  const size_t V = g.V;
  const int l = threadIdx.x, lane = l & 63, w = l >> 6;
  const int nw = blockDim.x >> 6;
  const bool act = l < g.vblock;
  const size_t site = (size_t)ci * g.vblock + (act ? l : 0);
  const double m = act ? 1.0 : 0.0;
  auto X = [&](int a, int k) -> cx<double>* { return W + ((size_t)a * 12 + 6 * h + k) * V + site; };
  const int nti = (n + TI - 1) / TI, ntj = (n + TJ - 1) / TJ;
  for (int pass = 0; pass < 2; ++pass) {
    for (int jt = 0; jt < ntj; ++jt) {
      cx<double> xj[6][TJ];
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int q = 0; q < TJ; ++q) {
          const int a = min(jt * TJ + q, n - 1);
          const double mm = (jt * TJ + q < n) ? m : 0.0;
          xj[k][q] = mm * *X(a, k);
        }
      for (int it = 0; it < nti; ++it) {
        double v[GNV];
#pragma unroll
        for (int p = 0; p < TI; ++p) {
          const int a = min(it * TI + p, n - 1);
          const double mm = (it * TI + p < n) ? m : 0.0;
          cx<double> xi[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) xi[k] = mm * *X(a, k);
#pragma unroll
          for (int q = 0; q < TJ; ++q) {
            cx<double> acc = mk(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc = cfmac(xi[k], xj[k][q], acc);
            v[(p * TJ + q) * 2] = acc.r;
            v[(p * TJ + q) * 2 + 1] = acc.i;
          }
        }
        const double mine = reduce_scatter(v, lane);
        if (lane < GNV) red[w][it][lane] = mine;
      }
      __syncthreads();
      for (int e = l; e < nti * GNV; e += blockDim.x) {
        const int it = e / GNV, idx = e % GNV;
        double t = 0.0;
        for (int k = 0; k < nw; ++k) t += red[k][it][idx];
        const int part = idx & 1, pq = idx >> 1, p = pq / TJ, q = pq % TJ;
        const int i = it * TI + p, j = jt * TJ + q;
        if (i < n && j < n) reinterpret_cast<double*>(&G[i][j])[part] = t;
      }
      __syncthreads();
    }
    // Cholesky G = T^H T (T upper, real positive diagonal), right-looking,
    // in place in the upper triangle of G: step k scales row k by the pivot
    // and updates the trailing upper triangle, its entries spread over the
    // workgroup
    if (l == 0) fail = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const double dk = G[k][k].r;  // every thread reads the same pivot
      if (!(dk > 0.0)) {
        if (l == 0) fail = 1;
        break;
      }
      const double d = sqrt(dk);
      __syncthreads();
      for (int j = k + l; j < n; j += blockDim.x) G[k][j] = j == k ? mk(d, 0.0) : (1.0 / d) * G[k][j];
      __syncthreads();
      const int m = n - k - 1;  // trailing size
      for (int p = l; p < m * m; p += blockDim.x) {
        const int i = k + 1 + p / m, j = k + 1 + p % m;
        if (j >= i) G[i][j] = G[i][j] - cmulc(G[k][i], G[k][j]);
      }
      __syncthreads();
    }
    __syncthreads();
    if (fail) {
      if (l == 0) atomicExch(status, 1);
      return;
    }
    // T^{-1} by back substitution, one column per lane
    if (l < n) {
      const int j = l;
      for (int i = j + 1; i < n; ++i) Ti[i][j] = mk(0.0, 0.0);
      Ti[j][j] = mk(1.0 / G[j][j].r, 0.0);
      for (int i = j - 1; i >= 0; --i) {
        cx<double> vv = mk(0.0, 0.0);
        for (int mm = i + 1; mm <= j; ++mm) vv = cfma(G[i][mm], Ti[mm][j], vv);
        Ti[i][j] = (-1.0 / G[i][i].r) * vv;
      }
    }
    __syncthreads();
    // X <- X T^{-1}: lane = site, one row (spin-colour k) at a time; each
    // input entry is read once and added into every output it feeds, and the
    // row is written back after all its entries have been read
    if (act) {
      for (int k = 0; k < 6; ++k) {
        cx<double> y[MAX_NTV];
#pragma unroll
        for (int j = 0; j < MAX_NTV; ++j) y[j] = mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < MAX_NTV; ++i) {
          if (i < n) {
            const cx<double> xi = *X(i, k);
#pragma unroll
            for (int j = i; j < MAX_NTV; ++j)
              if (j < n) y[j] = cfma(xi, Ti[i][j], y[j]);
          }
          if ((i & 3) == 3) asm volatile("" ::: "memory");  // bound the loads in flight
        }
#pragma unroll
        for (int j = 0; j < MAX_NTV; ++j)
          if (j < n) *X(j, k) = y[j];
      }
    }
    __syncthreads();
  }
}

template <typename S>
__global__ void quantize_basis_kernel(stc_t<S>* Wq, float* Wsc, const cx<double>* W, int V, int ntv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ntv * V) return;
  const int s = (int)(idx % V);
  const int a = (int)(idx / V);
  if constexpr (is_half<S>()) {
    double m = 0.0;
    for (int k = 0; k < 12; ++k) {
      cx<double> v = W[((size_t)a * 12 + k) * V + s];
      m = fmax(m, fmax(fabs(v.r), fabs(v.i)));
    }
    const float fm = (float)m;
    Wsc[idx] = fm;
    const double inv = fm > 0.f ? 1.0 / (double)fm : 0.0;
    for (int k = 0; k < 12; ++k) {
      cx<double> v = W[((size_t)a * 12 + k) * V + s];
      Wq[((size_t)a * 12 + k) * V + s] = __floats2half2_rn((float)(v.r * inv), (float)(v.i * inv));
    }
  } else {
    for (int k = 0; k < 12; ++k) stc_store(Wq, ((size_t)a * 12 + k) * V + s, W[((size_t)a * 12 + k) * V + s]);
  }
}

template <typename T, typename S>
__global__ void dequantize_basis_kernel(cx<T>* out, BasisView<S> bv, int V, int ntv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ntv * 12 * V) return;
  const int s = (int)(idx % V);
  const int a = (int)(idx / ((size_t)12 * V));
  T sc = (T)1;
  if constexpr (is_half<S>()) sc = (T)bv.Wsc[(size_t)a * V + s];
  out[idx] = sc * ldc<T>(bv.W, idx);
}

}  // namespace

void launch_aggregate_qr(cx<double>* W, const Geom& g, int* status, hipStream_t st) {
  aggregate_qr_kernel<<<2 * g.nblocks, QR_THREADS, 0, st>>>(W, g, status);
}

template <typename S>
void launch_quantize_basis(stc_t<S>* Wq, float* Wsc, const cx<double>* W, const Geom& g, hipStream_t st) {
  size_t n = (size_t)g.ntv * g.V;
  quantize_basis_kernel<S><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(Wq, Wsc, W, g.V, g.ntv);
}
template <typename T, typename S>
void launch_dequantize_basis(cx<T>* out, const BasisView<S>& bv, const Geom& g, hipStream_t st) {
  size_t n = (size_t)g.ntv * 12 * g.V;
  dequantize_basis_kernel<T, S><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, bv, g.V, g.ntv);
}

template void launch_quantize_basis<double>(stc_t<double>*, float*, const cx<double>*, const Geom&, hipStream_t);
template void launch_quantize_basis<float>(stc_t<float>*, float*, const cx<double>*, const Geom&, hipStream_t);
template void launch_quantize_basis<__half>(stc_t<__half>*, float*, const cx<double>*, const Geom&, hipStream_t);
template void launch_dequantize_basis<double, double>(cx<double>*, const BasisView<double>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<float, float>(cx<float>*, const BasisView<float>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<float, __half>(cx<float>*, const BasisView<__half>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<double, __half>(cx<double>*, const BasisView<__half>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<double, float>(cx<double>*, const BasisView<float>&, const Geom&, hipStream_t);

}  // namespace ddamg
