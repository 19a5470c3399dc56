// Setup kernels of Alg. 5: orthonormalisation of the test vectors on every
// aggregate (Gram-Schmidt on the rows of R_i^h) and the storage formats of
// the resulting basis.
//
// The paper uses classical block Gram-Schmidt for fewer global sums and
// better cache reuse.  Here each aggregate (block b, chirality h: 6 V_block
// rows, ntv columns) is one workgroup running CholQR2 in FP64: the Gram
// matrix X^H X is accumulated from LDS-staged row chunks, Cholesky-factored
// (positive real diagonal), and X <- X T^{-1}; doing it twice restores
// orthogonality to rounding.  The result is the unique Q of X = Q T with
// positive diag(T), i.e. the same basis Gram-Schmidt produces.
#include "ddamg_internal.h"

namespace ddamg {

namespace {

constexpr int QR_THREADS = 256;
constexpr int QR_CHUNK_SITES = 8;  // rows staged per chunk: 6 * 8 = 48
constexpr int MAX_NTV = 32;

__device__ inline void upper_pair(int p, int n, int& i, int& j) {
  // p enumerates (i, j), i <= j, row by row
  i = 0;
  int rowlen = n;
  while (p >= rowlen) {
    p -= rowlen;
    ++i;
    --rowlen;
  }
  j = i + p;
}

__global__ __launch_bounds__(QR_THREADS) void aggregate_qr_kernel(cx<double>* W, Geom g, int* status) {
  __shared__ cx<double> L[6 * QR_CHUNK_SITES][MAX_NTV];
  __shared__ cx<double> G[MAX_NTV][MAX_NTV];
  __shared__ cx<double> Ti[MAX_NTV][MAX_NTV];  // T^{-1}, upper triangular
  __shared__ int fail;
  const int ci = blockIdx.x >> 1;  // internal block: its sites are ci * vblock + [0, vblock)
  const int h = blockIdx.x & 1;
  const int n = g.ntv;
  const int npairs = n * (n + 1) / 2;
  const size_t V = g.V;
  const int tid = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    cx<double> acc[3];
    int pi[3], pj[3];
    for (int q = 0; q < 3; ++q) {
      acc[q] = mk(0.0, 0.0);
      int p = tid + q * QR_THREADS;
      pi[q] = pj[q] = -1;
      if (p < npairs) upper_pair(p, n, pi[q], pj[q]);
    }
    for (int l0 = 0; l0 < g.vblock; l0 += QR_CHUNK_SITES) {
      const int nsites = min(QR_CHUNK_SITES, g.vblock - l0);
      for (int e = tid; e < nsites * 6 * n; e += QR_THREADS) {
        const int a = e % n;
        const int rk = e / n;  // row in chunk = site_local * 6 + k
        const int k = rk % 6;
        const int s = ci * g.vblock + l0 + rk / 6;
        L[rk][a] = W[((size_t)a * 12 + 6 * h + k) * V + s];
      }
      __syncthreads();
      for (int q = 0; q < 3; ++q) {
        if (pi[q] < 0) continue;
        cx<double> t = acc[q];
        for (int rr = 0; rr < nsites * 6; ++rr) t = t + cmulc(L[rr][pi[q]], L[rr][pj[q]]);
        acc[q] = t;
      }
      __syncthreads();
    }
    for (int q = 0; q < 3; ++q)
      if (pi[q] >= 0) {
        G[pi[q]][pj[q]] = acc[q];
        G[pj[q]][pi[q]] = conj(acc[q]);
      }
    if (tid == 0) fail = 0;
    __syncthreads();
    if (tid == 0) {
      // Cholesky G = T^H T (T upper, real positive diagonal), in place in
      // the upper triangle of G
      for (int k = 0; k < n && !fail; ++k) {
        double d = G[k][k].r;
        for (int m = 0; m < k; ++m) d -= G[m][k].r * G[m][k].r + G[m][k].i * G[m][k].i;
        if (!(d > 0.0)) {
          fail = 1;
          break;
        }
        d = sqrt(d);
        G[k][k] = mk(d, 0.0);
        for (int j = k + 1; j < n; ++j) {
          cx<double> v = G[k][j];
          for (int m = 0; m < k; ++m) v = v - cmulc(G[m][k], G[m][j]);
          G[k][j] = (1.0 / d) * v;
        }
      }
      // T^{-1} by back substitution, column by column
      if (!fail)
        for (int j = 0; j < n; ++j) {
          for (int i = j + 1; i < n; ++i) Ti[i][j] = mk(0.0, 0.0);
          Ti[j][j] = mk(1.0 / G[j][j].r, 0.0);
          for (int i = j - 1; i >= 0; --i) {
            cx<double> v = mk(0.0, 0.0);
            for (int m = i + 1; m <= j; ++m) v = v + G[i][m] * Ti[m][j];
            Ti[i][j] = (-1.0 / G[i][i].r) * v;
          }
        }
    }
    __syncthreads();
    if (fail) {
      if (tid == 0) atomicExch(status, 1);
      return;
    }
    // X <- X T^{-1}, one row per thread iteration
    for (int row = tid; row < 6 * g.vblock; row += QR_THREADS) {
      const int k = row % 6;
      const int s = ci * g.vblock + row / 6;
      cx<double> x[MAX_NTV];
      for (int a = 0; a < n; ++a) x[a] = W[((size_t)a * 12 + 6 * h + k) * V + s];
      for (int j = n - 1; j >= 0; --j) {
        cx<double> v = mk(0.0, 0.0);
        for (int i = 0; i <= j; ++i) v = v + x[i] * Ti[i][j];
        W[((size_t)j * 12 + 6 * h + k) * V + s] = v;
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
