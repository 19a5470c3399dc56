// Krylov linear algebra on block vectors (one independent system per rhs):
// several inner products in one pass (the classical Gram-Schmidt step of
// GMRES), linear combinations, scaling, and the Arnoldi/Givens state of
// GMRES kept on the device in FP64 (Hessenberg least squares).
//
// Reductions are deterministic: each workgroup writes one partial per
// (rhs, vector, chunk) and a second kernel sums the chunks in a fixed
// order, so repeated runs give bitwise identical results.
#include "ddamg_internal.h"

namespace ddamg {

namespace {

constexpr int BT = 256;
constexpr int JG = 8;  // basis vectors per pass over the chunk
constexpr int MAX_MDOT_VECS = 66;  // restart length 64 plus w itself

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// With a single chunk the workgroup's sums are the inner products: they go
// straight to h (row stride ldh) and no final kernel runs.
template <typename T>
__global__ __launch_bounds__(BT) void mdot_partial_kernel(cx<double>* part, const cx<T>* __restrict__ Vb,
                                                          size_t vsj, size_t vsr, int nvec,
                                                          const cx<T>* __restrict__ w, size_t wsr, size_t n,
                                                          size_t chunk, int nchunk, const int* active,
                                                          cx<double>* h, int ldh) {
  __shared__ cx<double> red[MAX_MDOT_VECS][BT / 64];
  const int c = blockIdx.x;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const size_t beg = (size_t)c * chunk;
  const size_t end = min(n, beg + chunk);
  const cx<T>* wr = w + (size_t)r * wsr;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j0 = 0; j0 < nvec; j0 += JG) {
    cx<T> acc[JG];
#pragma unroll
    for (int q = 0; q < JG; ++q) acc[q] = mk((T)0, (T)0);
    for (size_t i = beg + threadIdx.x; i < end; i += BT) {
      const cx<T> wv = wr[i];
#pragma unroll
      for (int q = 0; q < JG; ++q)
        if (j0 + q < nvec) acc[q] = acc[q] + cmulc(Vb[(size_t)(j0 + q) * vsj + (size_t)r * vsr + i], wv);
    }
#pragma unroll
    for (int q = 0; q < JG; ++q) {
      double re = wave_sum_d((double)acc[q].r), im = wave_sum_d((double)acc[q].i);
      if (lane == 0 && j0 + q < nvec) red[j0 + q][wid] = mk(re, im);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nvec; j += BT) {
    cx<double> s = mk(0.0, 0.0);
    for (int k = 0; k < BT / 64; ++k) s = s + red[j][k];
    if (nchunk == 1)
      h[(size_t)r * ldh + j] = s;
    else
      part[((size_t)r * nvec + j) * nchunk + c] = s;
  }
}

__global__ void mdot_final_kernel(cx<double>* h, int ldh, const cx<double>* part, int nvec, int nchunk,
                                  const int* active) {
  const int j = blockIdx.x;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  double re = 0.0, im = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 64) {
    cx<double> v = part[((size_t)r * nvec + j) * nchunk + c];
    re += v.r;
    im += v.i;
  }
  re = wave_sum_d(re);
  im = wave_sum_d(im);
  if (threadIdx.x == 0) h[(size_t)r * ldh + j] = mk(re, im);
}

// w <- (w + sign sum_j h_j V_j) [* post[r] if post], and an FP32 copy of the
// result in w32 (same strides) if w32 is given
template <typename Tw, typename Tv>
__global__ __launch_bounds__(BT) void maxpy_kernel(cx<Tw>* w, size_t wsr, const cx<Tv>* __restrict__ Vb, size_t vsj,
                                                   size_t vsr, int nvec, const cx<double>* __restrict__ h, int ldh,
                                                   double sign, size_t n, const int* active, const double* post,
                                                   cx<float>* w32) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  using Tc = typename std::conditional<(sizeof(Tw) > sizeof(Tv)), Tw, Tv>::type;
  const cx<double>* hr = h + (size_t)r * ldh;
  const Tc f = post ? (Tc)post[r] : (Tc)1;
  for (size_t i = (size_t)blockIdx.x * BT + threadIdx.x; i < n; i += (size_t)gridDim.x * BT) {
    cx<Tc> acc = cvt<Tc>(w[(size_t)r * wsr + i]);
    for (int j = 0; j < nvec; ++j)
      acc = acc + cvt<Tc>(sign * hr[j]) * cvt<Tc>(Vb[(size_t)j * vsj + (size_t)r * vsr + i]);
    const cx<Tw> res = cvt<Tw>(f * acc);
    w[(size_t)r * wsr + i] = res;
    if (w32) w32[(size_t)r * wsr + i] = cvt<float>(res);
  }
}

// Second step of classical Gram-Schmidt done twice, in one pass over the
// data: w <- w - sum_j h_j V_j, then the partial sums of V_j^H w (j < nvec)
// and |w|^2 (entry nvec) of the updated w, as mdot_partial_kernel writes
// them.  The nvec basis entries of an element stay in registers between
// the update and the inner products, so every vector is read once.
template <int MAXV>
__global__ __launch_bounds__(BT) void gs_fused_kernel(cx<double>* part, const cx<double>* __restrict__ Vb, size_t vsj,
                                                      size_t vsr, int nvec, cx<double>* w, size_t wsr,
                                                      const cx<double>* __restrict__ h, int ldh, size_t n,
                                                      size_t chunk, int nchunk, const int* active,
                                                      cx<double>* h2) {
  __shared__ cx<double> red[MAXV + 1][BT / 64];
  const int c = blockIdx.x;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const size_t beg = (size_t)c * chunk;
  const size_t end = min(n, beg + chunk);
  cx<double>* wr = w + (size_t)r * wsr;
  const cx<double>* hr = h + (size_t)r * ldh;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  cx<double> acc[MAXV];
  double nacc = 0.0;
#pragma unroll
  for (int j = 0; j < MAXV; ++j) acc[j] = mk(0.0, 0.0);
  for (size_t i = beg + threadIdx.x; i < end; i += BT) {
    cx<double> v[MAXV];
    cx<double> x = wr[i];
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
      if (j < nvec) {
        v[j] = Vb[(size_t)j * vsj + (size_t)r * vsr + i];
        x = x - hr[j] * v[j];
      }
    wr[i] = x;
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
      if (j < nvec) acc[j] = acc[j] + cmulc(v[j], x);
    nacc += x.r * x.r + x.i * x.i;
  }
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    if (j < nvec) {
      const double re = wave_sum_d(acc[j].r), im = wave_sum_d(acc[j].i);
      if (lane == 0) red[j][wid] = mk(re, im);
    }
  }
  nacc = wave_sum_d(nacc);
  if (lane == 0) red[nvec][wid] = mk(nacc, 0.0);
  __syncthreads();
  for (int j = threadIdx.x; j <= nvec; j += BT) {
    cx<double> sum = mk(0.0, 0.0);
    for (int k = 0; k < BT / 64; ++k) sum = sum + red[j][k];
    if (nchunk == 1)
      h2[(size_t)r * ldh + j] = sum;  // a single chunk: the sums are final
    else
      part[((size_t)r * (nvec + 1) + j) * nchunk + c] = sum;
  }
}

// Second step of classical Gram-Schmidt done twice with the subtraction of
// the previous step's second projection deferred into it.  Slot k holds the
// pending vector u (the previous new vector, projected once); with the
// previous second-projection coefficients c and normalisation sigma it
// becomes v_k = sigma (u - sum_{j<k} c_j V_j), the vector a separate pass
// would have written, and is stored back (correct = false: u is v_k
// already).  In the same pass over the data: w <- w - sum_{j<=k} h_j V_j
// with the corrected v_k, its FP32 copy in w32 if given, and the partial
// sums of V_j^H w (j <= k) and |w|^2 as gs_fused_kernel writes them.
// The FP32 copy is scaled by wsc[r] (an estimate of 1 / |w''|) so that the
// preconditioner, which receives it, sees a vector of about unit norm.
template <int MAXV>
__global__ __launch_bounds__(BT) void gs_defer_kernel(cx<double>* part, cx<double>* Vb, size_t vsj, size_t vsr, int k,
                                                      int correct, const cx<double>* __restrict__ c, int ldc,
                                                      const double* __restrict__ sigma, cx<double>* w, size_t wsr,
                                                      const cx<double>* __restrict__ h, int ldh, size_t n,
                                                      size_t chunk, int nchunk, const int* active, cx<double>* h2,
                                                      cx<float>* w32, const double* __restrict__ wsc) {
  __shared__ cx<double> red[MAXV + 1][BT / 64];
  const int cb = blockIdx.x;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int nvec = k + 1;
  const size_t beg = (size_t)cb * chunk;
  const size_t end = min(n, beg + chunk);
  cx<double>* wr = w + (size_t)r * wsr;
  cx<double>* uk = Vb + (size_t)k * vsj + (size_t)r * vsr;
  const cx<double>* hr = h + (size_t)r * ldh;
  const cx<double>* cr = c + (size_t)r * ldc;
  const double sg = sigma[r];
  const double ws = w32 ? wsc[r] : 1.0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  cx<double> acc[MAXV];
  double nacc = 0.0;
#pragma unroll
  for (int j = 0; j < MAXV; ++j) acc[j] = mk(0.0, 0.0);
  for (size_t i = beg + threadIdx.x; i < end; i += BT) {
    cx<double> v[MAXV];
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
      if (j < k) v[j] = Vb[(size_t)j * vsj + (size_t)r * vsr + i];
    cx<double> u = uk[i];
    if (correct) {
#pragma unroll
      for (int j = 0; j < MAXV; ++j)
        if (j < k) u = u - cr[j] * v[j];
      u = sg * u;
      uk[i] = u;
    }
    cx<double> x = wr[i];
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
      if (j < nvec) {
        if (j == k) v[j] = u;
        x = x - hr[j] * v[j];
      }
    wr[i] = x;
    if (w32) w32[(size_t)r * wsr + i] = cvt<float>(ws * x);
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
      if (j < nvec) acc[j] = acc[j] + cmulc(v[j], x);
    nacc += x.r * x.r + x.i * x.i;
  }
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    if (j < nvec) {
      const double re = wave_sum_d(acc[j].r), im = wave_sum_d(acc[j].i);
      if (lane == 0) red[j][wid] = mk(re, im);
    }
  }
  nacc = wave_sum_d(nacc);
  if (lane == 0) red[nvec][wid] = mk(nacc, 0.0);
  __syncthreads();
  for (int j = threadIdx.x; j <= nvec; j += BT) {
    cx<double> sum = mk(0.0, 0.0);
    for (int q = 0; q < BT / 64; ++q) sum = sum + red[j][q];
    if (nchunk == 1)
      h2[(size_t)r * ldh + j] = sum;
    else
      part[((size_t)r * (nvec + 1) + j) * nchunk + cb] = sum;
  }
}

// Before the deferred pass, with h[r][0..k] = V_j^H w and h[r][k + 1] =
// |w|^2 from the first pass: if correct, c[r][j] = h2[r][j] (j < k), the
// pending vector's corrections, kept apart from h2 (which that pass
// overwrites), and h[r][k] = sigma_r (h[r][k] - sum_{j<k} conj(c_j) h[r][j]),
// the inner product of w with the corrected v_k from those with the stored
// vectors; then wsc[r] = 1 / |w'| from |w'|^2 = |w|^2 - sum_{j<=k} |h_j|^2,
// floored at 1e-20 |w|^2 against cancellation (only a scale: the exact
// |w''| follows the pass).
__global__ void gs_defer_coef_kernel(cx<double>* h, cx<double>* c, const cx<double>* h2, int ldh,
                                     const double* sigma, int k, int correct, double* wsc, int nrhs,
                                     const int* active) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  if (active && !active[r]) return;
  cx<double>* hr = h + (size_t)r * ldh;
  if (correct) {
    cx<double> d = hr[k];
    for (int j = 0; j < k; ++j) {
      const cx<double> cj = h2[(size_t)r * ldh + j];
      c[(size_t)r * ldh + j] = cj;
      d = d - conj(cj) * hr[j];
    }
    hr[k] = sigma[r] * d;
  }
  const double w2 = hr[k + 1].r;
  double e = w2;
  for (int j = 0; j <= k; ++j) e -= hr[j].r * hr[j].r + hr[j].i * hr[j].i;
  e = fmax(e, 1e-20 * w2);
  wsc[r] = (e > 0.0 && isfinite(e)) ? 1.0 / sqrt(e) : 0.0;
}

// |w''|^2 = |w'|^2 - sum_j |h2_j|^2 (w'' = w' - V h2 with V orthonormal),
// and the factor that normalises w''; zero for a vanishing or non-finite
// norm (the Arnoldi step then stops that rhs)
__global__ void gs_norm_kernel(cx<double>* n2, double* inv, const cx<double>* h2, int ldh, int nvec, int nrhs,
                               const int* active) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  if (active && !active[r]) return;
  const cx<double>* hr = h2 + (size_t)r * ldh;
  double t = hr[nvec].r;
  for (int j = 0; j < nvec; ++j) t -= hr[j].r * hr[j].r + hr[j].i * hr[j].i;
  t = fmax(t, 0.0);
  n2[r] = mk(t, 0.0);
  const double nr = sqrt(t);
  inv[r] = (nr > 0.0 && isfinite(nr)) ? 1.0 / nr : 0.0;
}

template <typename Ty, typename Tx>
__global__ __launch_bounds__(BT) void scale_kernel(cx<Ty>* y, size_t ystr, const cx<Tx>* x, size_t xstr,
                                                   const double* s, size_t n, const int* active, cx<float>* y32) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const double f = s[r];
  for (size_t i = (size_t)blockIdx.x * BT + threadIdx.x; i < n; i += (size_t)gridDim.x * BT) {
    cx<double> v = cvt<double>(x[(size_t)r * xstr + i]);
    const cx<Ty> res = cvt<Ty>(f * v);
    y[(size_t)r * ystr + i] = res;
    if (y32) y32[(size_t)r * ystr + i] = cvt<float>(res);
  }
}

template <typename T>
__global__ __launch_bounds__(BT) void sub_kernel(cx<T>* y, size_t ystr, const cx<T>* a, size_t astr, const cx<T>* b,
                                                 size_t bstr, size_t n) {
  const int r = blockIdx.y;
  for (size_t i = (size_t)blockIdx.x * BT + threadIdx.x; i < n; i += (size_t)gridDim.x * BT)
    y[(size_t)r * ystr + i] = a[(size_t)r * astr + i] - b[(size_t)r * bstr + i];
}

template <typename Ty, typename Tx>
__global__ __launch_bounds__(BT) void copy_kernel(cx<Ty>* y, size_t ystr, const cx<Tx>* x, size_t xstr, size_t n) {
  const int r = blockIdx.y;
  for (size_t i = (size_t)blockIdx.x * BT + threadIdx.x; i < n; i += (size_t)gridDim.x * BT)
    y[(size_t)r * ystr + i] = cvt<Ty>(x[(size_t)r * xstr + i]);
}

inline unsigned grid_for(size_t n) {
  size_t b = (n + BT - 1) / BT;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// ----------------------------------------------------- Arnoldi / Givens
__device__ inline double cabs2(cx<double> a) { return a.r * a.r + a.i * a.i; }

// rotation [c s; -conj(s) c] (c real) with c a + s b = r, -conj(s) a + c b = 0
__device__ inline void givens(cx<double> a, cx<double> b, double& c, cx<double>& s, cx<double>& r) {
  const double na = sqrt(cabs2(a)), nb = sqrt(cabs2(b));
  if (nb == 0.0) {
    c = 1.0;
    s = mk(0.0, 0.0);
    r = a;
    return;
  }
  if (na == 0.0) {
    c = 0.0;
    s = (1.0 / nb) * conj(b);
    r = mk(nb, 0.0);
    return;
  }
  const double nrm = sqrt(na * na + nb * nb);
  const cx<double> ph = (1.0 / na) * a;
  c = na / nrm;
  s = (1.0 / nrm) * (ph * conj(b));
  r = nrm * ph;
}

// active flags of all rhs into *any (one 64-lane wave, nrhs <= 64)
__device__ inline void publish_any(const ArnoldiState& s, bool act) {
  const unsigned long long b = __ballot(act);
  if (threadIdx.x == 0) *s.any = b != 0ull ? 1 : 0;
}

__global__ void arnoldi_start_kernel(ArnoldiState s, const cx<double>* norm2, int ldn, int nrhs) {
  const int r = threadIdx.x;
  bool act = false;
  if (r < nrhs) {
    const int m = s.m;
    const double beta = sqrt(fmax(norm2[(size_t)r * ldn].r, 0.0));
    for (int j = 0; j <= m; ++j) s.g[(size_t)r * (m + 1) + j] = mk(0.0, 0.0);
    s.g[(size_t)r * (m + 1)] = mk(beta, 0.0);
    const double tol = s.abstol[r];
    act = tol < 0.0 ? beta > 0.0 : beta > tol;
    s.active[r] = act ? 1 : 0;
    s.inv_h[r] = act ? 1.0 / beta : 0.0;
    s.kdone[r] = 0;
    s.est[r] = beta;
  }
  publish_any(s, act);
}

__global__ void arnoldi_column_kernel(ArnoldiState s, int k, const cx<double>* h1, const cx<double>* h2, int ldh,
                                      const cx<double>* norm2, int ldn, int nrhs) {
  const int r = threadIdx.x;
  bool act = false;
  if (r < nrhs && !s.active[r]) s.inv_h[r] = 0.0;
  if (r < nrhs && s.active[r]) {
    const int m = s.m;
    cx<double>* H = s.H + (size_t)r * (m + 1) * m + (size_t)k * (m + 1);
    cx<double>* cs = s.cs + (size_t)r * m;
    cx<double>* sn = s.sn + (size_t)r * m;
    cx<double>* g = s.g + (size_t)r * (m + 1);
    for (int j = 0; j <= k; ++j) {
      cx<double> v = h1[(size_t)r * ldh + j];
      if (h2) v = v + h2[(size_t)r * ldh + j];
      H[j] = v;
    }
    const double hn = sqrt(fmax(norm2[(size_t)r * ldn].r, 0.0));
    H[k + 1] = mk(hn, 0.0);
    for (int j = 0; j < k; ++j) {
      const double c = cs[j].r;
      const cx<double> sj = sn[j];
      const cx<double> t = c * H[j] + sj * H[j + 1];
      H[j + 1] = c * H[j + 1] - conj(sj) * H[j];
      H[j] = t;
    }
    double c;
    cx<double> sv, rr;
    givens(H[k], H[k + 1], c, sv, rr);
    cs[k] = mk(c, 0.0);
    sn[k] = sv;
    H[k] = rr;
    H[k + 1] = mk(0.0, 0.0);
    const cx<double> gk = g[k];
    g[k + 1] = neg(conj(sv) * gk);
    g[k] = c * gk;
    const double est = sqrt(cabs2(g[k + 1]));
    s.est[r] = est;
    s.kdone[r] = k + 1;
    const double tol = s.abstol[r];
    const bool stop = !(hn > 0.0) || (tol >= 0.0 && est <= tol) || k + 1 >= m;
    act = !stop;
    s.active[r] = stop ? 0 : 1;
    s.inv_h[r] = stop ? 0.0 : 1.0 / hn;
  }
  publish_any(s, act);
}

__global__ void arnoldi_solve_kernel(ArnoldiState s, int nrhs) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  const int m = s.m;
  const int kd = s.kdone[r];
  const cx<double>* H = s.H + (size_t)r * (m + 1) * m;
  const cx<double>* g = s.g + (size_t)r * (m + 1);
  cx<double>* y = s.y + (size_t)r * m;
  for (int j = kd; j < m; ++j) y[j] = mk(0.0, 0.0);
  for (int i = kd - 1; i >= 0; --i) {
    cx<double> v = g[i];
    for (int j = i + 1; j < kd; ++j) v = v - H[(size_t)j * (m + 1) + i] * y[j];
    const cx<double> d = H[(size_t)i * (m + 1) + i];
    const double dn = cabs2(d);
    y[i] = dn > 0.0 ? (1.0 / dn) * (conj(d) * v) : mk(0.0, 0.0);
  }
}

// ---------------------------------------------------- small coarse lattices
// The whole coarse solve of Alg. 2 for one rhs in one workgroup: the
// even/odd Schur complement S = D_oo - D_oe D_ee^{-1} D_eo, restarted GMRES
// on S with classical Gram-Schmidt twice, the Givens rotations and the
// convergence test of arnoldi_start/column_kernel, the back substitution,
// then x_e = D_ee^{-1} (y_e - D_eo x_o).  For a coarse lattice of a few
// dozen sites one GMRES iteration is a few microseconds of work; as ten
// separate launches it is a chain of ten launch latencies, which is what
// bounds the solve of a small lattice.  Every loop is bounded by maxit or
// by the restart length m <= SG_M.
constexpr int SG_T = 512;
constexpr int SG_M = COARSE_SMALL_MAX_RESTART;

__device__ inline int sg_flag(int* sh, int v) {
  if (threadIdx.x == 0) *sh = v;
  __syncthreads();
  const int r = *sh;
  __syncthreads();
  return r;
}

// One workgroup on one CU streams the coarse operator from L2 once per
// stencil pass, so the loads in flight set the speed: the neighbour slots
// (or the columns of a block matvec) are split over G groups of threads that
// each own one output element, with the inner loop unrolled, and the G
// partial sums are added in a fixed order through LDS (part: SG_T entries).
__device__ inline int sg_groups(int nelem, int nsplit) {
  int G = nelem > 0 ? SG_T / nelem : 1;
  if (G < 1) G = 1;
  if (G > nsplit) G = nsplit;
  return G;
}

template <typename T>
__device__ void sg_finish(cx<T>* out, const cx<T>* add, cx<T>* part, int G, int nelem, bool mine, int e,
                          cx<T> acc) {
  // G == 1: every thread owns its elements and wrote them already
  if (G == 1) {
    __syncthreads();
    return;
  }
  if (mine) part[threadIdx.x] = acc;  // threadIdx.x = q * nelem + e
  __syncthreads();
  if (threadIdx.x < nelem) {
    cx<T> sum = add ? add[e] : mk((T)0, (T)0);
    for (int q = 0; q < G; ++q) sum = sum + part[q * nelem + e];
    out[e] = sum;
  }
  __syncthreads();
}

// out[e], e < nsite * nc, for the sites out_first .. out_first + nsite - 1:
//   add[e] + cs D_self xs(site) + cn sum_{slot > 0} D_slot xn(nbr(slot))
// The inputs are first copied to xl (LDS, nblocks * nc entries, site-major
// over the whole lattice): every row of a site reads the same x entries, and
// as LDS broadcasts they leave the memory pipeline to the operator.  xs holds
// the out sites, xn the sites of the other parity (all neighbours).
template <typename T, typename S>
__device__ void sg_stencil(cx<T>* out, int out_first, int nsite, const cx<T>* add, const cx<T>* xs, int xs_first,
                           T cs, const cx<T>* xn, int xn_first, T cn, const CoarseView<S>& cv, int nc, int nblocks,
                           cx<T>* part, cx<T>* xl) {
  const size_t nn = (size_t)nc * nc;
  const int nelem = nsite * nc;
  const int s_beg = cs != (T)0 ? 0 : 1, s_end = cn != (T)0 ? 9 : 1;
  if (cs != (T)0)
    for (int e = threadIdx.x; e < nelem; e += SG_T)
      xl[(size_t)out_first * nc + e] = xs[(size_t)(out_first - xs_first) * nc + e];
  if (cn != (T)0) {
    const int nx = xn_first == 0 ? out_first : nblocks - xn_first;
    for (int e = threadIdx.x; e < nx * nc; e += SG_T) xl[(size_t)xn_first * nc + e] = xn[e];
  }
  __syncthreads();
  const int G = sg_groups(nelem, s_end - s_beg);
  auto element = [&](int e, int q) {
    const int ls = e / nc, row = e - ls * nc;
    const int ci = out_first + ls;
    cx<T> acc = mk((T)0, (T)0);
    for (int slot = s_beg + q; slot < s_end; slot += G) {
      const int nb = slot == 0 ? ci : cv.nbr[ci * 9 + slot];
      const cx<T>* xv = xl + (size_t)nb * nc;
      T coef = slot == 0 ? cs : cn;
      if constexpr (is_half<S>()) coef *= (T)cv.Dsc[ci * 9 + slot];
      const size_t base = ((size_t)ci * 9 + slot) * nn + row;
      cx<T> sum = mk((T)0, (T)0);
#pragma unroll 8
      for (int k = 0; k < nc; ++k) sum = sum + ldc<T>(cv.D, base + (size_t)k * nc) * xv[k];
      acc = acc + coef * sum;
    }
    return acc;
  };
  if (G == 1) {
    for (int e = threadIdx.x; e < nelem; e += SG_T) {
      const cx<T> acc = element(e, 0);
      out[e] = add ? add[e] + acc : acc;
    }
    sg_finish<T>(out, add, part, 1, nelem, false, 0, mk((T)0, (T)0));
    return;
  }
  const int q = threadIdx.x / nelem, e = threadIdx.x - q * nelem;
  const bool mine = q < G;
  const cx<T> acc = mine ? element(e, q) : mk((T)0, (T)0);
  sg_finish<T>(out, add, part, G, nelem, mine, e, acc);
}

// out = M x per site (M: nsite column-major nc x nc blocks)
template <typename T>
__device__ void sg_block_matvec(cx<T>* out, const cx<T>* M, const cx<T>* x, int nsite, int nc, cx<T>* part,
                                cx<T>* xl) {
  const size_t nn = (size_t)nc * nc;
  const int nelem = nsite * nc;
  for (int e = threadIdx.x; e < nelem; e += SG_T) xl[e] = x[e];
  __syncthreads();
  const int G = sg_groups(nelem, 8);
  auto element = [&](int e, int q) {
    const int ls = e / nc, row = e - ls * nc;
    const cx<T>* Mk = M + (size_t)ls * nn + row;
    const cx<T>* xk = xl + (size_t)ls * nc;
    cx<T> sum = mk((T)0, (T)0);
#pragma unroll 4
    for (int k = q; k < nc; k += G) sum = sum + Mk[(size_t)k * nc] * xk[k];
    return sum;
  };
  if (G == 1) {
    for (int e = threadIdx.x; e < nelem; e += SG_T) out[e] = element(e, 0);
    sg_finish<T>(out, nullptr, part, 1, nelem, false, 0, mk((T)0, (T)0));
    return;
  }
  const int q = threadIdx.x / nelem, e = threadIdx.x - q * nelem;
  const bool mine = q < G;
  const cx<T> acc = mine ? element(e, q) : mk((T)0, (T)0);
  sg_finish<T>(out, nullptr, part, G, nelem, mine, e, acc);
}

constexpr int SG_DB = 4;  // dot products per pass over w

// h[j] = V_j^H w, j < nv (V_j = V + j vsj), summed in FP64; h in shared memory
template <typename T>
__device__ void sg_dots(cx<double>* h, const cx<T>* V, size_t vsj, int nv, const cx<T>* w, int n,
                        cx<double> (*red)[SG_T / 64]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j0 = 0; j0 < nv; j0 += SG_DB) {
    cx<double> acc[SG_DB];
#pragma unroll
    for (int q = 0; q < SG_DB; ++q) acc[q] = mk(0.0, 0.0);
    for (int e = threadIdx.x; e < n; e += SG_T) {
      const cx<double> wv = cvt<double>(w[e]);
#pragma unroll
      for (int q = 0; q < SG_DB; ++q)
        if (j0 + q < nv) acc[q] = acc[q] + cmulc(cvt<double>(V[(size_t)(j0 + q) * vsj + e]), wv);
    }
#pragma unroll
    for (int q = 0; q < SG_DB; ++q) {
      const double re = wave_sum_d(acc[q].r), im = wave_sum_d(acc[q].i);
      if (lane == 0) red[q][wid] = mk(re, im);
    }
    __syncthreads();
    if (threadIdx.x < SG_DB && j0 + threadIdx.x < nv) {
      cx<double> sum = mk(0.0, 0.0);
      for (int k = 0; k < SG_T / 64; ++k) sum = sum + red[threadIdx.x][k];
      h[j0 + threadIdx.x] = sum;
    }
    __syncthreads();
  }
}

// w[e] = f * (w[e] - sum_{j < nv} h[j] V_j[e])
template <typename T>
__device__ void sg_update(cx<T>* w, const cx<T>* V, size_t vsj, int nv, const cx<double>* h, double f, int n) {
  for (int e = threadIdx.x; e < n; e += SG_T) {
    cx<T> acc = w[e];
    for (int j = 0; j < nv; ++j) acc = acc + cvt<T>(-1.0 * h[j]) * V[(size_t)j * vsj + e];
    w[e] = cvt<T>(f * cvt<double>(acc));
  }
  __syncthreads();
}

template <typename T, typename S>
__device__ void sg_schur(cx<T>* w, const cx<T>* v, cx<T>* te, cx<T>* ue, const CoarseView<S>& cv,
                         const cx<T>* Dinv, int nc, int neven, int nodd, cx<T>* part, cx<T>* xl) {
  const int nb = neven + nodd;
  sg_stencil<T, S>(te, 0, neven, nullptr, nullptr, 0, (T)0, v, neven, (T)1, cv, nc, nb, part, xl);
  sg_block_matvec<T>(ue, Dinv, te, neven, nc, part, xl);
  sg_stencil<T, S>(w, neven, nodd, nullptr, v, neven, (T)1, ue, 0, (T)-1, cv, nc, nb, part, xl);
}

template <typename T, typename S>
__global__ __launch_bounds__(SG_T) void coarse_gmres_small_kernel(cx<T>* xc, const cx<T>* yc, size_t cstr,
                                                                  CoarseView<S> cv, const cx<T>* Dinv, int nc,
                                                                  int neven, int nodd, cx<T>* te_, cx<T>* ue_,
                                                                  cx<T>* bo_, cx<T>* cw_, cx<T>* V_, size_t vsj,
                                                                  int m, int maxit, double tol, int* its_stat) {
  __shared__ cx<double> red[SG_DB][SG_T / 64];
  __shared__ cx<double> h1[SG_M + 1], h2[SG_M + 1];
  // the Hessenberg matrix (column k at H + k (m + 1)), the rotations, the
  // rotated rhs and the back-substituted coefficients: thread 0 updates
  // them serially, so they live in LDS rather than behind global latency
  __shared__ cx<double> H[(SG_M + 1) * SG_M], sn[SG_M], g[SG_M + 1], yv[SG_M];
  __shared__ double cs[SG_M];
  __shared__ cx<T> part[SG_T];
  __shared__ cx<T> xl[COARSE_SMALL_MAX_VECTOR];
  __shared__ int sh;
  const int r = blockIdx.x;
  const int nb = neven + nodd;
  const int ne = neven * nc, no = nodd * nc;
  const cx<T>* y = yc + (size_t)r * cstr;
  cx<T>* x = xc + (size_t)r * cstr;
  cx<T>* xo = x + ne;
  cx<T>* te = te_ + (size_t)r * ne;
  cx<T>* ue = ue_ + (size_t)r * ne;
  cx<T>* bo = bo_ + (size_t)r * no;
  cx<T>* cw = cw_ + (size_t)r * no;
  cx<T>* V = V_ + (size_t)r * no;  // V_j = V + j vsj
  // |y_c| -> absolute tolerance (tol < 0: never test)
  sg_dots<T>(h1, y, 0, 1, y, ne + no, red);
  const double abstol = tol < 0.0 ? -1.0 : tol * sqrt(fmax(h1[0].r, 0.0));
  // b_o = y_o - D_oe D_ee^{-1} y_e, x_o = 0
  sg_block_matvec<T>(te, Dinv, y, neven, nc, part, xl);
  sg_stencil<T, S>(bo, neven, nodd, y + ne, nullptr, 0, (T)0, te, 0, (T)-1, cv, nc, nb, part, xl);
  for (int e = threadIdx.x; e < no; e += SG_T) xo[e] = mk((T)0, (T)0);
  __syncthreads();
  int its = 0;
  bool first = true;
  while (its < maxit) {
    // r = b_o - S x_o into V_0, its norm, the start of a cycle
    if (first) {
      for (int e = threadIdx.x; e < no; e += SG_T) V[e] = bo[e];
      __syncthreads();
    } else {
      sg_schur<T, S>(cw, xo, te, ue, cv, Dinv, nc, neven, nodd, part, xl);
      for (int e = threadIdx.x; e < no; e += SG_T) V[e] = bo[e] - cw[e];
      __syncthreads();
    }
    first = false;
    sg_dots<T>(h1, V, 0, 1, V, no, red);
    const double beta = sqrt(fmax(h1[0].r, 0.0));
    const bool act = abstol < 0.0 ? beta > 0.0 : beta > abstol;
    if (!act) break;  // uniform: every lane computed beta from the same sums
    if (threadIdx.x == 0) {
      for (int j = 0; j <= m; ++j) g[j] = mk(0.0, 0.0);
      g[0] = mk(beta, 0.0);
    }
    sg_update<T>(V, V, vsj, 0, h1, 1.0 / beta, no);
    int k = 0;
    for (; k < m && its < maxit; ++k) {
      cx<T>* w = V + (size_t)(k + 1) * vsj;
      sg_schur<T, S>(w, V + (size_t)k * vsj, te, ue, cv, Dinv, nc, neven, nodd, part, xl);
      // classical Gram-Schmidt twice, then |w|^2
      sg_dots<T>(h1, V, vsj, k + 1, w, no, red);
      sg_update<T>(w, V, vsj, k + 1, h1, 1.0, no);
      sg_dots<T>(h2, V, vsj, k + 1, w, no, red);
      sg_update<T>(w, V, vsj, k + 1, h2, 1.0, no);
      sg_dots<T>(h2 + k + 1, w, 0, 1, w, no, red);
      int stop = 0;
      double hn = 0.0;
      if (threadIdx.x == 0) {
        cx<double>* Hk = H + (size_t)k * (m + 1);
        for (int j = 0; j <= k; ++j) Hk[j] = h1[j] + h2[j];
        hn = sqrt(fmax(h2[k + 1].r, 0.0));
        Hk[k + 1] = mk(hn, 0.0);
        for (int j = 0; j < k; ++j) {
          const double c = cs[j];
          const cx<double> sj = sn[j];
          const cx<double> t = c * Hk[j] + sj * Hk[j + 1];
          Hk[j + 1] = c * Hk[j + 1] - conj(sj) * Hk[j];
          Hk[j] = t;
        }
        double c;
        cx<double> sv, rr;
        givens(Hk[k], Hk[k + 1], c, sv, rr);
        cs[k] = c;
        sn[k] = sv;
        Hk[k] = rr;
        Hk[k + 1] = mk(0.0, 0.0);
        const cx<double> gk = g[k];
        g[k + 1] = neg(conj(sv) * gk);
        g[k] = c * gk;
        const double est = sqrt(cabs2(g[k + 1]));
        stop = (!(hn > 0.0) || (abstol >= 0.0 && est <= abstol) || k + 1 >= m) ? 1 : 0;
      }
      stop = sg_flag(&sh, stop);
      ++its;
      if (stop) {
        ++k;
        break;
      }
      const double inv = 1.0 / sqrt(fmax(h2[k + 1].r, 0.0));
      sg_update<T>(w, V, vsj, 0, h1, inv, no);
    }
    // y = H^{-1} g (upper triangular, k columns), then x_o += V y
    if (threadIdx.x == 0) {
      for (int i = k - 1; i >= 0; --i) {
        cx<double> v = g[i];
        for (int j = i + 1; j < k; ++j) v = v - H[(size_t)j * (m + 1) + i] * yv[j];
        const cx<double> d = H[(size_t)i * (m + 1) + i];
        const double dn = cabs2(d);
        yv[i] = dn > 0.0 ? (1.0 / dn) * (conj(d) * v) : mk(0.0, 0.0);
      }
      for (int j = 0; j < k; ++j) h1[j] = neg(yv[j]);
    }
    __syncthreads();
    sg_update<T>(xo, V, vsj, k, h1, 1.0, no);
  }
  // x_e = D_ee^{-1} (y_e - D_eo x_o)
  sg_stencil<T, S>(te, 0, neven, y, nullptr, 0, (T)0, xo, neven, (T)-1, cv, nc, nb, part, xl);
  sg_block_matvec<T>(x, Dinv, te, neven, nc, part, xl);
  if (threadIdx.x == 0) {
    atomicAdd(its_stat, its);
    atomicMax(its_stat + 1, its);
  }
}

// abstol[r] = tol * sqrt(|n2[r]|) (tol < 0: -1, i.e. never test)
__global__ void set_abstol_kernel(double* abstol, const cx<double>* n2, double tol, int nrhs) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  abstol[r] = tol < 0.0 ? -1.0 : tol * sqrt(fmax(n2[r].r, 0.0));
}

// s[r] = 1 / sqrt(n2[r]); flags a zero or non-finite norm in *status
__global__ void inv_norm_kernel(double* s, const cx<double>* n2, int nrhs, int* status) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  const double nr = sqrt(fmax(n2[r].r, 0.0));
  if (!(nr > 0.0) || !isfinite(nr)) {
    atomicExch(status, 1);
    s[r] = 0.0;
  } else {
    s[r] = 1.0 / nr;
  }
}

}  // namespace

template <typename T, typename S>
void launch_coarse_gmres_small(cx<T>* xc, const cx<T>* yc, size_t cstr, const CoarseView<S>& cv, const cx<T>* Dinv,
                               const Geom& g, cx<T>* te, cx<T>* ue, cx<T>* bo, cx<T>* cw, cx<T>* V, size_t vsj,
                               int m, int maxit, double tol, int* its_stat, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  if (m < 1 || m > SG_M || g.nblocks * g.nc > COARSE_SMALL_MAX_VECTOR)
    throw std::runtime_error("single-kernel coarse solve: restart length or lattice above its bound");
  coarse_gmres_small_kernel<T, S><<<nrhs, SG_T, 0, st>>>(xc, yc, cstr, cv, Dinv, g.nc, g.neven,
                                                          g.nblocks - g.neven, te, ue, bo, cw, V, vsj, m, maxit, tol,
                                                          its_stat);
}
template void launch_coarse_gmres_small<double, double>(cx<double>*, const cx<double>*, size_t,
                                                        const CoarseView<double>&, const cx<double>*, const Geom&,
                                                        cx<double>*, cx<double>*, cx<double>*, cx<double>*,
                                                        cx<double>*, size_t, int, int, double, int*, int,
                                                        hipStream_t);
template void launch_coarse_gmres_small<float, float>(cx<float>*, const cx<float>*, size_t, const CoarseView<float>&,
                                                      const cx<float>*, const Geom&, cx<float>*, cx<float>*,
                                                      cx<float>*, cx<float>*, cx<float>*, size_t, int, int, double,
                                                      int*, int, hipStream_t);
template void launch_coarse_gmres_small<float, __half>(cx<float>*, const cx<float>*, size_t,
                                                       const CoarseView<__half>&, const cx<float>*, const Geom&,
                                                       cx<float>*, cx<float>*, cx<float>*, cx<float>*, cx<float>*,
                                                       size_t, int, int, double, int*, int, hipStream_t);

void launch_set_abstol(double* abstol, const cx<double>* n2, double tol, int nrhs, hipStream_t st) {
  set_abstol_kernel<<<1, 64, 0, st>>>(abstol, n2, tol, nrhs);
}
void launch_inv_norm(double* s, const cx<double>* n2, int nrhs, int* status, hipStream_t st) {
  inv_norm_kernel<<<1, 64, 0, st>>>(s, n2, nrhs, status);
}

template <typename T>
bool launch_mdot(cx<double>* h, int ldh, cx<double>* part, size_t part_cap, const cx<T>* Vb, size_t vsj, size_t vsr,
                 int nvec, const cx<T>* w, size_t wsr, size_t n, int nrhs, const int* active, hipStream_t st) {
  if (nrhs <= 0 || nvec <= 0) return true;
  if (nvec > MAX_MDOT_VECS || mdot_part_entries(n, nvec, nrhs) > part_cap) return false;
  const int nchunk = blas_nchunks(n);
  const size_t chunk = (n + nchunk - 1) / nchunk;
  mdot_partial_kernel<T><<<dim3(nchunk, nrhs), BT, 0, st>>>(part, Vb, vsj, vsr, nvec, w, wsr, n, chunk, nchunk,
                                                            active, h, ldh);
  if (nchunk > 1) mdot_final_kernel<<<dim3(nvec, nrhs), 64, 0, st>>>(h, ldh, part, nvec, nchunk, active);
  return true;
}

template <typename Tw, typename Tv>
void launch_maxpy(cx<Tw>* w, size_t wsr, const cx<Tv>* Vb, size_t vsj, size_t vsr, int nvec, const cx<double>* h,
                  int ldh, double sign, size_t n, int nrhs, const int* active, hipStream_t st, const double* post,
                  cx<float>* w32) {
  if (nrhs <= 0 || (nvec <= 0 && !post && !w32)) return;
  maxpy_kernel<Tw, Tv>
      <<<dim3(grid_for(n), nrhs), BT, 0, st>>>(w, wsr, Vb, vsj, vsr, nvec, h, ldh, sign, n, active, post, w32);
}

bool launch_gs_fused(cx<double>* h2, int ldh, cx<double>* part, size_t part_cap, const cx<double>* Vb, size_t vsj,
                     size_t vsr, int nvec, cx<double>* w, size_t wsr, const cx<double>* h1, size_t n, int nrhs,
                     const int* active, hipStream_t st) {
  if (nrhs <= 0 || nvec <= 0) return true;
  if (nvec > GS_FUSED_MAXV || mdot_part_entries(n, nvec + 1, nrhs) > part_cap) return false;
  const int nchunk = blas_nchunks(n);
  const size_t chunk = (n + nchunk - 1) / nchunk;
  // the narrowest instance that holds nvec basis entries per element (fewer
  // registers, more waves in flight for this streaming kernel)
  const dim3 grid(nchunk, nrhs);
  if (nvec <= 4)
    gs_fused_kernel<4><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, nvec, w, wsr, h1, ldh, n, chunk, nchunk, active, h2);
  else if (nvec <= 8)
    gs_fused_kernel<8><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, nvec, w, wsr, h1, ldh, n, chunk, nchunk, active, h2);
  else if (nvec <= 16)
    gs_fused_kernel<16><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, nvec, w, wsr, h1, ldh, n, chunk, nchunk, active, h2);
  else
    gs_fused_kernel<GS_FUSED_MAXV><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, nvec, w, wsr, h1, ldh, n, chunk, nchunk,
                                                        active, h2);
  if (nchunk > 1) mdot_final_kernel<<<dim3(nvec + 1, nrhs), 64, 0, st>>>(h2, ldh, part, nvec + 1, nchunk, active);
  return true;
}

bool launch_gs_defer(cx<double>* h2, int ldh, cx<double>* part, size_t part_cap, cx<double>* Vb, size_t vsj,
                     size_t vsr, int k, bool correct, const cx<double>* c, const double* sigma, cx<double>* w,
                     size_t wsr, const cx<double>* h, size_t n, int nrhs, const int* active, cx<float>* w32,
                     const double* wsc, hipStream_t st) {
  if (nrhs <= 0) return true;
  const int nvec = k + 1;
  if (nvec > GS_FUSED_MAXV || mdot_part_entries(n, nvec + 1, nrhs) > part_cap) return false;
  const int nchunk = blas_nchunks(n);
  const size_t chunk = (n + nchunk - 1) / nchunk;
  dim3 grid(nchunk, nrhs);
  const int cr = correct ? 1 : 0;
  if (nvec <= 4)
    gs_defer_kernel<4><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, k, cr, c, ldh, sigma, w, wsr, h, ldh, n, chunk, nchunk,
                                            active, h2, w32, wsc);
  else if (nvec <= 8)
    gs_defer_kernel<8><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, k, cr, c, ldh, sigma, w, wsr, h, ldh, n, chunk, nchunk,
                                            active, h2, w32, wsc);
  else if (nvec <= 16)
    gs_defer_kernel<16><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, k, cr, c, ldh, sigma, w, wsr, h, ldh, n, chunk,
                                             nchunk, active, h2, w32, wsc);
  else
    gs_defer_kernel<GS_FUSED_MAXV><<<grid, BT, 0, st>>>(part, Vb, vsj, vsr, k, cr, c, ldh, sigma, w, wsr, h, ldh, n,
                                                        chunk, nchunk, active, h2, w32, wsc);
  if (nchunk > 1)
    mdot_final_kernel<<<dim3(nvec + 1, nrhs), 64, 0, st>>>(h2, ldh, part, nvec + 1, nchunk, active);
  return true;
}

void launch_gs_defer_coef(cx<double>* h, cx<double>* c, const cx<double>* h2, int ldh, const double* sigma, int k,
                          bool correct, double* wsc, int nrhs, const int* active, hipStream_t st) {
  gs_defer_coef_kernel<<<1, 64, 0, st>>>(h, c, h2, ldh, sigma, k, correct ? 1 : 0, wsc, nrhs, active);
}

void launch_gs_norm(cx<double>* n2, double* inv, const cx<double>* h2, int ldh, int nvec, int nrhs, const int* active,
                    hipStream_t st) {
  gs_norm_kernel<<<1, 64, 0, st>>>(n2, inv, h2, ldh, nvec, nrhs, active);
}

template <typename Ty, typename Tx>
void launch_scale(cx<Ty>* y, size_t ystr, const cx<Tx>* x, size_t xstr, const double* s, size_t n, int nrhs,
                  const int* active, hipStream_t st, cx<float>* y32) {
  if (nrhs <= 0) return;
  scale_kernel<Ty, Tx><<<dim3(grid_for(n), nrhs), BT, 0, st>>>(y, ystr, x, xstr, s, n, active, y32);
}

template <typename T>
void launch_sub(cx<T>* y, size_t ystr, const cx<T>* a, size_t astr, const cx<T>* b, size_t bstr, size_t n, int nrhs,
                hipStream_t st) {
  if (nrhs <= 0) return;
  sub_kernel<T><<<dim3(grid_for(n), nrhs), BT, 0, st>>>(y, ystr, a, astr, b, bstr, n);
}

template <typename Ty, typename Tx>
void launch_copy(cx<Ty>* y, size_t ystr, const cx<Tx>* x, size_t xstr, size_t n, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  copy_kernel<Ty, Tx><<<dim3(grid_for(n), nrhs), BT, 0, st>>>(y, ystr, x, xstr, n);
}

void launch_arnoldi_start(ArnoldiState s, const cx<double>* norm2, int ldn, int nrhs, hipStream_t st) {
  arnoldi_start_kernel<<<1, 64, 0, st>>>(s, norm2, ldn, nrhs);
}
void launch_arnoldi_column(ArnoldiState s, int k, const cx<double>* h1, const cx<double>* h2, int ldh,
                           const cx<double>* norm2, int ldn, int nrhs, hipStream_t st) {
  arnoldi_column_kernel<<<1, 64, 0, st>>>(s, k, h1, h2, ldh, norm2, ldn, nrhs);
}
void launch_arnoldi_solve(ArnoldiState s, int nrhs, hipStream_t st) {
  arnoldi_solve_kernel<<<1, 64, 0, st>>>(s, nrhs);
}

template bool launch_mdot<double>(cx<double>*, int, cx<double>*, size_t, const cx<double>*, size_t, size_t, int,
                                  const cx<double>*, size_t, size_t, int, const int*, hipStream_t);
template bool launch_mdot<float>(cx<double>*, int, cx<double>*, size_t, const cx<float>*, size_t, size_t, int,
                                 const cx<float>*, size_t, size_t, int, const int*, hipStream_t);
#define INST2(A, B)                                                                                                   \
  template void launch_maxpy<A, B>(cx<A>*, size_t, const cx<B>*, size_t, size_t, int, const cx<double>*, int, double, \
                                   size_t, int, const int*, hipStream_t, const double*, cx<float>*);                  \
  template void launch_scale<A, B>(cx<A>*, size_t, const cx<B>*, size_t, const double*, size_t, int, const int*,      \
                                   hipStream_t, cx<float>*);                                                          \
  template void launch_copy<A, B>(cx<A>*, size_t, const cx<B>*, size_t, size_t, int, hipStream_t);
INST2(double, double)
INST2(float, float)
INST2(double, float)
INST2(float, double)
#undef INST2
template void launch_sub<double>(cx<double>*, size_t, const cx<double>*, size_t, const cx<double>*, size_t, size_t, int,
                                 hipStream_t);
template void launch_sub<float>(cx<float>*, size_t, const cx<float>*, size_t, const cx<float>*, size_t, size_t, int,
                                hipStream_t);

}  // namespace ddamg
