// Setup kernels of Alg. 5: orthonormalisation of the test vectors on every
// aggregate (Gram-Schmidt on the rows of R_i^h) and the storage formats of
// the resulting basis.
//
// The paper uses classical block Gram-Schmidt for fewer global sums and
// better cache reuse.  Here every aggregate (block, chirality h: 6 V_block
// rows, ntv columns) runs CholQR2 in FP64, all aggregates at once: the Gram
// matrix X^H X, its Cholesky factor (positive real diagonal) and X <- X T^{-1};
// doing it twice restores orthogonality to rounding.  The result is the
// unique Q of X = Q T with positive diag(T), i.e. the basis Gram-Schmidt
// produces.
#include "ddamg_internal.h"

namespace ddamg {

namespace {

constexpr int QR_THREADS = 256;
constexpr int MAX_NTV = 32;
constexpr int QR_CS = 8;             // sites per staged chunk of the Gram matrix pass
constexpr int QR_ROWS = QR_CS * 6;   // rows (site, spin-colour) per chunk
constexpr int QR_LD = MAX_NTV + 1;   // padded LDS row
// An aggregate is (internal block ci, chirality h): rows are the 6 V_block
// (spin of chirality h x colour, site) entries, columns the ntv test
// vectors.  Per CholQR pass, three kernels with one workgroup per aggregate:
//   G = X^H X: on the FP64 matrix cores.  A 16x16x4 f64 MFMA takes, in lane
//              l, entry (row l/16, column l%16) of a 4-row slice for both of
//              its operands, so one load per lane and column tile feeds all
//              of Re/Im X^T X; the waves split the rows and their partial
//              tiles are summed through LDS.  Every entry of X is read once.
//              G goes to the per-aggregate workspace.  The kernel holds no
//              LDS beyond its staging buffer, so several aggregates share a
//              compute unit and keep enough loads in flight.
//   G = T^H T: Cholesky (real positive diagonal) and T^{-1} by back
//              substitution, one 64-lane workgroup per aggregate on an
//              ntv x (ntv+1) LDS matrix; T^{-1} replaces G in the workspace;
//   X <- X T^{-1}: on the FP64 matrix cores, tiles of 16 sites x 16 test
//              vectors (in place for the second pass).
typedef double qr_v4d __attribute__((ext_vector_type(4)));

// Column layouts of the Gram tiles (upper triangle of G = X^H X, 16x16
// tiles, one lane per column in each operand):
//   NT = 1, ntv <= 16: columns 0..15 x 0..15;
//   NT = 2, ntv <= 24: columns 0..15 x 8..23 and {0..7, 16..23} x {0..7,
//          16..23}: with columns in groups of eight, two tiles hold every
//          pair i <= j (the pairs 0..7 x 16..23 of the second are dropped);
//   NT = 3, ntv <= 32: 0..15 x 0..15, 0..15 x 16..31 and 16..31 x 16..31.
template <typename Tin, int NT>
__global__ __launch_bounds__(QR_THREADS) void qr_gram_kernel(const cx<Tin>* W, Geom g, cx<double>* Gout) {
  constexpr int NACC = 2 * NT;  // Re and Im of each tile
  // the staged rows of the Gram matrix pass, later the partial tiles of two
  // waves
  constexpr size_t STAGE_BYTES = sizeof(cx<double>) * QR_ROWS * QR_LD > sizeof(qr_v4d) * 2 * NACC * 64
                                     ? sizeof(cx<double>) * QR_ROWS * QR_LD
                                     : sizeof(qr_v4d) * 2 * NACC * 64;
  __shared__ __attribute__((aligned(32))) char stage_raw[STAGE_BYTES];
  auto Xs = reinterpret_cast<cx<double>(*)[QR_LD]>(stage_raw);
  auto part = reinterpret_cast<qr_v4d(*)[NACC][64]>(stage_raw);
  const int ci = blockIdx.x >> 1;  // internal block: its sites are ci * vblock + [0, vblock)
  const int h = blockIdx.x & 1;
  const int n = g.ntv;
  const size_t V = g.V;
  const int vb = g.vblock;
  const int l = threadIdx.x, lane = l & 63, w = l >> 6;
  const size_t base = (size_t)ci * vb;
  const int col0 = lane & 15, rsub = lane >> 4;
  // operand columns of this lane: ca (first operand of tile 0), cb (second
  // operand of tile 0), cc (both operands of the last tile)
  const int ca = col0;
  const int cb = NT == 2 ? 8 + col0 : col0;
  const int cc = NT == 2 ? (col0 < 8 ? col0 : col0 + 8) : 16 + col0;
  qr_v4d acc[NACC];
#pragma unroll
  for (int t = 0; t < NACC; ++t) acc[t] = (qr_v4d){0.0, 0.0, 0.0, 0.0};
  // Rows (site, spin-colour) of QR_CS sites at a time are staged in LDS with
  // coalesced loads (QR_CS consecutive sites of one test vector and
  // component); the loads of the next two chunks are in flight, held in the
  // input precision, while the MFMAs consume the current one.  Padded test
  // vectors (a >= ntv) are not loaded.
  constexpr int NQ = QR_ROWS * 32 / 256;
  cx<Tin> xq0[NQ], xq1[NQ];
  auto fetch = [&](cx<Tin>(&xq)[NQ], int s0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = l + 256 * q;
      const int sl = e % QR_CS, rest = e / QR_CS, c = rest % 6, a = rest / 6;
      const int sx = min(s0 + sl, vb - 1);
      xq[q] = a < n ? W[((size_t)a * 12 + 6 * h + c) * V + base + sx] : mk((Tin)0, (Tin)0);
    }
  };
  auto chunk = [&](cx<Tin>(&xq)[NQ], int s0) {
    __syncthreads();  // the previous chunk has been consumed
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = l + 256 * q;
      const int sl = e % QR_CS, rest = e / QR_CS, c = rest % 6, a = rest / 6;
      Xs[sl * 6 + c][a] = s0 + sl < vb ? cvt<double>(xq[q]) : mk(0.0, 0.0);
    }
    if (s0 + 2 * QR_CS < vb) fetch(xq, s0 + 2 * QR_CS);
    __syncthreads();
    // 4-row slices; the two products feeding one accumulator are issued
    // apart so no MFMA waits on the one before it
    for (int t = w; t < QR_ROWS / 4; t += 4) {
      const cx<double> y0 = Xs[4 * t + rsub][ca];
      if constexpr (NT == 1) {
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, y0.r, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, y0.i, acc[1], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.i, y0.i, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y0.i, y0.r, acc[1], 0, 0, 0);
      } else if constexpr (NT == 2) {
        const cx<double> yb = Xs[4 * t + rsub][cb];
        const cx<double> yc = Xs[4 * t + rsub][cc];
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, yb.r, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, yb.i, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(yc.r, yc.r, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(yc.r, yc.i, acc[3], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.i, yb.i, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y0.i, yb.r, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(yc.i, yc.i, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(-yc.i, yc.r, acc[3], 0, 0, 0);
      } else {
        const cx<double> y1 = Xs[4 * t + rsub][cc];
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, y0.r, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, y0.i, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, y1.r, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.r, y1.i, acc[3], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1.r, y1.r, acc[4], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1.r, y1.i, acc[5], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.i, y0.i, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y0.i, y0.r, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0.i, y1.i, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y0.i, y1.r, acc[3], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1.i, y1.i, acc[4], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y1.i, y1.r, acc[5], 0, 0, 0);
      }
    }
  };
  fetch(xq0, 0);
  if (QR_CS < vb) fetch(xq1, QR_CS);
  for (int s0 = 0; s0 < vb; s0 += 2 * QR_CS) {
    chunk(xq0, s0);
    if (s0 + QR_CS < vb) chunk(xq1, s0 + QR_CS);
  }
  __syncthreads();  // the staging buffer is reused for the partial tiles
  // sum the four waves' tiles: waves 2,3 hand theirs to waves 0,1, then wave 1
  // to wave 0, which writes the upper triangle of G (row-major, stride
  // MAX_NTV)
  if (w >= 2)
#pragma unroll
    for (int t = 0; t < NACC; ++t) part[w - 2][t][lane] = acc[t];
  __syncthreads();
  if (w < 2)
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t] += part[w][t][lane];
  __syncthreads();
  if (w == 1)
#pragma unroll
    for (int t = 0; t < NACC; ++t) part[0][t][lane] = acc[t];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t] += part[0][t][lane];
    cx<double>* G = Gout + (size_t)blockIdx.x * QR_TWS_PER_AGG;
    // f64 16x16x4 result v of lane l: row l/16 + 4v (first operand's
    // column), column l%16 (second operand's column)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rsub + 4 * v, j = col0;
      if constexpr (NT == 1) {
        if (i < n && j < n) G[i * MAX_NTV + j] = mk(acc[0][v], acc[1][v]);
      } else if constexpr (NT == 2) {
        const int ib = 8 + j;  // tile 0: rows 0..15, columns 8..23
        if (i <= ib && ib < n) G[i * MAX_NTV + ib] = mk(acc[0][v], acc[1][v]);
        const int ic = i < 8 ? i : i + 8, jc = j < 8 ? j : j + 8;  // tile 1
        if (ic <= jc && jc < n && !(ic < 8 && jc >= 16)) G[ic * MAX_NTV + jc] = mk(acc[2][v], acc[3][v]);
      } else {
        if (i < n && j < n) G[i * MAX_NTV + j] = mk(acc[0][v], acc[1][v]);
        if (i < n && 16 + j < n) G[i * MAX_NTV + 16 + j] = mk(acc[2][v], acc[3][v]);
        if (16 + i < n && 16 + j < n) G[(16 + i) * MAX_NTV + 16 + j] = mk(acc[4][v], acc[5][v]);
      }
    }
  }
}

// Cholesky G = T^H T (T upper, real positive diagonal) and T^{-1} of one
// aggregate per 64-lane workgroup.  G (upper triangle, stride MAX_NTV) is
// read from the workspace into an n x (n+1) LDS matrix; T overwrites its
// upper triangle and the strictly upper part of T^{-1} is kept transposed in
// the free lower triangle, its diagonal in dg.  T^{-1} (n x n, row-major)
// replaces G in the workspace; a pivot that is not positive sets *status
// and leaves zeros.
__global__ __launch_bounds__(64) void qr_chol_kernel(cx<double>* tws, Geom g, int* status) {
  extern __shared__ cx<double> sh[];
  __shared__ double dg[MAX_NTV];
  __shared__ int fail;
  const int n = g.ntv, ld = n + 1;
  const int l = threadIdx.x;
  cx<double>* Tg = tws + (size_t)blockIdx.x * QR_TWS_PER_AGG;
  for (int e = l; e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    if (j >= i) sh[i * ld + j] = Tg[i * MAX_NTV + j];
  }
  if (l == 0) fail = 0;
  __syncthreads();
  // right-looking: step k scales row k by the pivot and updates the
  // trailing upper triangle, its entries spread over the lanes
  for (int k = 0; k < n; ++k) {
    const double dk = sh[k * ld + k].r;  // every lane reads the same pivot
    if (!(dk > 0.0)) {
      if (l == 0) fail = 1;
      break;
    }
    const double d = sqrt(dk);
    __syncthreads();
    for (int j = k + l; j < n; j += 64) sh[k * ld + j] = j == k ? mk(d, 0.0) : (1.0 / d) * sh[k * ld + j];
    __syncthreads();
    const int m = n - k - 1;  // trailing size
    for (int p = l; p < m * m; p += 64) {
      const int i = k + 1 + p / m, j = k + 1 + p % m;
      if (j >= i) sh[i * ld + j] = sh[i * ld + j] - cmulc(sh[k * ld + i], sh[k * ld + j]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail) {
    if (l == 0) atomicExch(status, 1);
    for (int e = l; e < n * n; e += 64) Tg[e] = mk(0.0, 0.0);
    return;
  }
  // T^{-1} by back substitution, one column j per lane: entry (i, j), i < j,
  // lives at sh[j][i]; lane j reads T (i < mm) and its own column only
  if (l < n) {
    const int j = l;
    dg[j] = 1.0 / sh[j * ld + j].r;
#pragma unroll 1
    for (int i = j - 1; i >= 0; --i) {
      cx<double> vv = mk(0.0, 0.0);
#pragma unroll 1
      for (int mm = i + 1; mm < j; ++mm) vv = cfma(sh[i * ld + mm], sh[j * ld + mm], vv);
      vv = cfma(sh[i * ld + j], mk(dg[j], 0.0), vv);
      sh[j * ld + i] = (-1.0 / sh[i * ld + i].r) * vv;
    }
  }
  __syncthreads();
  for (int e = l; e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    Tg[e] = i < j ? sh[j * ld + i] : i == j ? mk(dg[i], 0.0) : mk(0.0, 0.0);
  }
}

// Wout <- Xin T^{-1} on the FP64 matrix cores (16x16x4 MFMA): per aggregate
// W (rows = 16 consecutive sites of one component, columns = test vectors)
// = X T^{-1}, T^{-1} (upper triangular, from the Cholesky kernel) in LDS, the
// rows of X loaded straight from memory (16 consecutive sites per lane
// group, coalesced).  The K loop runs over NQ = ceil(ntv / 4) steps of 4 test
// vectors, unrolled, with clamped loads and zero factors for the padding, so
// all loads of a tile are in flight together.  Since T^{-1} is upper
// triangular, the column tile 0..15 takes only the K steps below 16 and the
// column tile 16..31 exists only for ntv > 16: the skipped products are
// exact zeros.  The result tile is transposed through the wave's own LDS
// tile so that each store writes 16 consecutive sites (256 bytes) of 4 test
// vectors.  A wave finishes reading its row tile before it writes it and no
// other wave touches those rows, so the update may run in place.  Waves may
// run different numbers of tiles, so the LDS exchange is ordered by
// wave-scope fences, not workgroup barriers.
template <typename Tin, int NQ>
__global__ __launch_bounds__(QR_THREADS) void qr_update_mfma_kernel(cx<double>* Wout, const cx<Tin>* Xin, Geom g,
                                                                    const cx<double>* Tinv) {
  __shared__ cx<double> Ti[MAX_NTV][MAX_NTV + 1];
  __shared__ cx<double> Sw[QR_THREADS / 64][MAX_NTV * 17];
  const int ci = blockIdx.x >> 1;
  const int h = blockIdx.x & 1;
  const int n = g.ntv;
  const size_t V = g.V;
  const int vb = g.vblock;
  const int l = threadIdx.x, lane = l & 63, w = l >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  const size_t base = (size_t)ci * vb;
  const int tiles_per_comp = (vb + 15) / 16;
  const int ntile = 6 * tiles_per_comp;
  // the X rows of this wave's next tile, loaded (in the input precision)
  // while the current tile is multiplied and stored; the rows of different
  // tiles are disjoint, so this holds in place too
  cx<Tin> xr[NQ];
  auto fetch = [&](int tile) {
    const int c = tile / tiles_per_comp, s0 = (tile % tiles_per_comp) * 16;
    const int sa = min(s0 + i16, vb - 1);  // A operand: site of this lane's row (clamped)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = min(4 * q + k4, n - 1);
      xr[q] = Xin[((size_t)k * 12 + 6 * h + c) * V + base + sa];
    }
  };
  if (w < ntile) fetch(w);
  const cx<double>* Tg = Tinv + (size_t)blockIdx.x * MAX_NTV * MAX_NTV;
  for (int e = l; e < MAX_NTV * MAX_NTV; e += blockDim.x) {
    const int i = e / MAX_NTV, j = e % MAX_NTV;
    Ti[i][j] = (i < n && j < n) ? Tg[i * n + j] : mk(0.0, 0.0);
  }
  __syncthreads();
  for (int tile = w; tile < ntile; tile += QR_THREADS / 64) {
    const int c = tile / tiles_per_comp, s0 = (tile % tiles_per_comp) * 16;
    cx<double> xa[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) xa[q] = cvt<double>(xr[q]);
    if (tile + QR_THREADS / 64 < ntile) fetch(tile + QR_THREADS / 64);
    qr_v4d RR[2], II[2], RI[2], IR[2];
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) RR[tj][v] = II[tj][v] = RI[tj][v] = IR[tj][v] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double f = 4 * q + k4 < n ? 1.0 : 0.0;  // padded test vectors add nothing
      const double ar = f * xa[q].r, ai = f * xa[q].i;
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        if (tj == 0 && q >= 4) continue;  // rows 16.. of T^{-1} vanish in columns 0..15
        if (tj == 1 && NQ <= 4) continue;  // no columns 16..31
        const cx<double> b = Ti[4 * q + k4][16 * tj + i16];
        RR[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b.r, RR[tj], 0, 0, 0);
        II[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b.i, II[tj], 0, 0, 0);
        RI[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b.i, RI[tj], 0, 0, 0);
        IR[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b.r, IR[tj], 0, 0, 0);
      }
    }
    // result row lane / 16 + 4 v (site), column lane % 16 (test vector):
    // transposed through this wave's LDS tile [column][site] (stride 17)
    cx<double>* St = Sw[w];
#pragma unroll
    for (int tj = 0; tj < (NQ > 4 ? 2 : 1); ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        St[(16 * tj + i16) * 17 + k4 + 4 * v] = mk(RR[tj][v] - II[tj][v], RI[tj][v] + IR[tj][v]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < (NQ > 4 ? 8 : 4); ++r) {
      const int j = 4 * r + k4, srow = s0 + i16;
      if (srow < vb && j < n) Wout[((size_t)j * 12 + 6 * h + c) * V + base + srow] = St[j * 17 + i16];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <typename S>
__global__ void quantize_basis_kernel(stc_t<S>* Wq, float* Wsc, const cx<double>* W, int V, int ntv, cx<float>* Wt) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ntv * V) return;
  const int s = (int)(idx % V);
  const int a = (int)(idx / V);
  if constexpr (is_half<S>()) {
    cx<double> v[12];  // one read of the 12 entries: max, then the scaled copy
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v[k] = W[((size_t)a * 12 + k) * V + s];
      m = fmax(m, fmax(fabs(v[k].r), fabs(v[k].i)));
    }
    const float fm = (float)m;
    Wsc[idx] = fm;
    const double inv = fm > 0.f ? 1.0 / (double)fm : 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const __half2 hq = __floats2half2_rn((float)(v[k].r * inv), (float)(v[k].i * inv));
      Wq[((size_t)a * 12 + k) * V + s] = hq;
      if (Wt) {
        const float2 f = __half22float2(hq);
        Wt[((size_t)a * 12 + k) * V + s] = mk(fm * f.x, fm * f.y);
      }
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

// the Gram kernel with the fewest column tiles for ntv (ntv <= 32 is validated)
template <typename Tin>
void launch_qr_gram(const cx<Tin>* X, const Geom& g, cx<double>* tws, hipStream_t st) {
  const unsigned nagg = 2 * g.nblocks;
  if (g.ntv <= 16)
    qr_gram_kernel<Tin, 1><<<nagg, QR_THREADS, 0, st>>>(X, g, tws);
  else if (g.ntv <= 24)
    qr_gram_kernel<Tin, 2><<<nagg, QR_THREADS, 0, st>>>(X, g, tws);
  else
    qr_gram_kernel<Tin, 3><<<nagg, QR_THREADS, 0, st>>>(X, g, tws);
}
// the update kernel for K = ceil(ntv / 4) steps (ntv <= 32 is validated)
template <typename Tin, int NQ = 8>
void launch_qr_update(cx<double>* W, const cx<Tin>* X, const Geom& g, const cx<double>* tws, hipStream_t st) {
  if constexpr (NQ > 1) {
    if ((g.ntv + 3) / 4 < NQ) {
      launch_qr_update<Tin, NQ - 1>(W, X, g, tws, st);
      return;
    }
  }
  qr_update_mfma_kernel<Tin, NQ><<<2 * g.nblocks, QR_THREADS, 0, st>>>(W, X, g, tws);
}
}  // namespace

template <typename Tin>
void launch_aggregate_qr(cx<double>* W, const cx<Tin>* X, const Geom& g, int* status, cx<double>* tws,
                         hipStream_t st) {
  // CholQR2: pass 1 from X into W, pass 2 on W in place
  const unsigned nagg = 2 * g.nblocks;
  const size_t chol_lds = sizeof(cx<double>) * g.ntv * (g.ntv + 1);
  launch_qr_gram<Tin>(X, g, tws, st);
  qr_chol_kernel<<<nagg, 64, chol_lds, st>>>(tws, g, status);
  launch_qr_update<Tin>(W, X, g, tws, st);
  launch_qr_gram<double>(W, g, tws, st);
  qr_chol_kernel<<<nagg, 64, chol_lds, st>>>(tws, g, status);
  launch_qr_update<double>(W, W, g, tws, st);
}
template void launch_aggregate_qr<double>(cx<double>*, const cx<double>*, const Geom&, int*, cx<double>*,
                                          hipStream_t);
template void launch_aggregate_qr<float>(cx<double>*, const cx<float>*, const Geom&, int*, cx<double>*, hipStream_t);

template <typename S>
void launch_quantize_basis(stc_t<S>* Wq, float* Wsc, const cx<double>* W, const Geom& g, hipStream_t st,
                           cx<float>* Wt) {
  size_t n = (size_t)g.ntv * g.V;
  quantize_basis_kernel<S><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(Wq, Wsc, W, g.V, g.ntv, Wt);
}
template <typename T, typename S>
void launch_dequantize_basis(cx<T>* out, const BasisView<S>& bv, const Geom& g, hipStream_t st) {
  size_t n = (size_t)g.ntv * 12 * g.V;
  dequantize_basis_kernel<T, S><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, bv, g.V, g.ntv);
}

template void launch_quantize_basis<double>(stc_t<double>*, float*, const cx<double>*, const Geom&, hipStream_t,
                                            cx<float>*);
template void launch_quantize_basis<float>(stc_t<float>*, float*, const cx<double>*, const Geom&, hipStream_t,
                                            cx<float>*);
template void launch_quantize_basis<__half>(stc_t<__half>*, float*, const cx<double>*, const Geom&, hipStream_t,
                                            cx<float>*);
template void launch_dequantize_basis<double, double>(cx<double>*, const BasisView<double>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<float, float>(cx<float>*, const BasisView<float>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<float, __half>(cx<float>*, const BasisView<__half>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<double, __half>(cx<double>*, const BasisView<__half>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<double, float>(cx<double>*, const BasisView<float>&, const Geom&, hipStream_t);
template void launch_dequantize_basis<float, double>(cx<float>*, const BasisView<double>&, const Geom&, hipStream_t);

}  // namespace ddamg
