// Internal declarations of the gfx950 DD-alpha-AMG library: complex and
// storage types, lattice geometry, field views and the host-side launchers
// of every kernel.  Not part of the public ABI (include/ddamg.h).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "blas_sizes.h"

namespace ddamg {

// ---------------------------------------------------------------- complex
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T r, i;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) { cx<T> c; c.r = r; c.i = i; return c; }
template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.r + b.r, a.i + b.i); }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.r - b.r, a.i - b.i); }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r);
}
template <typename T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return mk(s * a.r, s * a.i); }
template <typename T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return mk(a.r, -a.i); }
// conj(a) * b
template <typename T>
__host__ __device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r);
}
// acc + a * b and acc + conj(a) * b with four fused multiply-adds each
template <typename T>
__host__ __device__ inline cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(-a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(a.i, b.r, acc.i);
  return acc;
}
template <typename T>
__host__ __device__ inline cx<T> cfmac(cx<T> a, cx<T> b, cx<T> acc) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(-a.i, b.r, acc.i);
  return acc;
}
template <typename T>
__host__ __device__ inline cx<T> times_i(cx<T> a) { return mk(-a.i, a.r); }
template <typename T>
__host__ __device__ inline cx<T> times_mi(cx<T> a) { return mk(a.i, -a.r); }
template <typename T>
__host__ __device__ inline cx<T> neg(cx<T> a) { return mk(-a.r, -a.i); }
template <typename T, typename U>
__host__ __device__ inline cx<T> cvt(cx<U> a) { return mk((T)a.r, (T)a.i); }

// ------------------------------------------------------- storage formats
// Static fields (links, clover, aggregate basis, coarse operator) are
// stored as S = double, float or __half.  Half storage carries one FP32
// scale per group (stored value = x / scale, scale = max |re|, |im| of the
// group) so that every group fits the FP16 range with full relative
// resolution.
template <typename S> struct stc;
template <> struct stc<double> { using type = cx<double>; };
template <> struct stc<float> { using type = cx<float>; };
template <> struct stc<__half> { using type = __half2; };
template <typename S> using stc_t = typename stc<S>::type;

template <typename S> constexpr bool is_half() { return std::is_same<S, __half>::value; }

template <typename T>
__device__ inline cx<T> ldc(const cx<double>* p, size_t i) { cx<double> v = p[i]; return mk((T)v.r, (T)v.i); }
template <typename T>
__device__ inline cx<T> ldc(const cx<float>* p, size_t i) { cx<float> v = p[i]; return mk((T)v.r, (T)v.i); }
template <typename T>
__device__ inline cx<T> ldc(const __half2* p, size_t i) {
  float2 f = __half22float2(p[i]);
  return mk((T)f.x, (T)f.y);
}
// Element i < 2^28 of a field plane whose base is wave-uniform: the byte
// offset is formed in 32 bits, so the load takes the scalar-base +
// 32-bit-offset form instead of a 64-bit address per lane and load.
template <typename X>
__device__ inline const X& elem(const X* p, unsigned i) {
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(p) + i * (unsigned)sizeof(X));
}
template <typename T>
__device__ inline cx<T> ldc(const cx<double>* p, unsigned i) { cx<double> v = elem(p, i); return mk((T)v.r, (T)v.i); }
template <typename T>
__device__ inline cx<T> ldc(const cx<float>* p, unsigned i) { cx<float> v = elem(p, i); return mk((T)v.r, (T)v.i); }
template <typename T>
__device__ inline cx<T> ldc(const __half2* p, unsigned i) {
  float2 f = __half22float2(elem(p, i));
  return mk((T)f.x, (T)f.y);
}
template <typename T>
__device__ inline T ldr(const double* p, size_t i) { return (T)p[i]; }
template <typename T>
__device__ inline T ldr(const float* p, size_t i) { return (T)p[i]; }
template <typename T>
__device__ inline T ldr(const __half* p, size_t i) { return (T)__half2float(p[i]); }

__device__ inline void stc_store(cx<double>* p, size_t i, cx<double> v) { p[i] = v; }
__device__ inline void stc_store(cx<float>* p, size_t i, cx<double> v) { p[i] = mk((float)v.r, (float)v.i); }
__device__ inline void stc_store(__half2* p, size_t i, cx<double> v) {
  p[i] = __floats2half2_rn((float)v.r, (float)v.i);
}

// ---------------------------------------------------------------- geometry
// Internal site order is block-major: site S = ci * vblock + l, where l is
// the lexicographic site inside the block (x fastest) and ci the internal
// block index.  Blocks are ordered by parity (sum of block coordinates mod 2,
// i.e. the SAP colour and the coarse even/odd parity) and lexicographically
// within a parity.  With an even number of blocks along x the rank of the
// lexicographic block b inside its parity is b >> 1, so
//   ci = parity(b) * nblocks / 2 + (b >> 1).
// Every block's sites are contiguous, so block-local work (SAP, R, P,
// aggregate Gram-Schmidt) reads whole cache lines; the coarse-site order of
// coarse vectors and D_c is the same ci.
struct Geom {
  int L[4];      // lattice extents x, y, z, t
  int bs[4];     // block extents
  int NB[4];     // block-lattice extents
  int lstr[4];   // strides of the local coordinates inside a block
  int V;         // sites
  int vblock;    // sites per block
  int nblocks;   // blocks = coarse sites
  int ntv;       // test vectors
  int nc;        // coarse components per site = 2 ntv
  int neven;     // coarse sites of even parity (= nblocks / 2)
};

__host__ __device__ inline int lex_block(const Geom& g, const int bc[4]) {
  return bc[0] + g.NB[0] * (bc[1] + g.NB[1] * (bc[2] + g.NB[2] * bc[3]));
}
__host__ __device__ inline int block_to_int(const Geom& g, const int bc[4]) {
  const int p = (bc[0] + bc[1] + bc[2] + bc[3]) & 1;
  return p * g.neven + (lex_block(g, bc) >> 1);
}
// block coordinates of internal block ci
__host__ __device__ inline void int_block_coords(const Geom& g, int ci, int bc[4]) {
  const int p = ci >= g.neven ? 1 : 0;
  int b = 2 * (ci - p * g.neven);
  int t = b;
  bc[0] = t % g.NB[0]; t /= g.NB[0];
  bc[1] = t % g.NB[1]; t /= g.NB[1];
  bc[2] = t % g.NB[2];
  bc[3] = t / g.NB[2];
  if (((bc[0] + bc[1] + bc[2] + bc[3]) & 1) != p) bc[0] += 1;  // the odd partner of the pair along x
}
__host__ __device__ inline void local_coords(const Geom& g, int l, int lc[4]) {
  lc[0] = l % g.bs[0]; l /= g.bs[0];
  lc[1] = l % g.bs[1]; l /= g.bs[1];
  lc[2] = l % g.bs[2];
  lc[3] = l / g.bs[2];
}
// global coordinates of internal site S
__host__ __device__ inline void site_coords(const Geom& g, int S, int c[4]) {
  int bc[4], lc[4];
  int_block_coords(g, S / g.vblock, bc);
  local_coords(g, S % g.vblock, lc);
  for (int m = 0; m < 4; ++m) c[m] = bc[m] * g.bs[m] + lc[m];
}
// internal site of global coordinates c
__host__ __device__ inline int site_index(const Geom& g, const int c[4]) {
  int bc[4], l = 0;
  for (int m = 0; m < 4; ++m) bc[m] = c[m] / g.bs[m];
  for (int m = 3; m >= 0; --m) l = l * g.bs[m] + (c[m] - bc[m] * g.bs[m]);
  return block_to_int(g, bc) * g.vblock + l;
}
// in-block index of face site f (0 <= f < vblock / bs[mu]) of the layer
// lc[mu] = layer, the other local coordinates lexicographic
__host__ __device__ inline int face_site(const Geom& g, int mu, int layer, int f) {
  int lc[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d == mu) {
      lc[d] = layer;
    } else {
      lc[d] = f % g.bs[d];
      f /= g.bs[d];
    }
  }
  return lc[0] + g.bs[0] * (lc[1] + g.bs[1] * (lc[2] + g.bs[2] * lc[3]));
}
// MI355X has 8 XCDs with separate L2 caches and hands out consecutive
// workgroup ids round-robin over them.  xcd_swizzle maps the hardware id to
// a logical id such that each XCD works on one contiguous 1/8 of the
// logical range (when the grid divides evenly), so neighbouring lattice
// regions share an L2.
__device__ inline int xcd_swizzle(int wg, int nwg) {
  if (nwg % 8) return wg;
  return (wg & 7) * (nwg >> 3) + (wg >> 3);
}

// lexicographic (canonical) index of global coordinates c
__host__ __device__ inline int lex_site(const Geom& g, const int c[4]) {
  return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

// Links [mu][9][V] (row-major 3x3 per link), clover [2][18][V] pairs: per
// chirality the 6 real diagonal entries as 3 pairs (d0, d1), (d2, d3),
// (d4, d5), then the 15 upper off-diagonal entries (i < j, row-major) as
// (re, im); row/col index = 3 * spin_in_chirality + colour.  Pairs are
// loaded as one 4/8/16-byte word.
constexpr int CLOVER_PAIRS = 18;
template <typename S>
struct GaugeView {
  const stc_t<S>* U;
  const float* Usc;   // [V] link scale (half only)
  const stc_t<S>* A;
  const float* Asc;   // [V] clover scale (half only)
};

// Aggregate basis [ntv][12][V] complex + scale [ntv][V] (half only).
template <typename S>
struct BasisView {
  const stc_t<S>* W;
  const float* Wsc;
};

// Coarse operator, internal coarse-site order: [Nb][9][col][row] complex
// (column-major blocks) + scale [Nb][9] (half only); neighbour table
// nbr[Nb][9] in internal order.
template <typename S>
struct CoarseView {
  const stc_t<S>* D;
  const float* Dsc;
  const int* nbr;
};

// dslash variants
enum { DS_FULL = 0, DS_BLOCK = 1, DS_CROSS_FWD = 2, DS_CROSS_BWD = 3 };

// ---------------------------------------------------------------- launchers
// fields
void launch_gauge_import(cx<double>* U, const cx<double>* canon, const Geom& g, hipStream_t st);
void launch_clover_build(cx<double>* A, const cx<double>* U, const Geom& g, double m0, double csw, hipStream_t st);
template <typename S>
void launch_quantize_gauge(stc_t<S>* Uq, float* Usc, stc_t<S>* Aq, float* Asc, const cx<double>* U,
                           const cx<double>* A, const Geom& g, hipStream_t st);
template <typename T>
// nonzero (if given, nrhs ints the caller zeroed): nonzero[r] = 1 when the
// canonical field of rhs r has a nonzero entry
void launch_spinor_to_internal(cx<T>* out, const cx<double>* canon, const Geom& g, int nrhs, hipStream_t st,
                               int* nonzero = nullptr);
template <typename T>
void launch_spinor_to_canonical(cx<double>* canon, const cx<T>* in, const Geom& g, int nrhs, hipStream_t st);
void launch_clover_export(cx<double>* out, const cx<double>* A, const Geom& g, hipStream_t st);
// n complex Gaussian spinor fields (internal layout) from the counter-based
// generator Philox4x32-10 keyed by seed, element by canonical index
template <typename T>
void launch_gaussian_fields(cx<T>* out, const Geom& g, int n, uint64_t seed, hipStream_t st);

// dslash: out[r] = piece of D applied to in[r] (chi_in >= 0 keeps only that
// chirality of the input; mu selects the direction of the cross variants).
// The cross variants write only the block layer they reach (lc[mu] = bs - 1
// forward, 0 backward); out keeps its values on every other site.
template <typename Tin, typename Tout, typename S, typename Tc>
void launch_dslash(cx<Tout>* out, const cx<Tin>* in, const GaugeView<S>& gv, const Geom& g, int nrhs, int mode,
                   int mu, int chi_in, size_t in_rstride, size_t out_rstride, hipStream_t st);

// loads the code object of the dslash kernels (see k_dslash.hip)
void preload_dslash_code();

// SAP: one colour phase of multiplicative Schwarz with n_mr MR steps per
// block, in place on x, for nrhs fields.
template <typename T, typename S>
void launch_sap_phase(cx<T>* x, const cx<T>* y, const GaugeView<S>& gv, const Geom& g, int colour, int n_mr, int nrhs,
                      hipStream_t st);

// restriction / prolongation; coarse output addressed as
// out[r * ostr_r + cint(b) * ostr_b + h * ntv + a].  face_mu >= 0: only the
// last layer of every block in direction face_mu (lc[face_mu] =
// bs[face_mu] - 1) is summed, whatever y holds elsewhere.
template <typename T, typename S>
void launch_restrict(cx<T>* out, size_t ostr_r, size_t ostr_b, const cx<T>* y, size_t ystr, const BasisView<S>& bv,
                     const Geom& g, int nrhs, hipStream_t st, int face_mu = -1);
template <typename T, typename S>
void launch_prolong(cx<T>* x, size_t xstr, const cx<T>* xc, size_t cstr, const BasisView<S>& bv, const Geom& g,
                    int nrhs, hipStream_t st);

// coarse stencil: for internal output sites [out_first, out_first + nout):
// out = add + cs * D_self xs + cn * sum_{slot>0} D_slot xn(nbr)
// vectors are addressed as ptr[r * str + (ci - first) * nc + k].
// gate (device int, optional): the kernel does nothing when *gate == 0
template <typename T, typename S>
void launch_coarse_stencil(cx<T>* out, size_t ostr, int out_first, int nout, const cx<T>* add, size_t astr,
                           const cx<T>* xs, size_t xsstr, int xs_first, T cs, const cx<T>* xn, size_t xnstr,
                           int xn_first, T cn, const CoarseView<S>& cv, const Geom& g, int nrhs, hipStream_t st,
                           const int* gate = nullptr);
// out[k] = M[k] x[k] for dense nc x nc column-major blocks M (k < nsites)
template <typename T>
void launch_block_matvec(cx<T>* out, size_t ostr, const cx<T>* M, const cx<T>* x, size_t xstr, int nsites, int nc,
                         int nrhs, hipStream_t st, const int* gate = nullptr);

// setup kernels
// tws: workspace of 2 nblocks * QR_TWS_PER_AGG complex doubles (per aggregate the
// Gram matrix, then T^{-1})
constexpr int QR_TWS_PER_AGG = 32 * 32;
// Orthonormalises the test vectors X (precision Tin) on every aggregate into
// the FP64 basis W (CholQR2; status set to 1 for a rank-deficient aggregate)
template <typename Tin>
void launch_aggregate_qr(cx<double>* W, const cx<Tin>* X, const Geom& g, int* status, cx<double>* tws,
                         hipStream_t st);
// Stores the FP64 basis W in precision S (FP16 with a per-(vector, site)
// scale in Wsc); for FP16, Wt (if given) receives the dequantised FP32
// values scale * half, the same numbers launch_dequantize_basis produces
template <typename S>
void launch_quantize_basis(stc_t<S>* Wq, float* Wsc, const cx<double>* W, const Geom& g, hipStream_t st,
                           cx<float>* Wt = nullptr);
template <typename T, typename S>
void launch_dequantize_basis(cx<T>* out, const BasisView<S>& bv, const Geom& g, hipStream_t st);
template <typename T>
void launch_dagger_fill(cx<T>* Dc, const int* nbr, const Geom& g, hipStream_t st);
// D_c in the exported layout -> internal accumulation layout
template <typename T>
void launch_coarse_import(cx<T>* D, const cx<double>* in, const Geom& g, hipStream_t st);
template <typename T, typename S>
void launch_quantize_coarse(stc_t<S>* Dq, float* Dsc, const cx<T>* Dc, const Geom& g, hipStream_t st);
template <typename T, typename S>
void launch_invert_even_blocks(cx<T>* Dinv, const CoarseView<S>& cv, const Geom& g, int* status, hipStream_t st);
template <typename T, typename S>
void launch_export_coarse(cx<double>* out, const CoarseView<S>& cv, const Geom& g, hipStream_t st);
template <typename T>
void launch_coarse_to_internal(cx<T>* out, const cx<double>* canon, const Geom& g, int nrhs, hipStream_t st);
template <typename T>
void launch_coarse_to_canonical(cx<double>* canon, const cx<T>* in, const Geom& g, int nrhs, hipStream_t st);

// ---------------------------------------------- learned test-vector network
// (k_learn.hip) fields FP32 internal [channel][12][V]; layer weights
// [C_out][C_in][NET_NFEAT] complex
constexpr int NET_NFEAT = 18;
constexpr int NET_WGRAD_SPT = 16;  // sites per thread of the weight-gradient kernel
// out = layer(in); gate_in: in holds pre-gate activations; gate_bwd_pre != NULL:
// the transposed layer's result passed back through the gate of the
// channels whose pre-gate activations are gate_bwd_pre
void launch_net_layer(cx<float>* out, const cx<float>* in, const cx<float>* W, int cin, int cout, bool gate_in,
                      const cx<float>* gate_bwd_pre, const GaugeView<float>& gv, const Geom& g, hipStream_t st);
// weights of the transposed layer (C_in x C_out) from W (C_out x C_in)
void launch_net_transpose(cx<float>* Wb, const cx<float>* W, int cin, int cout, hipStream_t st);
// chunks of the weight-gradient reduction; part needs chunks * cin * cout * 18 entries
int net_wgrad_chunks(const Geom& g);
void launch_net_wgrad(cx<float>* grad, cx<double>* part, const cx<float>* in, bool gate_in, const cx<float>* gam,
                      int cin, int cout, const GaugeView<float>& gv, const Geom& g, hipStream_t st);
// span loss (device *loss), per-aggregate terms loss_agg[2 nblocks] and its
// gradient gam with respect to X; *status = 1 if an aggregate's X^H X is
// not positive definite
void launch_net_span_loss(cx<float>* gam, double* loss_agg, double* loss, const cx<float>* X, const cx<float>* T,
                          const Geom& g, int ntv, int* status, hipStream_t st);
void launch_adam(float* w, float* m, float* v, const float* grad, size_t n, float lr, int64_t step, hipStream_t st);

// BLAS on block vectors x[r * rstride + i], i < n, r < nrhs.
// partial dots: part[(r * nvec + j) * nchunk + c]; final h[r * ldh + j].
// The multi-dot launchers take the capacity of part in entries and return
// false, launching nothing, if the call needs more (mdot_part_entries).
template <typename T>
bool launch_mdot(cx<double>* h, int ldh, cx<double>* part, size_t part_cap, const cx<T>* Vb, size_t vstride_j,
                 size_t vstride_r, int nvec, const cx<T>* w, size_t wstride_r, size_t n, int nrhs, const int* active,
                 hipStream_t st);
// w[r] += sign * sum_j h[r * ldh + j] * V_j[r], then w[r] *= post[r] if post;
// w32 (same strides) receives an FP32 copy of the result if given
template <typename Tw, typename Tv>
void launch_maxpy(cx<Tw>* w, size_t wstride_r, const cx<Tv>* Vb, size_t vstride_j, size_t vstride_r, int nvec,
                  const cx<double>* h, int ldh, double sign, size_t n, int nrhs, const int* active, hipStream_t st,
                  const double* post = nullptr, cx<float>* w32 = nullptr);
// Fused second Gram-Schmidt pass over FP64 vectors: w <- w - V h1, then
// h2[r][j] = V_j^H w (j < nvec) and h2[r][nvec] = |w|^2, nvec <= GS_FUSED_MAXV
constexpr int GS_FUSED_MAXV = 24;
bool launch_gs_fused(cx<double>* h2, int ldh, cx<double>* part, size_t part_cap, const cx<double>* Vb,
                     size_t vstride_j, size_t vstride_r, int nvec, cx<double>* w, size_t wstride_r,
                     const cx<double>* h1, size_t n, int nrhs, const int* active, hipStream_t st);
// The same pass with the previous step's second subtraction folded in: slot
// k of Vb holds the pending vector u, replaced by v_k = sigma (u - sum_{j<k}
// c_j V_j) if correct; then w <- w - sum_{j<=k} h_j V_j, w32 = FP32(wsc[r] w)
// if given, h2[r][j] = V_j^H w (j <= k) and h2[r][k + 1] = |w|^2; k + 1 <= GS_FUSED_MAXV
bool launch_gs_defer(cx<double>* h2, int ldh, cx<double>* part, size_t part_cap, cx<double>* Vb, size_t vsj,
                     size_t vsr, int k, bool correct, const cx<double>* c, const double* sigma, cx<double>* w,
                     size_t wsr, const cx<double>* h, size_t n, int nrhs, const int* active, cx<float>* w32,
                     const double* wsc, hipStream_t st);
// With h[r][k + 1] = |w|^2: if correct, c[r][j] = h2[r][j] (j < k) and h[r][k] =
// sigma[r] (h[r][k] - sum_{j<k} conj(c_j) h[r][j]); then wsc[r] = 1 / |w - sum_{j<=k}
// h_j V_j| estimated from |w|^2 - sum |h_j|^2 (nrhs <= 64)
void launch_gs_defer_coef(cx<double>* h, cx<double>* c, const cx<double>* h2, int ldh, const double* sigma, int k,
                          bool correct, double* wsc, int nrhs, const int* active, hipStream_t st);
// n2[r] = h2[r][nvec] - sum_{j<nvec} |h2[r][j]|^2, inv[r] = 1/sqrt(n2[r]) (0 if not positive)
void launch_gs_norm(cx<double>* n2, double* inv, const cx<double>* h2, int ldh, int nvec, int nrhs,
                    const int* active, hipStream_t st);
// y[r] = s[r] * x[r] (s real double, per rhs) ; y and x may alias; y32 (same
// strides as y) receives an FP32 copy of y if given
template <typename Ty, typename Tx>
void launch_scale(cx<Ty>* y, size_t ystr, const cx<Tx>* x, size_t xstr, const double* s, size_t n, int nrhs,
                  const int* active, hipStream_t st, cx<float>* y32 = nullptr);
// abstol[r] = tol * |n2[r]|^(1/2) (tol < 0 gives -1); s[r] = |n2[r]|^(-1/2)
// with *status set to 1 if a norm is zero or not finite (nrhs <= 64)
void launch_set_abstol(double* abstol, const cx<double>* n2, double tol, int nrhs, hipStream_t st);
void launch_inv_norm(double* s, const cx<double>* n2, int nrhs, int* status, hipStream_t st);
// y[r] = a[r] - b[r]
template <typename T>
void launch_sub(cx<T>* y, size_t ystr, const cx<T>* a, size_t astr, const cx<T>* b, size_t bstr, size_t n, int nrhs,
                hipStream_t st);
template <typename Ty, typename Tx>
void launch_copy(cx<Ty>* y, size_t ystr, const cx<Tx>* x, size_t xstr, size_t n, int nrhs, hipStream_t st);

// Arnoldi / Givens state on the device (FP64).  Per rhs r: H[r][(m+1) * m]
// column-major (H[r][k * (m+1) + j]), cs/sn[r][m], g[r][m+1].
struct ArnoldiState {
  cx<double>* H;
  cx<double>* cs;
  cx<double>* sn;
  cx<double>* g;
  cx<double>* y;       // [r][m] least-squares solution
  double* est;         // [r] current residual estimate |g_{k+1}|
  double* inv_h;       // [r] 1 / h_{k+1,k} (0 if breakdown or inactive)
  double* abstol;      // [r] stop threshold (< 0: never)
  int* active;         // [r]
  int* any;            // [1] 1 if some rhs is active (written with active)
  int* kdone;          // [r] iterations done in this cycle
  int m;
};
// start a cycle: g = (beta, 0, ...), active = beta > abstol (or beta > 0
// when abstol < 0), kdone = 0, inv_h = 1 / beta; beta from norm2[r] = |.|^2
void launch_arnoldi_start(ArnoldiState s, const cx<double>* norm2, int ldn, int nrhs, hipStream_t st);
// column k: H[0..k, k] = h1 + h2, H[k+1, k] = sqrt(norm2), rotations, g,
// est, convergence -> active, kdone
void launch_arnoldi_column(ArnoldiState s, int k, const cx<double>* h1, const cx<double>* h2, int ldh,
                           const cx<double>* norm2, int ldn, int nrhs, hipStream_t st);
// y = H(1:kd, 1:kd)^{-1} g(1:kd) per rhs (upper triangular)
void launch_arnoldi_solve(ArnoldiState s, int nrhs, hipStream_t st);
// the whole coarse solve (Alg. 2) of each rhs in one workgroup, for coarse
// lattices small enough that launch latency bounds the multi-kernel solve
// (restart m <= COARSE_SMALL_MAX_RESTART; its_stat[0] += iterations,
// its_stat[1] = max).
// One workgroup reads the coarse operator at the L2 bandwidth of one CU, so
// the path is taken while one stencil pass over the lattice (9 nc x nc
// blocks per site) stays within COARSE_SMALL_MAX_BYTES.
constexpr int COARSE_SMALL_MAX_SITES = 64;
constexpr size_t COARSE_SMALL_MAX_BYTES = (size_t)3 << 19;  // 1.5 MiB
constexpr int COARSE_SMALL_MAX_RESTART = 32;
constexpr int COARSE_SMALL_MAX_VECTOR = 1536;  // sites x nc: the LDS copy of a coarse vector
template <typename T, typename S>
void launch_coarse_gmres_small(cx<T>* xc, const cx<T>* yc, size_t cstr, const CoarseView<S>& cv, const cx<T>* Dinv,
                               const Geom& g, cx<T>* te, cx<T>* ue, cx<T>* bo, cx<T>* cw, cx<T>* V, size_t vsj,
                               int m, int maxit, double tol, int* its_stat, int nrhs, hipStream_t st);

}  // namespace ddamg
