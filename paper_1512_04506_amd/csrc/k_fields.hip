// Field preparation kernels: gauge import, clover term, storage
// quantisation and canonical <-> internal spinor layouts.
#include "ddamg_internal.h"

namespace ddamg {

namespace {

constexpr int TPB = 256;

inline unsigned nblk(size_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

__global__ void gauge_import_kernel(cx<double>* U, const cx<double>* canon, Geom g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int c[4];
  site_coords(g, s, c);
  const size_t lex = lex_site(g, c);
  const size_t V = g.V;
  for (int mu = 0; mu < 4; ++mu)
    for (int e = 0; e < 9; ++e) U[((size_t)mu * 9 + e) * V + s] = canon[(lex * 4 + mu) * 9 + e];
}

struct M3 {
  cx<double> a[3][3];
};

__device__ inline M3 load_link(const cx<double>* U, int V, int mu, int s) {
  M3 m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = U[((size_t)mu * 9 + 3 * i + j) * V + s];
  return m;
}
__device__ inline M3 mul(const M3& x, const M3& y) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cx<double> acc = mk(0.0, 0.0);
      for (int k = 0; k < 3; ++k) acc = acc + x.a[i][k] * y.a[k][j];
      r.a[i][j] = acc;
    }
  return r;
}
__device__ inline M3 dag(const M3& x) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = conj(x.a[j][i]);
  return r;
}
__device__ inline int nb(const Geom& g, const int c[4], int mu, int d) {
  int e[4] = {c[0], c[1], c[2], c[3]};
  e[mu] = (e[mu] + d + g.L[mu]) % g.L[mu];
  return site_index(g, e);
}
__device__ inline int nb2(const Geom& g, const int c[4], int mu, int dmu, int nu, int dnu) {
  int e[4] = {c[0], c[1], c[2], c[3]};
  e[mu] = (e[mu] + dmu + g.L[mu]) % g.L[mu];
  e[nu] = (e[nu] + dnu + g.L[nu]) % g.L[nu];
  return site_index(g, e);
}

// F_{mu nu}(x) = (Q - Q^dag) / 8 with Q the sum of the four plaquette leaves
// at x in the (mu, nu) plane, all traversed in the same sense.
__device__ M3 field_strength(const cx<double>* U, const Geom& g, const int c[4], int s, int mu, int nu) {
  const int V = g.V;
  int xpm = nb(g, c, mu, +1), xpn = nb(g, c, nu, +1);
  int xmm = nb(g, c, mu, -1), xmn = nb(g, c, nu, -1);
  int xmm_pn = nb2(g, c, mu, -1, nu, +1);
  int xmm_mn = nb2(g, c, mu, -1, nu, -1);
  int xpm_mn = nb2(g, c, mu, +1, nu, -1);
  M3 Umu = load_link(U, V, mu, s), Unu = load_link(U, V, nu, s);
  // x -> x+mu -> x+mu+nu -> x+nu -> x
  M3 q1 = mul(mul(Umu, load_link(U, V, nu, xpm)), mul(dag(load_link(U, V, mu, xpn)), dag(Unu)));
  // x -> x+nu -> x-mu+nu -> x-mu -> x
  M3 q2 = mul(mul(Unu, dag(load_link(U, V, mu, xmm_pn))), mul(dag(load_link(U, V, nu, xmm)), load_link(U, V, mu, xmm)));
  // x -> x-mu -> x-mu-nu -> x-nu -> x
  M3 q3 = mul(mul(dag(load_link(U, V, mu, xmm)), dag(load_link(U, V, nu, xmm_mn))),
              mul(load_link(U, V, mu, xmm_mn), load_link(U, V, nu, xmn)));
  // x -> x-nu -> x+mu-nu -> x+mu -> x
  M3 q4 = mul(mul(dag(load_link(U, V, nu, xmn)), load_link(U, V, mu, xmn)), mul(load_link(U, V, nu, xpm_mn), dag(Umu)));
  M3 F;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cx<double> q = q1.a[i][j] + q2.a[i][j] + q3.a[i][j] + q4.a[i][j];
      cx<double> qd = conj(q1.a[j][i] + q2.a[j][i] + q3.a[j][i] + q4.a[j][i]);
      F.a[i][j] = 0.125 * (q - qd);
    }
  return F;
}

// Packing of one 6x6 Hermitian chirality block into 36 reals.
__device__ inline int upper_index(int i, int j) {  // i < j
  // number of pairs before row i: sum_{k<i} (5 - k)
  return i * 5 - (i * (i - 1)) / 2 + (j - i - 1);
}

// In the chiral basis sigma_{mu nu} is block diagonal.  With Pauli matrices
// s_l and planes written 0-based (x, y, z, t):
//   left  block: sum_{mu<nu} sigma F = s1 B1 + s2 B2 + s3 B3 with
//       B1 = -(F12 + F03), B2 = F02 - F13, B3 = -(F01 + F23)
//   right block: B1 = F03 - F12, B2 = F02 + F13, B3 = F23 - F01
// (sigma_{k4} = diag(-s_k, s_k), sigma_{jk} = -eps_{jkl} diag(s_l, s_l)),
// and A^h = (4 + m0) + c_sw (i/2) sum_l s_l (x) B_l.
__global__ void clover_kernel(cx<double>* A, const cx<double>* U, Geom g, double m0, double csw) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int c[4];
  site_coords(g, s, c);
  M3 F01 = field_strength(U, g, c, s, 0, 1);
  M3 F02 = field_strength(U, g, c, s, 0, 2);
  M3 F12 = field_strength(U, g, c, s, 1, 2);
  M3 F03 = field_strength(U, g, c, s, 0, 3);
  M3 F13 = field_strength(U, g, c, s, 1, 3);
  M3 F23 = field_strength(U, g, c, s, 2, 3);
  const size_t V = g.V;
  for (int h = 0; h < 2; ++h) {
    M3 B1, B2, B3;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        if (h == 0) {
          B1.a[i][j] = neg(F12.a[i][j] + F03.a[i][j]);
          B2.a[i][j] = F02.a[i][j] - F13.a[i][j];
          B3.a[i][j] = neg(F01.a[i][j] + F23.a[i][j]);
        } else {
          B1.a[i][j] = F03.a[i][j] - F12.a[i][j];
          B2.a[i][j] = F02.a[i][j] + F13.a[i][j];
          B3.a[i][j] = F23.a[i][j] - F01.a[i][j];
        }
      }
    // spin blocks of M = sum s_l B_l: [[B3, B1 - i B2], [B1 + i B2, -B3]]
    cx<double> full[6][6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cx<double> m00 = B3.a[i][j];
        cx<double> m01 = B1.a[i][j] + times_mi(B2.a[i][j]);
        cx<double> m10 = B1.a[i][j] + times_i(B2.a[i][j]);
        cx<double> m11 = neg(B3.a[i][j]);
        double f = 0.5 * csw;
        full[i][j] = f * times_i(m00);
        full[i][3 + j] = f * times_i(m01);
        full[3 + i][j] = f * times_i(m10);
        full[3 + i][3 + j] = f * times_i(m11);
      }
    cx<double>* Ah = A + (size_t)h * CLOVER_PAIRS * V;
    for (int k = 0; k < 3; ++k) Ah[(size_t)k * V + s] = mk(4.0 + m0 + full[2 * k][2 * k].r, 4.0 + m0 + full[2 * k + 1][2 * k + 1].r);
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) Ah[(size_t)(3 + upper_index(i, j)) * V + s] = full[i][j];
  }
}

template <typename S>
__global__ void quantize_gauge_kernel(stc_t<S>* Uq, float* Usc, stc_t<S>* Aq, float* Asc, const cx<double>* U,
                                      const cx<double>* A, int V) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  if constexpr (is_half<S>()) {
    double mu = 0.0, ma = 0.0;
    for (int e = 0; e < 36; ++e) {
      cx<double> u = U[(size_t)e * V + s];
      mu = fmax(mu, fmax(fabs(u.r), fabs(u.i)));
    }
    for (int e = 0; e < 2 * CLOVER_PAIRS; ++e) {
      cx<double> a = A[(size_t)e * V + s];
      ma = fmax(ma, fmax(fabs(a.r), fabs(a.i)));
    }
    float fu = (float)mu, fa = (float)ma;
    double iu = fu > 0.f ? 1.0 / (double)fu : 0.0, ia = fa > 0.f ? 1.0 / (double)fa : 0.0;
    Usc[s] = fu;
    Asc[s] = fa;
    for (int e = 0; e < 36; ++e) {
      cx<double> u = U[(size_t)e * V + s];
      Uq[(size_t)e * V + s] = __floats2half2_rn((float)(u.r * iu), (float)(u.i * iu));
    }
    for (int e = 0; e < 2 * CLOVER_PAIRS; ++e) {
      cx<double> a = A[(size_t)e * V + s];
      Aq[(size_t)e * V + s] = __floats2half2_rn((float)(a.r * ia), (float)(a.i * ia));
    }
  } else {
    for (int e = 0; e < 36; ++e) stc_store(Uq, (size_t)e * V + s, U[(size_t)e * V + s]);
    for (int e = 0; e < 2 * CLOVER_PAIRS; ++e) stc_store(Aq, (size_t)e * V + s, A[(size_t)e * V + s]);
  }
}

// internal element (r, comp, S) <-> canonical element (r, lex(S), comp)
// One thread per (rhs, internal site): the 12 components of a canonical site
// are one contiguous 192-byte record, the internal components are 12
// site-contiguous planes, so both sides are read/written in full lines.
template <typename T>
__global__ void spinor_to_internal_kernel(cx<T>* out, const cx<double>* canon, Geom g, int nrhs, int* nonzero) {
  const size_t V = g.V;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = idx < (size_t)nrhs * V;
  const size_t ic = valid ? idx : 0;
  const int s = (int)(ic % V);
  const size_t r = ic / V;
  bool nz = false;
  if (valid) {
    int c[4];
    site_coords(g, s, c);
    const cx<double>* src = canon + (r * V + lex_site(g, c)) * 12;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = src[k];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      out[(r * 12 + k) * V + s] = cvt<T>(v[k]);
      nz = nz || v[k].r != 0.0 || v[k].i != 0.0;
    }
  }
  if (nonzero) {
    // nonzero[r] = 1 if the field of rhs r has a nonzero entry: one atomic
    // per wave and rhs present in it (the loop is uniform over the wave)
    const int lane = threadIdx.x & 63;
    unsigned long long todo = __ballot(valid && nz);
    while (todo) {
      const int l0 = __ffsll((unsigned long long)todo) - 1;
      const size_t rl = (size_t)__shfl((long long)r, l0, 64);
      const unsigned long long mine = __ballot(valid && nz && r == rl);
      if (lane == l0) atomicOr(&nonzero[rl], 1);
      todo &= ~mine;
    }
  }
}

template <typename T>
__global__ void spinor_to_canonical_kernel(cx<double>* canon, const cx<T>* in, Geom g, int nrhs) {
  const size_t V = g.V;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrhs * V) return;
  const int s = (int)(idx % V);
  const size_t r = idx / V;
  int c[4];
  site_coords(g, s, c);
  cx<double> v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = cvt<double>(in[(r * 12 + k) * V + s]);
  cx<double>* dst = canon + (r * V + lex_site(g, c)) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = v[k];
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of the
// two 32 x 32 -> 64-bit products with multipliers 0xD2511F53 and
// 0xCD9E8D57, the key advanced by the Weyl constants 0x9E3779B9 and
// 0xBB67AE85 between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

// Complex Gaussian draw for canonical element i (re, im ~ N(0, 1)): the
// counter (i mod 2^32, i >> 32, 0, 0) under the key (seed mod 2^32,
// seed >> 32) gives two 53-bit uniforms u1, u2 in [0, 1), and Box-Muller
// gives sqrt(-2 log(1 - u1)) (cos 2 pi u2, sin 2 pi u2).
__device__ inline cx<double> philox_gaussian(uint64_t i, uint64_t seed) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = (double)(c[0] >> 5) * 0x1p-27 + (double)(c[1] >> 6) * 0x1p-53;
  const double u2 = (double)(c[2] >> 5) * 0x1p-27 + (double)(c[3] >> 6) * 0x1p-53;
  const double rho = sqrt(-2.0 * log(1.0 - u1));
  double sn, cs;
  sincos(2.0 * M_PI * u2, &sn, &cs);
  return mk(rho * cs, rho * sn);
}

// n seeded Gaussian spinor fields in the internal layout; the draw of an
// element depends on its canonical index only, so the same seed gives the
// same fields whatever the internal order
template <typename T>
__global__ void gaussian_fields_kernel(cx<T>* out, Geom g, int n, uint64_t seed) {
  const size_t V = g.V;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * V) return;
  const int s = (int)(idx % V);
  const size_t r = idx / V;
  int c[4];
  site_coords(g, s, c);
  const uint64_t base = ((uint64_t)r * V + (uint64_t)lex_site(g, c)) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) out[(r * 12 + k) * V + s] = cvt<T>(philox_gaussian(base + k, seed));
}

__global__ void clover_export_kernel(cx<double>* out, const cx<double>* A, Geom g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const size_t V = g.V;
  int c[4];
  site_coords(g, s, c);
  const size_t lex = lex_site(g, c);
  for (int h = 0; h < 2; ++h) {
    const cx<double>* Ah = A + (size_t)h * CLOVER_PAIRS * V;
    cx<double>* o = out + (lex * 2 + h) * 36;
    for (int k = 0; k < 3; ++k) {
      const cx<double> d = Ah[(size_t)k * V + s];
      o[(2 * k) * 6 + 2 * k] = mk(d.r, 0.0);
      o[(2 * k + 1) * 6 + 2 * k + 1] = mk(d.i, 0.0);
    }
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        const cx<double> v = Ah[(size_t)(3 + upper_index(i, j)) * V + s];
        o[i * 6 + j] = v;
        o[j * 6 + i] = conj(v);
      }
  }
}

}  // namespace

void launch_gauge_import(cx<double>* U, const cx<double>* canon, const Geom& g, hipStream_t st) {
  gauge_import_kernel<<<nblk(g.V), TPB, 0, st>>>(U, canon, g);
}

void launch_clover_build(cx<double>* A, const cx<double>* U, const Geom& g, double m0, double csw, hipStream_t st) {
  clover_kernel<<<nblk(g.V, 128), 128, 0, st>>>(A, U, g, m0, csw);
}

template <typename S>
void launch_quantize_gauge(stc_t<S>* Uq, float* Usc, stc_t<S>* Aq, float* Asc, const cx<double>* U,
                           const cx<double>* A, const Geom& g, hipStream_t st) {
  quantize_gauge_kernel<S><<<nblk(g.V), TPB, 0, st>>>(Uq, Usc, Aq, Asc, U, A, g.V);
}
template void launch_quantize_gauge<double>(stc_t<double>*, float*, stc_t<double>*, float*, const cx<double>*,
                                            const cx<double>*, const Geom&, hipStream_t);
template void launch_quantize_gauge<float>(stc_t<float>*, float*, stc_t<float>*, float*, const cx<double>*,
                                           const cx<double>*, const Geom&, hipStream_t);
template void launch_quantize_gauge<__half>(stc_t<__half>*, float*, stc_t<__half>*, float*, const cx<double>*,
                                            const cx<double>*, const Geom&, hipStream_t);

template <typename T>
void launch_spinor_to_internal(cx<T>* out, const cx<double>* canon, const Geom& g, int nrhs, hipStream_t st,
                               int* nonzero) {
  size_t n = (size_t)nrhs * 12 * g.V;
  if (n) spinor_to_internal_kernel<T><<<nblk(n / 12), TPB, 0, st>>>(out, canon, g, nrhs, nonzero);
}
template <typename T>
void launch_spinor_to_canonical(cx<double>* canon, const cx<T>* in, const Geom& g, int nrhs, hipStream_t st) {
  size_t n = (size_t)nrhs * 12 * g.V;
  if (n) spinor_to_canonical_kernel<T><<<nblk(n / 12), TPB, 0, st>>>(canon, in, g, nrhs);
}
template void launch_spinor_to_internal<double>(cx<double>*, const cx<double>*, const Geom&, int, hipStream_t, int*);
template void launch_spinor_to_internal<float>(cx<float>*, const cx<double>*, const Geom&, int, hipStream_t, int*);
template void launch_spinor_to_canonical<double>(cx<double>*, const cx<double>*, const Geom&, int, hipStream_t);
template void launch_spinor_to_canonical<float>(cx<double>*, const cx<float>*, const Geom&, int, hipStream_t);

template <typename T>
void launch_gaussian_fields(cx<T>* out, const Geom& g, int n, uint64_t seed, hipStream_t st) {
  if (n > 0) gaussian_fields_kernel<T><<<nblk((size_t)n * g.V), TPB, 0, st>>>(out, g, n, seed);
}
template void launch_gaussian_fields<double>(cx<double>*, const Geom&, int, uint64_t, hipStream_t);
template void launch_gaussian_fields<float>(cx<float>*, const Geom&, int, uint64_t, hipStream_t);

void launch_clover_export(cx<double>* out, const cx<double>* A, const Geom& g, hipStream_t st) {
  clover_export_kernel<<<nblk(g.V), TPB, 0, st>>>(out, A, g);
}

}  // namespace ddamg
