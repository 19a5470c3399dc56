/*
 * ddamg.h -- C ABI of the MI355X (gfx950) two-level DD-alpha-AMG library.
 *
 * Method: Heybrock, Rottmann, Georg, Wettig, "Adaptive algebraic multigrid
 * on SIMD architectures", arXiv:1512.04506.  The library solves D u = f for
 * the Wilson-clover operator D (Sec. 1) with flexible GMRES, right-
 * preconditioned by the two-level V-cycle of Alg. 1: coarse-grid correction
 * (Alg. 2: restriction R of Eq. R, even/odd coarse GMRES on D_c,
 * prolongation P = R^dagger) followed by the domain-decomposition smoother of
 * Alg. 3 (red/black multiplicative Schwarz with block-local MR).  R and D_c
 * are built by the adaptive setup of Alg. 4 and Alg. 5.
 *
 * Conventions (fixed here because the paper leaves them open):
 *   lattice L = (Lx, Ly, Lz, Lt), periodic in space, antiperiodic in time;
 *   site index s = x + Lx (y + Ly (z + Lz t));
 *   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *                                          + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)],
 *   A(x) = (4 + m0) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x) (clover
 *   leaves), chiral gamma basis with g5 = diag(-1, -1, +1, +1): the
 *   left-handed aggregate of a block holds spins {0, 1}, the right-handed one
 *   spins {2, 3}.
 *
 * Canonical layouts at this boundary (all complex128 = interleaved re, im
 * doubles, C order, DEVICE pointers on the context's device):
 *   gauge field   [V][4 mu][3][3]                 (mu = x, y, z, t)
 *   spinor fields [nrhs][V][4 spin][3 colour]
 *   coarse fields [nrhs][Nblock][2 chirality][ntv] with block index
 *                 bx + NBx (by + NBy (bz + NBz bt)), NB = L / block
 *   coarse op     [Nblock][9 slot][2 ntv row][2 ntv col]; slot 0 = self,
 *                 1 + 2 mu = forward neighbour, 2 + 2 mu = backward neighbour
 *   test vectors  [ntv][V][4][3]
 *   clover        [V][2 chirality][6][6]  (row/col = 3 spin_in_chirality + colour)
 *
 * Ownership: the caller owns every pointer it passes and keeps it valid for
 * the duration of the call; the library never frees caller memory.  The
 * library owns the context and its device workspace (hipMalloc at create).
 *
 * Streams: every call enqueues work on the context's stream.  dirac_apply,
 * coarse_apply, mg_apply, mg_restrict, mg_prolong and the *_internal calls
 * are asynchronous with respect to the host; mg_setup and solve synchronise
 * (they test convergence) and return when done.  A context is not
 * thread-safe; use one context per stream.
 *
 * Errors: 0 = OK, 1 = not converged (best iterate returned, stats filled);
 * negative codes below.  Argument validation happens before any HIP call.
 * No exception or abort crosses this boundary; ddamg_last_error() gives text.
 */
#ifndef DDAMG_H
#define DDAMG_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDAMG_ABI_VERSION 2

/* precision of the preconditioner (smoother, R/P, coarse solve) */
#define DDAMG_FP64 0     /* everything FP64 */
#define DDAMG_FP32 1     /* FP32 storage and arithmetic, FP64 outer FGMRES */
#define DDAMG_MIXED16 2  /* FP16 storage of links, clover, test vectors and D_c
                            with per-site / per-block FP32 scales, FP32
                            arithmetic, FP64 outer FGMRES and setup Gram-Schmidt */

#define DDAMG_OK 0
#define DDAMG_NOT_CONVERGED 1
#define DDAMG_EARG (-1)      /* invalid argument */
#define DDAMG_ESTATE (-2)    /* call not valid in this state (e.g. before setup) */
#define DDAMG_EHIP (-3)      /* HIP runtime error */
#define DDAMG_ENOMEM (-4)    /* device allocation failed */
#define DDAMG_ENUMERIC (-5)  /* NaN/Inf, singular coarse block, rank-deficient aggregate */

typedef struct ddamg_ctx ddamg_ctx;

typedef struct {
  int32_t L[4];            /* lattice extents x, y, z, t */
  int32_t block[4];        /* SAP block = aggregate extents; must divide L, and
                              every L[mu]/block[mu] must be even (red/black SAP
                              and coarse even/odd need it) */
  double m0;               /* bare mass: diagonal 4 + m0 */
  double csw;              /* clover coefficient */
  int32_t ntv;             /* test vectors per aggregate (Sec. 2; 1 <= ntv <= 32,
                              6 * block volume >= ntv) */
  int32_t n_setup;         /* iterative setup passes after the initial 3 (Alg. 4) */
  int32_t nu;              /* SAP cycles per smoother application (Alg. 3) */
  int32_t n_mr;            /* MR steps per block solve */
  double coarse_tol;       /* coarse solve stops at ||r_c|| <= tol ||y_c|| (Alg. 2) */
  int32_t coarse_restart;  /* coarse GMRES restart length (<= 64) */
  int32_t coarse_maxit;    /* coarse iteration cap per solve */
  int32_t coarse_fixed_its;/* > 0: run exactly this many coarse iterations
                              (deterministic mode, no tolerance test) */
  int32_t outer_restart;   /* outer FGMRES restart length (<= 64) */
  int32_t outer_maxit;     /* outer iteration cap */
  int32_t prec;            /* DDAMG_FP64, DDAMG_FP32 or DDAMG_MIXED16 */
  int32_t max_rhs;         /* largest nrhs of any later call (>= 1, <= 64) */
  int32_t init_passes;     /* mg_setup's initial smoother passes on the start
                              vectors, N_smoother = 1, 2, ..., init_passes from a
                              zero guess (Alg. 4: 3); 0 uses the start vectors
                              as they are (e.g. a ddamg_net_propose output) */
  uint64_t seed;           /* key of the random starting test vectors that
                              mg_setup draws when it is given none */
} ddamg_params;

typedef struct {
  int32_t outer_iterations;     /* FGMRES iterations of the last solve */
  int32_t outer_restarts;       /* restart cycles of the last solve */
  int32_t coarse_solves;        /* coarse solves since the last reset */
  int32_t coarse_iterations_max;/* largest iteration count of one coarse solve */
  int64_t coarse_iterations;    /* total coarse iterations since the last reset */
  int32_t nrhs;                 /* right-hand sides of the last solve */
  int32_t converged;            /* 1 if every right-hand side converged */
  double relres[64];            /* final FP64 true relative residual per rhs */
  double setup_ms;              /* wall time of the last mg_setup */
  double solve_ms;              /* wall time of the last solve */
} ddamg_stats;

/* Fills *p with the defaults: block 4^4, m0 = 0, csw = 1, ntv = 24,
 * n_setup = 3, nu = 3, n_mr = 4, coarse_tol = 0.05, coarse_restart = 30,
 * coarse_maxit = 300, coarse_fixed_its = 0, outer_restart = 20,
 * outer_maxit = 2000, prec = DDAMG_MIXED16, max_rhs = 12, init_passes = 3,
 * seed = 0. */
void ddamg_default_params(ddamg_params* p);

/* Checks p without touching the GPU.  Returns 0 or DDAMG_EARG and, if msg is
 * not NULL, writes a NUL-terminated reason into msg[0..msg_len-1]. */
int ddamg_validate_params(const ddamg_params* p, char* msg, size_t msg_len);

/* Device allocator for the workspace of contexts created afterwards
 * (process-wide; alloc == NULL and free_fn == NULL restore hipMalloc /
 * hipFree).  alloc(bytes, user) returns device memory or NULL (the call
 * that needed it then fails with DDAMG_ENOMEM); every block is released
 * with the free_fn(ptr, user) that was installed when it was allocated,
 * after the device has finished all work queued before the release.
 * For callers that own device memory themselves, e.g. a framework's caching
 * allocator.  DDAMG_EARG if exactly one of alloc and free_fn is NULL. */
typedef void* (*ddamg_alloc_fn)(size_t bytes, void* user);
typedef void (*ddamg_free_fn)(void* ptr, void* user);
int ddamg_set_allocator(ddamg_alloc_fn alloc, ddamg_free_fn free_fn, void* user);

/* Creates a context on the current HIP device.  gauge: canonical links
 * (device, complex128), copied; the clover term A(x) is built from them
 * (Alg. 7 names its blocks C^{hh}(x)) and all storage precisions are
 * derived.  stream: hipStream_t the context enqueues on (NULL = default
 * stream).  *out receives the context, or NULL on error. */
int ddamg_create(const ddamg_params* p, const double* gauge, void* stream, ddamg_ctx** out);

int ddamg_destroy(ddamg_ctx* ctx);

/* Text of the last error on ctx (or of the last failed create if ctx is NULL). */
const char* ddamg_last_error(const ddamg_ctx* ctx);

/* Adaptive setup, Alg. 4 with Alg. 5: tv_init (device, canonical test
 * vectors [ntv][V][4][3]) are the random starting vectors; they are
 * smoothed with N_smoother = 1, 2, 3 from a zero guess, R and D_c are
 * built (aggregate Gram-Schmidt in FP64, D_c = R D P with backward couplings
 * from Eq. dagger), the vectors are normalised, then n_setup passes apply
 * the V-cycle to every test vector and rebuild R and D_c.  Synchronous.
 * tv_init == NULL: the starting vectors are drawn on the device from the
 * context's seed, complex element i of the canonical array (re, im ~ N(0,1))
 * by Philox4x32-10 (Salmon et al., SC 2011) with counter (i mod 2^32,
 * i >> 32, 0, 0) and key (seed mod 2^32, seed >> 32), whose output words
 * (x0, x1, x2, x3) give u1 = (x0 >> 5) 2^-27 + (x1 >> 6) 2^-53, u2 likewise
 * from (x2, x3), and Box-Muller sqrt(-2 log(1 - u1)) (cos, sin)(2 pi u2). */
int mg_setup(ddamg_ctx* ctx, const double* tv_init);

/* Replaces the aggregate basis by W (device, canonical [ntv][V][4][3],
 * orthonormal on every aggregate, e.g. as returned by ddamg_export_basis)
 * and rebuilds D_c = R D P from it (Alg. 5 without the Gram-Schmidt).
 * Synchronous. */
int ddamg_import_basis(ddamg_ctx* ctx, const double* W);

/* Exports the aggregate basis (the rows of R, i.e. the columns of P = R^dag,
 * as fields), dequantised to FP64, canonical [ntv][V][4][3]. */
int ddamg_export_basis(ddamg_ctx* ctx, double* W);

/* Exports the setup's current test vectors (FP64, canonical [ntv][V][4][3]). */
int ddamg_export_tv(ddamg_ctx* ctx, double* tv);

/* Takes tv (device, complex128 [ntv][V][4][3], e.g. from ddamg_export_tv of
 * a context with the same parameters) as the setup's test vectors and
 * builds R (the Gram-Schmidt of Alg. 5 on every aggregate) and D_c = R D P
 * from them, without smoothing: resumes a saved setup state.  Synchronous;
 * DDAMG_ENUMERIC for a rank-deficient aggregate. */
int ddamg_import_tv(ddamg_ctx* ctx, const double* tv);

/* Exports D_c (Eq. cgo), dequantised, as [Nblock][9][2ntv][2ntv] complex128. */
int ddamg_export_coarse(ddamg_ctx* ctx, double* Dc);

/* Replaces D_c by Dc (device, complex128, the layout ddamg_export_coarse
 * writes: block lexicographic, slots self, +x, -x, ..., +t, -t, each block
 * row-major) and prepares the coarse solve from it (storage precision of
 * the context, inverse of the even self blocks).  The basis is kept, so a
 * setup (mg_setup, ddamg_import_basis or ddamg_import_tv) must precede it
 * (DDAMG_ESTATE).  Synchronous; DDAMG_ENUMERIC for a singular even self
 * block. */
int ddamg_import_coarse(ddamg_ctx* ctx, const double* Dc);

/* Exports the clover term A(x) in FP64 as [V][2][6][6] complex128. */
int ddamg_export_clover(ddamg_ctx* ctx, double* A);

/* One V-cycle (Alg. 1) on nrhs canonical spinor fields: x = M^{-1} y.
 * Runs in the context's precision; x, y complex128 [nrhs][V][4][3],
 * x != y.  Requires setup. */
int mg_apply(ddamg_ctx* ctx, double* x, const double* y, int nrhs);

/* out = D in (Sec. 1) for nrhs canonical spinor fields with the links and
 * clover stored in precision prec (DDAMG_FP64 / FP32 / MIXED16); the result
 * is returned in FP64.  out != in. */
int dirac_apply(ddamg_ctx* ctx, double* out, const double* in, int nrhs, int prec);

/* out = D_c in on canonical coarse fields [nrhs][Nblock][2][ntv], using the
 * stored (possibly FP16) D_c with the context's arithmetic.  Requires setup. */
int coarse_apply(ddamg_ctx* ctx, double* out, const double* in, int nrhs);

/* y_c = R y (Eq. R) and x = P x_c (P = R^dag, Alg. 2) on canonical fields. */
int mg_restrict(ddamg_ctx* ctx, double* yc, const double* y, int nrhs);
int mg_prolong(ddamg_ctx* ctx, double* x, const double* xc, int nrhs);

/* Solves D u = f for nrhs right-hand sides with FGMRES(outer_restart),
 * right-preconditioned by the V-cycle (Sec. 1), to ||f - D u|| <= tol ||f||
 * per rhs, the residual recomputed in FP64.  u holds the initial guess on
 * entry (zero recommended) and the solution on return.  u, f canonical,
 * u != f.  st may be NULL.  Returns 0, DDAMG_NOT_CONVERGED or an error.
 * Synchronous. */
int solve(ddamg_ctx* ctx, double* u, const double* f, int nrhs, double tol, ddamg_stats* st);

/* Fills *st with the counters of the last calls; ddamg_reset_stats zeroes
 * the coarse-solve counters. */
int ddamg_get_stats(const ddamg_ctx* ctx, ddamg_stats* st);
int ddamg_reset_stats(ddamg_ctx* ctx);

/* ---- internal-layout fast path (benchmarks) --------------------------
 * Spinor fields in the library's internal layout: site-major
 * structure-of-arrays complex, element (rhs, comp, site) at
 * (rhs * 12 + comp) * V + site, comp = 3 spin + colour, complex128 for
 * DDAMG_FP64 and complex64 for DDAMG_FP32 / DDAMG_MIXED16.  Internal site
 * order (block-major): the site with coordinates x = block * bc + lc has
 * index ci * V_block + l, where l = lc_x + b_x (lc_y + b_y (lc_z + b_z lc_t))
 * is its place in the block (b = block extents), lexb the lexicographic
 * block index of bc (as for coarse fields above) and
 * ci = ((bc_x + bc_y + bc_z + bc_t) mod 2) * Nblock / 2 + lexb / 2 (integer
 * division): even blocks first.  No layout conversion is performed;
 * out != in; asynchronous. */
int dirac_apply_internal(ddamg_ctx* ctx, void* out, const void* in, int nrhs, int prec);

/* Coarse fields in the internal layout of the context's arithmetic
 * (complex128 for DDAMG_FP64, complex64 otherwise): [nrhs][Nblock][2 ntv]
 * with coarse sites in the internal order (even coarse sites first). */
int coarse_apply_internal(ddamg_ctx* ctx, void* out, const void* in, int nrhs);

/* ---- no-allocation variant -------------------------------------------
 * For callers that cannot allocate device memory during a call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * dirac_apply_noalloc computes what dirac_apply computes, with the same
 * kernels and the same result, but stages the internal-layout copies of in
 * and out in a fixed device array of DDAMG_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends (its address
 * is looked up once per device, at ddamg_create), instead of workspace that
 * dirac_apply allocates on first use and whenever nrhs grows.  It calls no
 * hipMalloc, hipFree or allocating library routine.
 * Limit: 2 * nrhs * 12 * V * e bytes (each half rounded up to 256) must fit,
 * e = 16 for DDAMG_FP64 and 8 otherwise; larger calls return DDAMG_EARG
 * before any work.  Every call on one GPU, from any context or stream, uses
 * that GPU's one array: calls that overlap in time on one GPU race, so
 * serialise them (e.g. one stream).  Nothing in the array is read before
 * this call writes it.  Asynchronous; out != in; 1 <= nrhs <= max_rhs. */
#define DDAMG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int dirac_apply_noalloc(ddamg_ctx* ctx, double* out, const double* in, int nrhs, int prec);

/* Convergence test of the coarse GMRES (Alg. 2), for timing comparisons.
 * Default (each_iteration = 0): pipelined -- the per-rhs convergence flags
 * of coarse iteration k are copied to pinned host memory behind its
 * kernels, and the host reads them only after it has enqueued iteration
 * k + 1, so the device never waits for the host's decision; every kernel of
 * an iteration is predicated on the flags, so the one iteration enqueued
 * past convergence does no work and changes no result.  With a fixed
 * iteration count (coarse_fixed_its > 0) nothing is read at all.
 * each_iteration = 1: the host waits for the flags after every iteration
 * (the device drains and idles while the next launches are issued).
 * Results are identical either way. */
int ddamg_set_coarse_host_sync(ddamg_ctx* ctx, int each_iteration);

/* ---- batched serving of independent instances ------------------------
 * Many small lattices of uneven sizes, each its own context, served
 * together: a pool of `workers` host threads (1 <= workers <= 64) takes the
 * instances in array order, each thread running one instance's call at a
 * time, so the kernels of up to `workers` instances are in flight at once;
 * an instance whose stream already has another instance in flight waits
 * and the next one is taken.
 * A small lattice fills a few compute units per launch; the instances'
 * kernels overlap on the GPU only if their contexts were created on
 * different streams (contexts sharing a stream, as ones drawn from a stream
 * pool may, are served one after the other, never concurrently).  Each instance gets exactly the
 * result of the single-instance call (same kernels, same order of work).
 * ctx[0 .. n-1] must be distinct contexts (a context is not thread-safe).
 * Per instance: rc[i] its return code; begin_ms[i] and end_ms[i] (either
 * may be NULL) when its call started and returned, in milliseconds from
 * the start of the batch.  Returns 0 if every rc is 0, DDAMG_NOT_CONVERGED
 * if none is negative and one is 1, else the first negative rc in instance
 * order (its context's ddamg_last_error tells why); argument errors are
 * returned before any instance starts.  Synchronous. */
/* mg_setup(ctx[i], NULL) for every instance (seeded starting vectors). */
int ddamg_batch_setup(ddamg_ctx* const* ctx, int n, int workers, int32_t* rc, double* begin_ms, double* end_ms);
/* solve(ctx[i], u[i], f[i], nrhs[i], tol, NULL) for every instance; u[i],
 * f[i] canonical device fields of instance i's lattice. */
int ddamg_batch_solve(ddamg_ctx* const* ctx, int n, double* const* u, const double* const* f, const int32_t* nrhs,
                      double tol, int workers, int32_t* rc, double* begin_ms, double* end_ms);

/* HIP graphs for the coarse GMRES (Alg. 2): on (the default), each coarse
 * iteration's launches (the Schur-complement stencil, the Gram-Schmidt
 * passes, the Arnoldi column, the scaling) are captured once per iteration
 * index and rhs count into a HIP graph on the context's stream and
 * replayed, one launch call per iteration instead of ten.  (Measured on
 * small lattices this changes little: the chain of small dependent kernels
 * on the device, not the host's launch calls, bounds such a solve.)
 * Results are identical either way.  Contexts on the null stream, and any context while
 * kernel timing is on, launch eagerly.  on = 0 launches eagerly always. */
int ddamg_set_graphs(ddamg_ctx* ctx, int on);

/* Small coarse lattices: at most 64 sites, at most 1.5 MiB of coarse
 * operator (9 blocks of nc x nc per site in the storage type, e.g. 8^4 with
 * 4^4 blocks and N_tv = 16 in FP32: 1.2 MiB) and a coarse restart length of
 * at most 32.  On (the default), the whole coarse solve of Alg. 2 for each
 * rhs -- the even/odd Schur complement, restarted GMRES with classical
 * Gram-Schmidt twice, the same Givens rotations and convergence test, the
 * back substitution and the even sites -- runs in one workgroup in one
 * launch, instead of about ten launches per GMRES iteration whose latencies
 * bound the solve of such a lattice.  One workgroup reads the operator at
 * the L2 bandwidth of one compute unit, hence the byte bound.  Results agree
 * with the multi-launch solve to rounding (sums in a different order).  Not
 * used while the host reads the convergence flags after every iteration
 * (ddamg_set_coarse_host_sync(ctx, 1)).  on = 0: always the multi-launch
 * solve. */
int ddamg_set_coarse_single_kernel(ddamg_ctx* ctx, int on);

/* Per-kernel-class timing for profiling: when enabled, every launch of the
 * classes below is bracketed by HIP events recorded on the context's stream
 * and the elapsed times are summed (the brackets add a few microseconds of
 * host overhead per launch).  ddamg_set_kernel_timing(ctx, on) zeroes the
 * sums; ddamg_get_kernel_times fills ms[k] (total milliseconds), count[k]
 * (timed launch groups) and rhs[k] (right-hand sides summed over those
 * groups) for k < n, synchronising the stream first. */
#define DDAMG_KERNEL_SAP 0              /* one SAP colour phase (Alg. 3) */
#define DDAMG_KERNEL_DSLASH 1           /* outer matvec w = D z (FP64 links) */
#define DDAMG_KERNEL_RESTRICT 2         /* y_c = R y (Eq. R) */
#define DDAMG_KERNEL_PROLONG 3          /* x = P x_c */
#define DDAMG_KERNEL_COARSE 4           /* D_c stencil pieces and D_ee^{-1} */
#define DDAMG_KERNEL_COARSE_GS 5        /* coarse GMRES Gram-Schmidt */
#define DDAMG_KERNEL_OUTER_GS 6         /* outer FGMRES Gram-Schmidt */
#define DDAMG_KERNEL_SETUP_QR 7         /* aggregate orthonormalisation (Alg. 5) */
#define DDAMG_KERNEL_SETUP_GALERKIN 8   /* D_ij P_j and its restriction (Eq. cgo) */
#define DDAMG_KERNEL_RESIDUAL 9         /* true residual f - D u at restarts (FP64) */
#define DDAMG_NKERNEL_KINDS 10
int ddamg_set_kernel_timing(ddamg_ctx* ctx, int on);
int ddamg_get_kernel_times(ddamg_ctx* ctx, double* ms, int64_t* count, int64_t* rhs, int n);

/* ---- learned proposal of test vectors --------------------------------
 * Not in the paper: the setup of Alg. 4 starts from random vectors; a
 * ddamg_net is a small gauge-covariant network that maps random fields to
 * proposed test vectors instead, trained on the device against the
 * aggregate basis (Alg. 5) of finished plain setups.
 *
 * Network: layers l = 0 .. L-1 map C_l channel fields phi_j (spinor fields)
 * to C_{l+1}:  psi_i(x) = sum_j [(a + b g5) phi_j(x) + sum_mu sum_s (c + d
 * g_mu) T_mu,s phi_j(x)] with the parallel transports T_mu,+ phi(x) =
 * U_mu(x) phi(x + mu), T_mu,- phi(x) = U_mu(x - mu)^dag phi(x - mu) under
 * the boundary conditions of D; between layers every channel passes the
 * gate phi / sqrt(1 + |phi(x)|^2 / 12) (|.| over spin and colour).  Weights,
 * complex64 (interleaved float pairs), layer after layer, each
 * [C_{l+1}][C_l][18]: index 0 = a, 1 = b, 2 + 2h = c and 3 + 2h = d of hop
 * h = 2 mu + s (s = 0 forward, 1 backward).  C_0 input fields (random),
 * C_L = ntv outputs.
 *
 * Span loss against an aggregate basis T (orthonormal per aggregate):
 * (1 / (N_A ntv)) sum_A ||(1 - P_A) T_A||_F^2, P_A the orthogonal
 * projector onto the span of the proposal on aggregate A; 0 when every
 * aggregate's proposal spans its target.  Gradients are dL/dRe w + i dL/dIm w.
 *
 * Random input fields: canonical complex128 [C_0][V][4][3] (device), or NULL
 * to draw them from seed exactly as mg_setup draws start vectors.
 * Arithmetic FP32.  A ddamg_net is not thread-safe; its calls synchronise
 * its stream. */
typedef struct ddamg_net ddamg_net;

/* channels[0 .. nlayers]: C_0 .. C_L, each in [1, 32], 1 <= nlayers <= 8;
 * weights start at zero; stream: hipStream_t (NULL = default). */
int ddamg_net_create(const int32_t* channels, int32_t nlayers, void* stream, ddamg_net** out);
int ddamg_net_destroy(ddamg_net* net);
const char* ddamg_net_last_error(const ddamg_net* net);
/* number of complex weights (float pairs) */
int64_t ddamg_net_num_weights(const ddamg_net* net);
/* device complex64 weights in the layout above; set resets Adam's state */
int ddamg_net_set_weights(ddamg_net* net, const float* w);
int ddamg_net_get_weights(ddamg_net* net, float* w);
/* Adds a training sample: the links of ctx (FP32) and its current aggregate
 * basis (dequantised to FP32) as the target.  ctx must have finished a
 * setup, have ntv = C_L, and all samples one lattice and blocking.
 * *index (may be NULL) receives the sample number. */
int ddamg_net_add_sample(ddamg_net* net, ddamg_ctx* ctx, int32_t* index);
/* Span loss of the proposal for sample's links and input fields against
 * its target; grad (device, complex64, weight layout, may be NULL)
 * receives the gradient.  DDAMG_ENUMERIC if the proposal has rank below
 * ntv on an aggregate. */
int ddamg_net_loss_grad(ddamg_net* net, int32_t sample, const double* noise, uint64_t seed, double* loss, float* grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, on real and imaginary
 * parts) with learning rate lr on the gradient of sample with input fields
 * drawn from seed; *loss (may be NULL) receives the loss before the step. */
int ddamg_net_train_step(ddamg_net* net, int32_t sample, uint64_t seed, float lr, double* loss);
/* Proposed test vectors on the lattice and links of ctx (ntv = C_L):
 * out canonical complex128 [ntv][V][4][3], for mg_setup (with init_passes
 * = 0 it starts the setup from them as they are). */
int ddamg_net_propose(ddamg_net* net, ddamg_ctx* ctx, const double* noise, uint64_t seed, double* out);

/* Geometry queries: number of sites and of blocks. */
int64_t ddamg_volume(const ddamg_ctx* ctx);
int32_t ddamg_nblocks(const ddamg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
