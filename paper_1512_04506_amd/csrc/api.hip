// C ABI of the library (include/ddamg.h) and the host-side orchestration of
// the two-level method: adaptive setup (Alg. 4, Alg. 5), V-cycle (Alg. 1),
// coarse-grid correction with the even/odd preconditioned coarse GMRES
// (Alg. 2), SAP smoother (Alg. 3) and the FP64 outer flexible GMRES
// (Sec. 1).  All arithmetic runs in the kernels of this library on the
// context's stream; the host only sequences launches and reads back the
// per-rhs convergence flags of the Krylov solvers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/ddamg.h"
#include "ddamg_internal.h"
#include "galerkin.h"

using namespace ddamg;

namespace {

struct Fail {
  int code;
  std::string msg;
};

#define HIPCK(call)                                                                   \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw Fail{DDAMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};      \
  } while (0)

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Fail{DDAMG_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
}

// A multi-dot launcher refuses (returns false, launches nothing) when its
// partial-sum buffer is smaller than the call needs; that is a sizing error
// of this library, reported instead of writing past the buffer.
inline void need_part(bool launched, const char* what) {
  if (!launched) throw Fail{DDAMG_ENOMEM, std::string(what) + ": partial-sum workspace too small"};
}

// Graph capture against device-wide calls.  HIP refuses a free or a device
// synchronisation while a stream of the process is being captured (the
// refused call's error then surfaces at a later check of that thread), and
// contexts served from several host threads capture on their own streams
// while other threads set up or grow their buffers.  So every capture holds
// this gate shared (captures on different streams still overlap) and every
// allocation, free or synchronous copy of the library holds it exclusively.
// An allocation inside a capture would deadlock on it and is refused.
std::shared_mutex g_capture_gate;
thread_local bool t_capturing = false;
using GateExclusive = std::unique_lock<std::shared_mutex>;

void* pinned_alloc(size_t bytes) {
  if (t_capturing) throw Fail{DDAMG_EHIP, "host allocation inside a graph capture"};
  GateExclusive lk(g_capture_gate);
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{DDAMG_ENOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  return p;
}
void pinned_free(void* p) {
  if (!p) return;
  GateExclusive lk(g_capture_gate);
  (void)hipHostFree(p);
}

// Workspace allocator: hipMalloc / hipFree unless the caller installed a
// hook; every buffer remembers the release function it was allocated with.
ddamg_alloc_fn g_alloc = nullptr;
ddamg_free_fn g_free = nullptr;
void* g_alloc_user = nullptr;

struct DevBuf {
  void* p = nullptr;
  ddamg_free_fn fr = nullptr;  // nullptr: hipFree
  void* user = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  template <typename X>
  X* get() const {
    return static_cast<X*>(p);
  }
  template <typename X>
  X* alloc(size_t n) {
    if (t_capturing) throw Fail{DDAMG_EHIP, "device allocation inside a graph capture"};
    GateExclusive lk(g_capture_gate);
    release_locked();
    const size_t bytes = (n == 0 ? 1 : n) * sizeof(X);
    if (g_alloc) {
      p = g_alloc(bytes, g_alloc_user);
      if (!p) throw Fail{DDAMG_ENOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes"};
      fr = g_free;
      user = g_alloc_user;
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        throw Fail{DDAMG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
      }
      fr = nullptr;
      user = nullptr;
    }
    return get<X>();
  }
  void release() {
    if (!p) return;
    GateExclusive lk(g_capture_gate);
    release_locked();
  }
  void release_locked() {
    if (p) {
      if (fr) {
        // hipFree waits for the device; a hook need not, so wait here (rare:
        // buffers change only at setup, first solves and destruction)
        (void)hipDeviceSynchronize();
        fr(p, user);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    fr = nullptr;
    user = nullptr;
  }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(fr, o.fr);
    std::swap(user, o.user);
  }
};

std::string g_create_error;

// Staging area of dirac_apply_noalloc: one copy of this array on every GPU
// the library runs on, held until the process ends.  Its host-side name is
// not a device address: resolve_scratch() looks up the address on the
// current device once, at context creation, and contexts keep it.
__device__ __align__(256) unsigned char scratch[DDAMG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* resolve_scratch() {
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Fail{DDAMG_EHIP, "device ordinal out of range"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Fail{DDAMG_EHIP, "hipGetSymbolAddress returned NULL for the staging array"};
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Opt-in per-kernel-class timing with HIP events recorded on the context's
// stream around each launch; elapsed times are collected at the next
// synchronisation point (or when many records are pending).
struct KTimer {
  bool on = false;
  struct Rec {
    int kind, nrhs;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  double ms[DDAMG_NKERNEL_KINDS] = {};
  int64_t count[DDAMG_NKERNEL_KINDS] = {};
  int64_t rhs[DDAMG_NKERNEL_KINDS] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) throw Fail{DDAMG_EHIP, "hipEventCreate failed"};
    return e;
  }
  template <typename F>
  void run(int kind, int nrhs, hipStream_t st, F&& f) {
    if (!on) {
      f();
      return;
    }
    hipEvent_t a = get(), b = get();
    (void)hipEventRecord(a, st);
    f();
    (void)hipEventRecord(b, st);
    pending.push_back({kind, nrhs, a, b});
    if (pending.size() >= 2048) collect();
  }
  void collect() {
    for (auto& r : pending) {
      (void)hipEventSynchronize(r.b);
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.kind] += t;
        count[r.kind] += 1;
        rhs[r.kind] += r.nrhs;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    collect();
    for (int k = 0; k < DDAMG_NKERNEL_KINDS; ++k) {
      ms[k] = 0.0;
      count[k] = 0;
      rhs[k] = 0;
    }
  }
  ~KTimer() {
    for (auto& r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct SolverBase;

struct ddamg_ctx {
  ddamg_params p{};
  Geom g{};
  hipStream_t st = nullptr;
  std::string err;
  // FP64 master fields and the derived storage precisions
  DevBuf U64, A64, U32, A32, Uh, Uhs, Ah, Ahs;
  // tables
  DevBuf nbr;
  DevBuf status;
  int* h_flags = nullptr;        // pinned host mirrors of small device arrays
  int* h_ring = nullptr;         // [2][64] pinned slots of the pipelined convergence test
  hipEvent_t ring_ev[2] = {nullptr, nullptr};
  double* h_dbl = nullptr;       // [128]
  cx<double>* h_cx = nullptr;    // [128]
  // canonical <-> internal staging
  DevBuf stage_in, stage_out;
  size_t stage_rhs = 0;
  void* scratch = nullptr;  // this device's address of the no-allocation staging array
  std::unique_ptr<SolverBase> sol;
  KTimer kt;
  bool setup_done = false;
  ddamg_stats stats{};

  GaugeView<double> gv64() const { return {U64.get<cx<double>>(), nullptr, A64.get<cx<double>>(), nullptr}; }
  GaugeView<float> gv32() const { return {U32.get<cx<float>>(), nullptr, A32.get<cx<float>>(), nullptr}; }
  GaugeView<__half> gvh() const {
    return {Uh.get<__half2>(), Uhs.get<float>(), Ah.get<__half2>(), Ahs.get<float>()};
  }
  void ensure_stage(int nrhs) {
    if ((size_t)nrhs <= stage_rhs) return;
    size_t n = (size_t)nrhs * 12 * g.V;
    stage_in.alloc<cx<double>>(n);
    stage_out.alloc<cx<double>>(n);
    stage_rhs = nrhs;
  }
  void sync() {
    HIPCK(hipStreamSynchronize(st));
    if (!kt.pending.empty()) kt.collect();
  }
  template <typename F>
  void timed(int kind, int nrhs, F&& f) {
    kt.run(kind, nrhs, st, f);
  }
  template <typename F>
  auto timed_ret(int kind, int nrhs, F&& f) -> decltype(f()) {
    decltype(f()) r{};
    kt.run(kind, nrhs, st, [&] { r = f(); });
    return r;
  }
  void free_pinned() {
    pinned_free(h_flags);
    pinned_free(h_ring);
    for (auto& e : ring_ev)
      if (e) (void)hipEventDestroy(e);
    h_ring = nullptr;
    ring_ev[0] = ring_ev[1] = nullptr;
    pinned_free(h_dbl);
    pinned_free(h_cx);
    h_flags = nullptr;
    h_dbl = nullptr;
    h_cx = nullptr;
  }
};

struct SolverBase {
  virtual ~SolverBase() = default;
  virtual void setup(const double* tv) = 0;
  virtual void import_basis(const double* W) = 0;
  virtual void export_basis(double* W) = 0;
  virtual void export_tv(double* tv) = 0;
  virtual void import_tv(const double* tv) = 0;
  virtual void import_coarse(const double* Dc) = 0;
  virtual void export_coarse(double* Dc) = 0;
  virtual void vcycle_canon(double* x, const double* y, int nrhs) = 0;
  virtual void coarse_canon(double* out, const double* in, int nrhs) = 0;
  virtual void coarse_internal(void* out, const void* in, int nrhs) = 0;
  virtual void restrict_canon(double* yc, const double* y, int nrhs) = 0;
  virtual void prolong_canon(double* x, const double* xc, int nrhs) = 0;
  virtual int solve(double* u, const double* f, int nrhs, double tol) = 0;
  virtual void coarse_stats(int& calls, int64_t& its, int& itmax) const = 0;
  virtual void set_coarse_host_sync(bool each_iteration) = 0;
  virtual void set_graphs(bool on) = 0;
  virtual void set_small_coarse(bool on) = 0;
  // the aggregate basis (dequantised) in FP32, internal layout [ntv][12][V]
  virtual void basis_f32(cx<float>* out) = 0;
  virtual void reset_coarse_stats() = 0;
};

namespace {

// Krylov workspace of one GMRES instance (coarse or outer)
struct Krylov {
  DevBuf H, cs, sn, g, y, est, inv_h, abstol, active, any, kdone, h1, h2, hc, n2, part, wscale, vscale;
  int m = 0, maxr = 0, ldh = 0;
  size_t part_cap = 0;  // entries of part
  ArnoldiState st{};
  void alloc(int m_, int maxr_, size_t n_per_rhs) {
    m = m_;
    maxr = maxr_;
    ldh = m + 1;
    H.alloc<cx<double>>((size_t)maxr * (m + 1) * m);
    cs.alloc<cx<double>>((size_t)maxr * m);
    sn.alloc<cx<double>>((size_t)maxr * m);
    g.alloc<cx<double>>((size_t)maxr * (m + 1));
    y.alloc<cx<double>>((size_t)maxr * m);
    est.alloc<double>(maxr);
    inv_h.alloc<double>(maxr);
    abstol.alloc<double>(maxr);
    active.alloc<int>(maxr);
    any.alloc<int>(1);
    kdone.alloc<int>(maxr);
    h1.alloc<cx<double>>((size_t)maxr * ldh);
    h2.alloc<cx<double>>((size_t)maxr * ldh);
    hc.alloc<cx<double>>((size_t)maxr * ldh);
    n2.alloc<cx<double>>(maxr);
    wscale.alloc<double>(maxr);
    vscale.alloc<double>(maxr);
    part_cap = krylov_part_entries(m, maxr, n_per_rhs);
    part.alloc<cx<double>>(part_cap);
    st.H = H.get<cx<double>>();
    st.cs = cs.get<cx<double>>();
    st.sn = sn.get<cx<double>>();
    st.g = g.get<cx<double>>();
    st.y = y.get<cx<double>>();
    st.est = est.get<double>();
    st.inv_h = inv_h.get<double>();
    st.abstol = abstol.get<double>();
    st.active = active.get<int>();
    st.any = any.get<int>();
    st.kdone = kdone.get<int>();
    st.m = m;
  }
};

template <typename T, typename S>
struct Solver final : SolverBase {
  ddamg_ctx* c;
  Geom g;
  hipStream_t st;
  GaugeView<S> gv;   // smoother links/clover (storage S)
  GaugeView<T> gva;  // links/clover used to assemble D_c (T)
  int maxr;          // max(max_rhs, ntv)
  // aggregate basis and coarse operator
  DevBuf Wq, Wsc, Dq, Dsc, Dinv, tv;
  // fine work vectors (T): y, x, r [maxr][12][V]
  DevBuf fy, fx;
  // setup workspace, allocated at the first setup and kept: FP64 copy of
  // the test vectors for the Gram-Schmidt, dequantised basis, D_c
  // accumulation buffer and the block operator applied to the basis columns
  DevBuf ws_Wd, ws_Wt, ws_D, ws_Z, ws_T;
  void ensure_setup_ws() {
    if (ws_Wd.p) return;
    ws_Wd.alloc<cx<double>>((size_t)g.ntv * fsz());
    ws_T.alloc<cx<double>>((size_t)2 * g.nblocks * QR_TWS_PER_AGG);
    if (is_half<S>()) ws_Wt.alloc<cx<T>>((size_t)g.ntv * fsz());  // else the stored basis is already cx<T>
    ws_D.alloc<cx<T>>((size_t)g.nblocks * 9 * g.nc * g.nc);
    ws_Z.alloc<cx<T>>((size_t)g.ntv * fsz());
  }
  // coarse work vectors (T)
  DevBuf yc, xc, te, ue, bo, cw, cV;
  Krylov ck;
  // partial sums of the setup's test-vector norms (fine vectors, ntv rhs)
  DevBuf npart;
  size_t npart_cap = 0;
  // outer FGMRES
  DevBuf oV, oZ, ow, of, ou, oyT;
  Krylov ok;
  int outer_m = 0, outer_r = 0;
  int coarse_calls = 0;
  int64_t coarse_its_total = 0;
  int coarse_its_max = 0;
  // read the coarse convergence flags after every iteration, stalling the
  // device (the former scheme, kept for the timing comparison)
  bool sync_each_coarse_it = false;
  // Each coarse GMRES iteration (Schur complement, CGS2, Arnoldi column,
  // scaling: ten launches) captured once per (iteration index, nrhs) into a
  // HIP graph and replayed: one launch call instead of ten.  The captured
  // kernels read only buffers allocated with the solver, so the graphs stay
  // valid for its lifetime; nothing captured is a memset or a host copy.
  // Not while kernel timing is on (its events would be captured too).
  bool use_graphs = true;
  std::map<std::pair<int, int>, hipGraphExec_t> step_graphs;
  // coarse lattices of at most COARSE_SMALL_MAX_SITES sites: the whole coarse
  // solve of a rhs in one workgroup (one launch instead of ten per
  // iteration); its iteration counts accumulate on the device
  bool use_small_coarse = true;
  DevBuf small_its;  // [2] iterations summed, maximum
  DevBuf u_nonzero;  // [maxr] flags: the solve's initial guess has a nonzero entry
  ~Solver() override {
    for (auto& kv : step_graphs) (void)hipGraphExecDestroy(kv.second);
  }
  void set_graphs(bool on) override { use_graphs = on; }
  void set_small_coarse(bool on) override { use_small_coarse = on; }
  bool small_coarse_applies() const {
    const size_t op_bytes = (size_t)g.nblocks * 9 * g.nc * g.nc * sizeof(stc_t<S>);
    return use_small_coarse && g.nblocks <= COARSE_SMALL_MAX_SITES && op_bytes <= COARSE_SMALL_MAX_BYTES &&
           (size_t)g.nblocks * g.nc <= (size_t)COARSE_SMALL_MAX_VECTOR &&
           c->p.coarse_restart <= COARSE_SMALL_MAX_RESTART && !sync_each_coarse_it;
  }
  template <typename F>
  void replay_step(int k, int nrhs, F&& enqueue) {
    // the null stream cannot be captured: contexts on it run eagerly
    if (!use_graphs || c->kt.on || st == nullptr) {
      enqueue();
      return;
    }
    auto it = step_graphs.find({k, nrhs});
    if (it == step_graphs.end()) {
      // thread-local capture: other contexts may capture on other threads;
      // the gate keeps other threads' allocations and frees out of it
      std::shared_lock<std::shared_mutex> gate(g_capture_gate);
      struct Flag {
        Flag() { t_capturing = true; }
        ~Flag() { t_capturing = false; }
      } flag;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        use_graphs = false;  // a stream that cannot be captured: stay eager
        t_capturing = false;
        enqueue();
        return;
      }
      hipGraph_t gr = nullptr;
      try {
        enqueue();
      } catch (...) {
        (void)hipStreamEndCapture(st, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      HIPCK(hipStreamEndCapture(st, &gr));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) throw Fail{DDAMG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
      it = step_graphs.emplace(std::make_pair(k, nrhs), ex).first;
    }
    HIPCK(hipGraphLaunch(it->second, st));
  }

  void coarse_stats(int& calls, int64_t& its, int& itmax) const override {
    calls = coarse_calls;
    its = coarse_its_total;
    itmax = coarse_its_max;
    int dev[2] = {0, 0};
    GateExclusive lk(g_capture_gate);
    if (hipStreamSynchronize(st) == hipSuccess &&
        hipMemcpy(dev, small_its.get<int>(), sizeof(dev), hipMemcpyDeviceToHost) == hipSuccess) {
      its += dev[0];
      itmax = std::max(itmax, dev[1]);
    }
  }
  void set_coarse_host_sync(bool each_iteration) override { sync_each_coarse_it = each_iteration; }
  void reset_coarse_stats() override {
    coarse_calls = 0;
    coarse_its_total = 0;
    coarse_its_max = 0;
    HIPCK(hipMemsetAsync(small_its.get<int>(), 0, 2 * sizeof(int), st));
  }

  size_t fsz() const { return (size_t)12 * g.V; }             // fine elements per rhs
  size_t csz() const { return (size_t)g.nblocks * g.nc; }      // coarse elements per rhs
  int nodd() const { return g.nblocks - g.neven; }
  size_t osz() const { return (size_t)nodd() * g.nc; }
  size_t esz() const { return (size_t)g.neven * g.nc; }

  BasisView<S> bv() const { return {Wq.get<stc_t<S>>(), Wsc.get<float>()}; }
  CoarseView<S> cv() const { return {Dq.get<stc_t<S>>(), Dsc.get<float>(), c->nbr.get<int>()}; }

  Solver(ddamg_ctx* ctx, GaugeView<S> gvs, GaugeView<T> gvt) : c(ctx), g(ctx->g), st(ctx->st), gv(gvs), gva(gvt) {
    maxr = std::max(c->p.max_rhs, g.ntv);
    Wq.alloc<stc_t<S>>((size_t)g.ntv * fsz());
    if (is_half<S>()) Wsc.alloc<float>((size_t)g.ntv * g.V);
    Dq.alloc<stc_t<S>>((size_t)g.nblocks * 9 * g.nc * g.nc);
    if (is_half<S>()) Dsc.alloc<float>((size_t)g.nblocks * 9);
    Dinv.alloc<cx<T>>((size_t)g.neven * g.nc * g.nc);
    tv.alloc<cx<T>>((size_t)maxr * fsz());  // as large as fy: the setup swaps the two
    fy.alloc<cx<T>>((size_t)maxr * fsz());
    fx.alloc<cx<T>>((size_t)maxr * fsz());
    yc.alloc<cx<T>>((size_t)maxr * csz());
    xc.alloc<cx<T>>((size_t)maxr * csz());
    te.alloc<cx<T>>((size_t)maxr * esz());
    ue.alloc<cx<T>>((size_t)maxr * esz());
    bo.alloc<cx<T>>((size_t)maxr * osz());
    cw.alloc<cx<T>>((size_t)maxr * osz());
    const int mc = c->p.coarse_restart;
    cV.alloc<cx<T>>((size_t)(mc + 1) * maxr * osz());
    ck.alloc(mc, maxr, std::max(osz(), csz()));
    npart_cap = setup_norm_part_entries(g.ntv, fsz());
    npart.alloc<cx<double>>(npart_cap);
    small_its.alloc<int>(2);
    HIPCK(hipMemsetAsync(small_its.get<int>(), 0, 2 * sizeof(int), st));
    u_nonzero.alloc<int>(maxr);
  }

  // ------------------------------------------------------------ smoother
  // nu cycles of red/black SAP on (x, y), Alg. 3
  void sap(cx<T>* x, const cx<T>* y, int nrhs, int nu) {
    for (int n = 0; n < nu; ++n)
      for (int col = 0; col < 2; ++col)
        c->timed(DDAMG_KERNEL_SAP, nrhs, [&] { launch_sap_phase<T, S>(x, y, gv, g, col, c->p.n_mr, nrhs, st); });
  }

  // -------------------------------------------------------- coarse solve
  // S v = D_oo v - D_oe D_ee^{-1} D_eo v on odd compact vectors
  // (v and w: odd-site vectors with rhs strides vstr and wstr)
  // gate (optional device flag): every kernel returns at once when it is 0
  void schur(cx<T>* w, size_t wstr, const cx<T>* v, size_t vstr, int nrhs, const int* gate = nullptr) {
    const CoarseView<S> C = cv();
    c->timed(DDAMG_KERNEL_COARSE, nrhs, [&] {
      launch_coarse_stencil<T, S>(te.get<cx<T>>(), esz(), 0, g.neven, nullptr, 0, nullptr, 0, 0, (T)0, v, vstr,
                                  g.neven, (T)1, C, g, nrhs, st, gate);
    });
    c->timed(DDAMG_KERNEL_COARSE, nrhs, [&] {
      launch_block_matvec<T>(ue.get<cx<T>>(), esz(), Dinv.get<cx<T>>(), te.get<cx<T>>(), esz(), g.neven, g.nc, nrhs,
                             st, gate);
    });
    c->timed(DDAMG_KERNEL_COARSE, nrhs, [&] {
      launch_coarse_stencil<T, S>(w, wstr, g.neven, nodd(), nullptr, 0, v, vstr, g.neven, (T)1, ue.get<cx<T>>(),
                                  esz(), 0, (T)-1, C, g, nrhs, st, gate);
    });
  }

  // Pipelined convergence test: post(slot) copies the per-rhs active flags
  // into a pinned host slot behind the work enqueued so far; any_posted(slot)
  // waits for that copy only.  Posting the flags of iteration k and reading
  // them after iteration k + 1 is enqueued keeps the device busy while the
  // host decides; kernels of inactive rhs return at once, so the iteration
  // enqueued past convergence changes nothing.
  void post_active(const Krylov& k, int nrhs, int slot) {
    HIPCK(hipMemcpyAsync(c->h_ring + 64 * slot, k.active.get<int>(), sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    HIPCK(hipEventRecord(c->ring_ev[slot], st));
  }
  int any_posted(int nrhs, int slot) {
    HIPCK(hipEventSynchronize(c->ring_ev[slot]));
    int any = 0;
    for (int r = 0; r < nrhs; ++r) any |= c->h_ring[64 * slot + r];
    return any;
  }

  int read_any_active(const Krylov& k, int nrhs) {
    HIPCK(hipMemcpyAsync(c->h_flags, k.active.get<int>(), sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    c->sync();
    int any = 0;
    for (int r = 0; r < nrhs; ++r) any |= c->h_flags[r];
    return any;
  }

  // classical Gram-Schmidt twice against V_0..V_k, then |w|^2
  template <typename Tv>
  void cgs2(Krylov& K, Tv* Vb, size_t vsj, size_t vsr, int k, Tv* w, size_t wsr, size_t n, int nrhs) {
    using E = typename std::remove_cv<decltype(Vb->r)>::type;
    const int* act = K.active.get<int>();
    cx<double>* part = K.part.get<cx<double>>();
    need_part(launch_mdot<E>(K.h1.get<cx<double>>(), K.ldh, part, K.part_cap, Vb, vsj, vsr, k + 1, w, wsr, n, nrhs,
                             act, st),
              "coarse Gram-Schmidt");
    launch_maxpy<E, E>(w, wsr, Vb, vsj, vsr, k + 1, K.h1.get<cx<double>>(), K.ldh, -1.0, n, nrhs, act, st);
    need_part(launch_mdot<E>(K.h2.get<cx<double>>(), K.ldh, part, K.part_cap, Vb, vsj, vsr, k + 1, w, wsr, n, nrhs,
                             act, st),
              "coarse Gram-Schmidt");
    launch_maxpy<E, E>(w, wsr, Vb, vsj, vsr, k + 1, K.h2.get<cx<double>>(), K.ldh, -1.0, n, nrhs, act, st);
    need_part(launch_mdot<E>(K.n2.get<cx<double>>(), 1, part, K.part_cap, w, 0, wsr, 1, w, wsr, n, nrhs, act, st),
              "coarse Gram-Schmidt");
  }

  // x_c = D_c^{-1} y_c approximately (Alg. 2), y_c/x_c full [nrhs][Nb][nc]
  int coarse_solve(cx<T>* xcv, const cx<T>* ycv, int nrhs) {
    const CoarseView<S> C = cv();
    const size_t cs_ = csz();
    const int fixed = c->p.coarse_fixed_its;
    const int m = c->p.coarse_restart;
    const int maxit = fixed > 0 ? fixed : c->p.coarse_maxit;
    if (small_coarse_applies()) {
      c->timed(DDAMG_KERNEL_COARSE, nrhs, [&] {
        launch_coarse_gmres_small<T, S>(xcv, ycv, cs_, C, Dinv.get<cx<T>>(), g, te.get<cx<T>>(), ue.get<cx<T>>(),
                                        bo.get<cx<T>>(), cw.get<cx<T>>(), cV.get<cx<T>>(), (size_t)maxr * osz(),
                                        m, maxit, fixed > 0 ? -1.0 : c->p.coarse_tol, small_its.get<int>(), nrhs, st);
      });
      check_launch("coarse solve");
      ++coarse_calls;
      return 0;  // the iterations are counted on the device
    }
    // ||y_c|| per rhs -> absolute tolerance (computed on the device)
    need_part(launch_mdot<T>(ck.n2.get<cx<double>>(), 1, ck.part.get<cx<double>>(), ck.part_cap, ycv, 0, cs_, 1, ycv,
                             cs_, cs_, nrhs, nullptr, st),
              "coarse right-hand side norm");
    launch_set_abstol(ck.abstol.get<double>(), ck.n2.get<cx<double>>(), fixed > 0 ? -1.0 : c->p.coarse_tol, nrhs, st);
    // b_o = y_o - D_oe D_ee^{-1} y_e
    launch_block_matvec<T>(te.get<cx<T>>(), esz(), Dinv.get<cx<T>>(), ycv, cs_, g.neven, g.nc, nrhs, st);
    launch_coarse_stencil<T, S>(bo.get<cx<T>>(), osz(), g.neven, nodd(), ycv + esz(), cs_, nullptr, 0, 0, (T)0,
                                te.get<cx<T>>(), esz(), 0, (T)-1, C, g, nrhs, st);
    cx<T>* xo = xcv + esz();
    HIPCK(hipMemsetAsync(xcv, 0, sizeof(cx<T>) * cs_ * nrhs, st));
    cx<T>* Vb = cV.get<cx<T>>();
    const size_t vsr = osz(), vsj = (size_t)maxr * osz();
    int its = 0;
    bool first = true;
    while (its < maxit) {
      // r = b_o - S x_o into V_0
      if (first) {
        launch_copy<T, T>(Vb, vsr, bo.get<cx<T>>(), osz(), osz(), nrhs, st);
      } else {
        schur(cw.get<cx<T>>(), osz(), xo, cs_, nrhs);
        launch_sub<T>(Vb, vsr, bo.get<cx<T>>(), osz(), cw.get<cx<T>>(), osz(), osz(), nrhs, st);
      }
      first = false;
      need_part(launch_mdot<T>(ck.n2.get<cx<double>>(), 1, ck.part.get<cx<double>>(), ck.part_cap, Vb, 0, vsr, 1, Vb,
                               vsr, osz(), nrhs, nullptr, st),
                "coarse residual norm");
      launch_arnoldi_start(ck.st, ck.n2.get<cx<double>>(), 1, nrhs, st);
      launch_scale<T, T>(Vb, vsr, Vb, vsr, ck.inv_h.get<double>(), osz(), nrhs, nullptr, st);
      // with a fixed iteration count the schedule is known: no host reads
      if ((fixed <= 0 || sync_each_coarse_it) && !read_any_active(ck, nrhs)) break;
      int k = 0;
      for (; k < m && its < maxit; ++k) {
        cx<T>* w = Vb + (size_t)(k + 1) * vsj;
        // every kernel of the iteration is predicated: on the rhs-wise
        // active flags, and the operator on "some rhs active"
        replay_step(k, nrhs, [&] {
          schur(w, vsr, Vb + (size_t)k * vsj, vsr, nrhs, ck.any.get<int>());
          c->timed(DDAMG_KERNEL_COARSE_GS, nrhs, [&] { cgs2(ck, Vb, vsj, vsr, k, w, vsr, osz(), nrhs); });
          launch_arnoldi_column(ck.st, k, ck.h1.get<cx<double>>(), ck.h2.get<cx<double>>(), ck.ldh,
                                ck.n2.get<cx<double>>(), 1, nrhs, st);
          launch_scale<T, T>(w, vsr, w, vsr, ck.inv_h.get<double>(), osz(), nrhs, ck.active.get<int>(), st);
        });
        ++its;
        if (sync_each_coarse_it) {
          if (!read_any_active(ck, nrhs)) {
            ++k;
            break;
          }
          continue;
        }
        if (fixed > 0) continue;
        post_active(ck, nrhs, k & 1);
        // iteration k is enqueued: decide on the flags of iteration k - 1
        if (k >= 1 && !any_posted(nrhs, (k - 1) & 1)) {
          --its;  // iteration k ran on inactive rhs only
          break;
        }
      }
      launch_arnoldi_solve(ck.st, nrhs, st);
      launch_maxpy<T, T>(xo, cs_, Vb, vsj, vsr, k, ck.y.get<cx<double>>(), m, 1.0, osz(), nrhs, nullptr, st);
    }
    // x_e = D_ee^{-1} (y_e - D_eo x_o)
    launch_coarse_stencil<T, S>(te.get<cx<T>>(), esz(), 0, g.neven, ycv, cs_, nullptr, 0, 0, (T)0, xo, cs_, g.neven,
                                (T)-1, C, g, nrhs, st);
    launch_block_matvec<T>(xcv, cs_, Dinv.get<cx<T>>(), te.get<cx<T>>(), esz(), g.neven, g.nc, nrhs, st);
    check_launch("coarse solve");
    ++coarse_calls;
    coarse_its_total += its;
    coarse_its_max = std::max(coarse_its_max, its);
    return its;
  }

  // -------------------------------------------------------------- V-cycle
  // x = M^{-1} y (Alg. 1): coarse-grid correction then SAP from it
  void vcycle(cx<T>* x, const cx<T>* y, int nrhs) {
    c->timed(DDAMG_KERNEL_RESTRICT, nrhs,
             [&] { launch_restrict<T, S>(yc.get<cx<T>>(), csz(), g.nc, y, fsz(), bv(), g, nrhs, st); });
    coarse_solve(xc.get<cx<T>>(), yc.get<cx<T>>(), nrhs);
    c->timed(DDAMG_KERNEL_PROLONG, nrhs,
             [&] { launch_prolong<T, S>(x, fsz(), xc.get<cx<T>>(), csz(), bv(), g, nrhs, st); });
    sap(x, y, nrhs, c->p.nu);
    check_launch("vcycle");
  }

  // ---------------------------------------------------------------- setup
  void normalise(cx<T>* v, int n) {
    need_part(launch_mdot<T>(ck.n2.get<cx<double>>(), 1, npart.get<cx<double>>(), npart_cap, v, 0, fsz(), 1, v, fsz(),
                             fsz(), n, nullptr, st),
              "test-vector norms");
    HIPCK(hipMemsetAsync(c->status.get<int>(), 0, sizeof(int), st));
    launch_inv_norm(ck.inv_h.get<double>(), ck.n2.get<cx<double>>(), n, c->status.get<int>(), st);
    launch_scale<T, T>(v, fsz(), v, fsz(), ck.inv_h.get<double>(), fsz(), n, nullptr, st);
    int stat = 0;
    HIPCK(hipMemcpyAsync(c->h_flags, c->status.get<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    c->sync();
    stat = c->h_flags[0];
    if (stat) throw Fail{DDAMG_ENUMERIC, "test vector with zero or non-finite norm"};
  }

  // Alg. 5 from an orthonormal FP64 basis Wd: store R (storage S), build
  // D_c = R D P from the stored basis, fill backward couplings by Eq. dagger,
  // quantise, and invert the even self blocks.
  void build_coarse_from(cx<double>* Wd) {
    ensure_setup_ws();
    const size_t nc = g.nc, nn = nc * nc;
    // the block pass reads the stored basis in T: for FP16 storage the FP32
    // values scale * half, written by the quantisation itself
    const cx<T>* Wtp;
    if constexpr (is_half<S>()) {
      static_assert(std::is_same<T, float>::value, "FP16 basis storage goes with FP32 arithmetic");
      launch_quantize_basis<S>(Wq.get<stc_t<S>>(), Wsc.get<float>(), Wd, g, st, ws_Wt.get<cx<float>>());
      Wtp = ws_Wt.get<cx<T>>();
    } else {
      launch_quantize_basis<S>(Wq.get<stc_t<S>>(), Wsc.get<float>(), Wd, g, st);
      Wtp = reinterpret_cast<const cx<T>*>(Wq.get<stc_t<S>>());
    }
    cx<T>* D = ws_D.get<cx<T>>();
    HIPCK(hipMemsetAsync(D, 0, sizeof(cx<T>) * g.nblocks * 9 * nn, st));
    // self slot: per chirality the block operator applied to all N_tv basis
    // columns, restricted; forward crossing slots: one fused contraction of
    // the basis (ntv <= 32 is validated at creation); backward slots by
    // Eq. (dagger)
    cx<T>* Zp = ws_Z.get<cx<T>>();
    for (int hp = 0; hp < 2; ++hp) {
      cx<T>* out = D + (size_t)(hp * g.ntv) * nc;  // slot 0, columns of chirality hp
      c->timed(DDAMG_KERNEL_SETUP_GALERKIN, g.ntv, [&] {
        launch_dslash<T, T, T, T>(Zp, Wtp, gva, g, g.ntv, DS_BLOCK, 0, hp, fsz(), fsz(), st);
        launch_restrict<T, S>(out, nc, 9 * nn, Zp, fsz(), bv(), g, g.ntv, st);
      });
    }
    c->timed(DDAMG_KERNEL_SETUP_GALERKIN, 2 * g.ntv, [&] { launch_galerkin_cross<T, S>(D, bv(), gva, g, st); });
    launch_dagger_fill<T>(D, c->nbr.get<int>(), g, st);
    launch_quantize_coarse<T, S>(Dq.get<stc_t<S>>(), Dsc.get<float>(), D, g, st);
    HIPCK(hipMemsetAsync(c->status.get<int>(), 0, sizeof(int), st));
    launch_invert_even_blocks<T, S>(Dinv.get<cx<T>>(), cv(), g, c->status.get<int>(), st);
    check_launch("build coarse");
    int stat = 0;
    HIPCK(hipMemcpyAsync(&stat, c->status.get<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    c->sync();
    if (stat) throw Fail{DDAMG_ENUMERIC, "singular even self-coupling block of D_c"};
  }

  // Gram-Schmidt of the current test vectors on every aggregate, then D_c
  void build_coarse() {
    ensure_setup_ws();
    cx<double>* W = ws_Wd.get<cx<double>>();
    HIPCK(hipMemsetAsync(c->status.get<int>(), 0, sizeof(int), st));
    // the first CholQR pass reads the test vectors in their own precision and
    // writes the FP64 copy W, the second works on W in place
    c->timed(DDAMG_KERNEL_SETUP_QR, g.ntv,
             [&] { launch_aggregate_qr<T>(W, tv.get<cx<T>>(), g, c->status.get<int>(), ws_T.get<cx<double>>(), st); });
    check_launch("aggregate qr");
    int stat = 0;
    HIPCK(hipMemcpyAsync(&stat, c->status.get<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    c->sync();
    if (stat) throw Fail{DDAMG_ENUMERIC, "rank-deficient aggregate in the Gram-Schmidt of the test vectors"};
    build_coarse_from(W);
  }

  void setup(const double* tv_canon) override {
    const int n = g.ntv;
    cx<T>* V = tv.get<cx<T>>();
    if (tv_canon)
      launch_spinor_to_internal<T>(V, reinterpret_cast<const cx<double>*>(tv_canon), g, n, st);
    else
      launch_gaussian_fields<T>(V, g, n, c->p.seed, st);
    // initial setup: smoother with N_smoother = 1, 2, 3 from a zero guess
    // (init_passes = 3, Alg. 4; fewer when the start vectors are already a
    // proposal); the current vectors move to fy (a buffer swap, no copy) and
    // the result is built in tv
    for (int k = 1; k <= c->p.init_passes; ++k) {
      tv.swap(fy);
      V = tv.get<cx<T>>();
      HIPCK(hipMemsetAsync(V, 0, sizeof(cx<T>) * fsz() * n, st));
      sap(V, fy.get<cx<T>>(), n, k);
    }
    build_coarse();
    normalise(V, n);
    // iterative setup: every test vector replaced by the V-cycle applied to
    // it, then R and D_c rebuilt (Alg. 4 normalises once, above; the
    // V-cycle is homogeneous and the aggregate Gram-Schmidt invariant to the
    // length of a vector, so the lengths only ride along)
    for (int i = 0; i < c->p.n_setup; ++i) {
      tv.swap(fy);
      V = tv.get<cx<T>>();
      vcycle(V, fy.get<cx<T>>(), n);
      build_coarse();
    }
    c->sync();
  }

  void import_basis(const double* Wc) override {
    ensure_setup_ws();
    cx<double>* W = ws_Wd.get<cx<double>>();
    launch_spinor_to_internal<double>(W, reinterpret_cast<const cx<double>*>(Wc), g, g.ntv, st);
    launch_copy<T, double>(tv.get<cx<T>>(), fsz(), W, fsz(), fsz(), g.ntv, st);
    build_coarse_from(W);
  }

  void basis_f32(cx<float>* out) override { launch_dequantize_basis<float, S>(out, bv(), g, st); }

  void export_basis(double* Wc) override {
    DevBuf Wt;
    cx<double>* W = Wt.alloc<cx<double>>((size_t)g.ntv * fsz());
    launch_dequantize_basis<double, S>(W, bv(), g, st);
    launch_spinor_to_canonical<double>(reinterpret_cast<cx<double>*>(Wc), W, g, g.ntv, st);
    c->sync();
  }
  void import_tv(const double* tvc) override {
    launch_spinor_to_internal<T>(tv.get<cx<T>>(), reinterpret_cast<const cx<double>*>(tvc), g, g.ntv, st);
    build_coarse();
    c->sync();
  }
  void import_coarse(const double* Dc) override {
    ensure_setup_ws();
    cx<T>* D = ws_D.get<cx<T>>();
    launch_coarse_import<T>(D, reinterpret_cast<const cx<double>*>(Dc), g, st);
    launch_quantize_coarse<T, S>(Dq.get<stc_t<S>>(), Dsc.get<float>(), D, g, st);
    HIPCK(hipMemsetAsync(c->status.get<int>(), 0, sizeof(int), st));
    launch_invert_even_blocks<T, S>(Dinv.get<cx<T>>(), cv(), g, c->status.get<int>(), st);
    check_launch("import coarse");
    int stat = 0;
    HIPCK(hipMemcpyAsync(&stat, c->status.get<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    c->sync();
    if (stat) throw Fail{DDAMG_ENUMERIC, "singular even self-coupling block of D_c"};
  }
  void export_tv(double* out) override {
    launch_spinor_to_canonical<T>(reinterpret_cast<cx<double>*>(out), tv.get<cx<T>>(), g, g.ntv, st);
    c->sync();
  }
  void export_coarse(double* out) override {
    launch_export_coarse<T, S>(reinterpret_cast<cx<double>*>(out), cv(), g, st);
    c->sync();
  }

  void vcycle_canon(double* x, const double* y, int nrhs) override {
    launch_spinor_to_internal<T>(fy.get<cx<T>>(), reinterpret_cast<const cx<double>*>(y), g, nrhs, st);
    vcycle(fx.get<cx<T>>(), fy.get<cx<T>>(), nrhs);
    launch_spinor_to_canonical<T>(reinterpret_cast<cx<double>*>(x), fx.get<cx<T>>(), g, nrhs, st);
  }

  void coarse_internal(void* out, const void* in, int nrhs) override {
    launch_coarse_stencil<T, S>(static_cast<cx<T>*>(out), csz(), 0, g.nblocks, nullptr, 0,
                                static_cast<const cx<T>*>(in), csz(), 0, (T)1, static_cast<const cx<T>*>(in), csz(), 0,
                                (T)1, cv(), g, nrhs, st);
  }
  void coarse_canon(double* out, const double* in, int nrhs) override {
    launch_coarse_to_internal<T>(yc.get<cx<T>>(), reinterpret_cast<const cx<double>*>(in), g, nrhs, st);
    coarse_internal(xc.get<cx<T>>(), yc.get<cx<T>>(), nrhs);
    launch_coarse_to_canonical<T>(reinterpret_cast<cx<double>*>(out), xc.get<cx<T>>(), g, nrhs, st);
  }
  void restrict_canon(double* ycn, const double* y, int nrhs) override {
    launch_spinor_to_internal<T>(fy.get<cx<T>>(), reinterpret_cast<const cx<double>*>(y), g, nrhs, st);
    launch_restrict<T, S>(yc.get<cx<T>>(), csz(), g.nc, fy.get<cx<T>>(), fsz(), bv(), g, nrhs, st);
    launch_coarse_to_canonical<T>(reinterpret_cast<cx<double>*>(ycn), yc.get<cx<T>>(), g, nrhs, st);
  }
  void prolong_canon(double* x, const double* xcn, int nrhs) override {
    launch_coarse_to_internal<T>(xc.get<cx<T>>(), reinterpret_cast<const cx<double>*>(xcn), g, nrhs, st);
    launch_prolong<T, S>(fx.get<cx<T>>(), fsz(), xc.get<cx<T>>(), csz(), bv(), g, nrhs, st);
    launch_spinor_to_canonical<T>(reinterpret_cast<cx<double>*>(x), fx.get<cx<T>>(), g, nrhs, st);
  }

  // ------------------------------------------------------- outer FGMRES
  // Classical Gram-Schmidt done twice against the outer basis V_0..V_k:
  // h1 = V^H w; w' = w - V h1 and h2 = V^H w' in one fused pass; |w''|^2 =
  // |w'|^2 - |h2|^2 (V orthonormal).  The Arnoldi column is h1 + h2 with
  // subdiagonal |w''|, complete after these two passes.  The vector itself,
  // v_{k+1} = (w' - V h2) / |w''|, is formed in the next step's fused pass,
  // which reads V_0..V_k anyway (gs_pending: slot k + 1 holds w', h2 and the
  // factor wait in hc and wscale); the inner products of the next w with it
  // follow from those with w' (launch_gs_defer_coef).  The preconditioner
  // then receives w' (in FP32 its copy, scaled to about unit norm by an
  // estimate of 1 / |w'| from the first pass, so that no FP32 quantity of
  // the V-cycle underflows), which FGMRES allows: it needs D z_k in the span
  // of V with the coefficients it records, whatever z_k is.  A step after which the next could not take the correction (basis
  // longer than GS_FUSED_MAXV) writes v_{k+1} in a third pass as before.
  bool gs_pending = false;
  void cgs2(cx<double>* V, size_t vsj, int k, int nrhs, cx<float>* w32) {
    const size_t n = fsz();
    const int* act = ok.active.get<int>();
    cx<double>* w = V + (size_t)(k + 1) * vsj;
    cx<double>* part = ok.part.get<cx<double>>();
    cx<double>* h1 = ok.h1.get<cx<double>>();
    cx<double>* h2 = ok.h2.get<cx<double>>();
    if (k + 1 <= GS_FUSED_MAXV) {
      // h1 = V^H w and, as the inner product of the last vector (w itself),
      // |w|^2, which gives the scale of the preconditioner's input
      need_part(launch_mdot<double>(h1, ok.ldh, part, ok.part_cap, V, vsj, n, k + 2, w, n, n, nrhs, act, st),
                "outer Gram-Schmidt");
      launch_gs_defer_coef(h1, ok.hc.get<cx<double>>(), h2, ok.ldh, ok.wscale.get<double>(), k, gs_pending,
                           ok.vscale.get<double>(), nrhs, act, st);
      const bool defer = k + 2 <= GS_FUSED_MAXV;
      need_part(launch_gs_defer(h2, ok.ldh, part, ok.part_cap, V, vsj, n, k, gs_pending, ok.hc.get<cx<double>>(),
                                ok.wscale.get<double>(), w, n, h1, n, nrhs, act, defer ? w32 : nullptr,
                                ok.vscale.get<double>(), st),
                "outer Gram-Schmidt");
      launch_gs_norm(ok.n2.get<cx<double>>(), ok.wscale.get<double>(), h2, ok.ldh, k + 1, nrhs, act, st);
      gs_pending = defer;
      if (defer) return;
    } else {  // long cycles: the same step in two passes (the last vector is w itself: |w|^2)
      need_part(launch_mdot<double>(h1, ok.ldh, part, ok.part_cap, V, vsj, n, k + 1, w, n, n, nrhs, act, st),
                "outer Gram-Schmidt");
      launch_maxpy<double, double>(w, n, V, vsj, n, k + 1, h1, ok.ldh, -1.0, n, nrhs, act, st);
      need_part(launch_mdot<double>(h2, ok.ldh, part, ok.part_cap, V, vsj, n, k + 2, w, n, n, nrhs, act, st),
                "outer Gram-Schmidt");
      launch_gs_norm(ok.n2.get<cx<double>>(), ok.wscale.get<double>(), h2, ok.ldh, k + 1, nrhs, act, st);
    }
    launch_maxpy<double, double>(w, n, V, vsj, n, k + 1, h2, ok.ldh, -1.0, n, nrhs, act, st,
                                 ok.wscale.get<double>(), w32);
  }

  // The outer basis V (FP64) and the preconditioned vectors Z grow with the
  // Krylov dimension actually reached: a 12-rhs FP64 vector of the 32^3x64
  // lattice is 4.8 GB, so a full FGMRES(20) basis would take most of HBM
  // although a cycle usually stops after a few iterations.
  int outer_cap = 0;  // vectors held by oV; oZ holds outer_cap - 1
  void ensure_outer(int m, int nrhs) {
    if (m == outer_m && nrhs <= outer_r) return;
    outer_m = m;
    outer_r = nrhs;
    const size_t n = fsz();
    outer_cap = std::min(m + 1, 2);  // doubled on demand by grow_outer
    oV.alloc<cx<double>>((size_t)outer_cap * nrhs * n);
    oZ.alloc<cx<T>>((size_t)(outer_cap - 1) * nrhs * n);
    ow.alloc<cx<double>>((size_t)nrhs * n);
    of.alloc<cx<double>>((size_t)nrhs * n);
    ou.alloc<cx<double>>((size_t)nrhs * n);
    ok.alloc(m, nrhs, n);
  }

  // room for basis vectors 0..kv-1 (and Z vectors 0..kv-2), contents kept
  void grow_outer(int kv) {
    if (kv <= outer_cap) return;
    const int cap = std::min(outer_m + 1, std::max(kv, 2 * outer_cap));
    const size_t vs = (size_t)outer_r * fsz();
    DevBuf nV, nZ;
    nV.alloc<cx<double>>((size_t)cap * vs);
    nZ.alloc<cx<T>>((size_t)(cap - 1) * vs);
    HIPCK(hipMemcpyAsync(nV.p, oV.p, sizeof(cx<double>) * outer_cap * vs, hipMemcpyDeviceToDevice, st));
    HIPCK(hipMemcpyAsync(nZ.p, oZ.p, sizeof(cx<T>) * (outer_cap - 1) * vs, hipMemcpyDeviceToDevice, st));
    c->sync();
    oV.swap(nV);
    oZ.swap(nZ);
    outer_cap = cap;
  }

  int solve(double* u_canon, const double* f_canon, int nrhs, double tol) override {
    const int m = c->p.outer_restart;
    ensure_outer(m, nrhs);
    const size_t n = fsz();
    const size_t vsj = (size_t)outer_r * n;  // stride between basis vectors
    cx<double>* V = oV.get<cx<double>>();
    cx<T>* Z = oZ.get<cx<T>>();
    cx<double>* w = ow.get<cx<double>>();
    cx<double>* f = of.get<cx<double>>();
    cx<double>* u = ou.get<cx<double>>();
    const GaugeView<double> g64 = c->gv64();
    launch_spinor_to_internal<double>(f, reinterpret_cast<const cx<double>*>(f_canon), g, nrhs, st);
    // the conversion of u also flags the rhs whose initial guess is nonzero
    HIPCK(hipMemsetAsync(u_nonzero.get<int>(), 0, sizeof(int) * nrhs, st));
    launch_spinor_to_internal<double>(u, reinterpret_cast<const cx<double>*>(u_canon), g, nrhs, st,
                                      u_nonzero.get<int>());
    // ||f||
    need_part(launch_mdot<double>(ok.n2.get<cx<double>>(), 1, ok.part.get<cx<double>>(), ok.part_cap, f, 0, n, 1, f, n,
                                  n, nrhs, nullptr, st),
              "right-hand side norm");
    std::vector<cx<double>> fn2(nrhs), rn2(nrhs);
    HIPCK(hipMemcpyAsync(c->h_cx, ok.n2.get<cx<double>>(), sizeof(cx<double>) * nrhs, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(c->h_flags, u_nonzero.get<int>(), sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    c->sync();
    std::copy(c->h_cx, c->h_cx + nrhs, fn2.begin());
    // all initial guesses zero: the first residual is f itself (D 0 = 0
    // exactly), a copy instead of the FP64 operator and a subtraction
    bool u_zero = true;
    for (int r = 0; r < nrhs; ++r) u_zero = u_zero && c->h_flags[r] == 0;
    std::vector<double> fnorm(nrhs), abstol(nrhs), zero_scale(nrhs, 1.0);
    bool any_zero = false;
    for (int r = 0; r < nrhs; ++r) {
      fnorm[r] = std::sqrt(std::max(fn2[r].r, 0.0));
      if (!std::isfinite(fnorm[r])) throw Fail{DDAMG_ENUMERIC, "non-finite right-hand side"};
      abstol[r] = tol * fnorm[r];
      if (fnorm[r] == 0.0) {
        zero_scale[r] = 0.0;  // f = 0: the solution is u = 0
        any_zero = true;
      }
    }
    std::copy(zero_scale.begin(), zero_scale.end(), c->h_dbl);
    std::copy(abstol.begin(), abstol.end(), c->h_dbl + 64);
    HIPCK(hipMemcpyAsync(ok.est.get<double>(), c->h_dbl, sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(ok.abstol.get<double>(), c->h_dbl + 64, sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    if (any_zero) launch_scale<double, double>(u, n, u, n, ok.est.get<double>(), n, nrhs, nullptr, st);
    int its = 0, restarts = 0;
    bool converged = false;
    std::vector<double> relres(nrhs, 0.0);
    for (;;) {
      // true residual r = f - D u in FP64, into V_0
      if (u_zero && its == 0) {
        launch_copy<double, double>(V, n, f, n, n, nrhs, st);
      } else {
        c->timed(DDAMG_KERNEL_RESIDUAL, nrhs,
                 [&] { launch_dslash<double, double, double, double>(w, u, g64, g, nrhs, DS_FULL, 0, -1, n, n, st); });
        launch_sub<double>(V, n, f, n, w, n, n, nrhs, st);
      }
      need_part(launch_mdot<double>(ok.n2.get<cx<double>>(), 1, ok.part.get<cx<double>>(), ok.part_cap, V, 0, n, 1, V,
                                    n, n, nrhs, nullptr, st),
                "residual norm");
      HIPCK(hipMemcpyAsync(c->h_cx, ok.n2.get<cx<double>>(), sizeof(cx<double>) * nrhs, hipMemcpyDeviceToHost, st));
      c->sync();
      std::copy(c->h_cx, c->h_cx + nrhs, rn2.begin());
      bool all = true;
      for (int r = 0; r < nrhs; ++r) {
        double rn = std::sqrt(std::max(rn2[r].r, 0.0));
        if (!std::isfinite(rn)) throw Fail{DDAMG_ENUMERIC, "non-finite residual in the outer solve"};
        relres[r] = fnorm[r] > 0.0 ? rn / fnorm[r] : 0.0;
        if (fnorm[r] > 0.0 && rn > abstol[r]) all = false;
      }
      if (all) {
        converged = true;
        break;
      }
      if (its >= c->p.outer_maxit) break;
      launch_arnoldi_start(ok.st, ok.n2.get<cx<double>>(), 1, nrhs, st);
      // V-cycle input: in FP32 a copy written with each new basis vector (or
      // with the w' that stands for it, see cgs2), in FP64 slot k itself
      constexpr bool f32 = std::is_same<T, float>::value;
      cx<float>* v32 = nullptr;
      if constexpr (f32) v32 = fy.get<cx<float>>();
      launch_scale<double, double>(V, n, V, n, ok.inv_h.get<double>(), n, nrhs, nullptr, st, v32);
      gs_pending = false;
      int k = 0;
      for (; k < m && its < c->p.outer_maxit; ++k) {
        grow_outer(k + 2);
        V = oV.get<cx<double>>();
        Z = oZ.get<cx<T>>();
        cx<double>* vk = V + (size_t)k * vsj;
        cx<T>* zk = Z + (size_t)k * vsj;
        // z_k = M^{-1} v_k (or M^{-1} w' while v_k is pending)
        if constexpr (f32)
          vcycle(zk, fy.get<cx<T>>(), nrhs);
        else
          vcycle(zk, vk, nrhs);
        // w = D z_k (FP64 operator)
        cx<double>* wk = V + (size_t)(k + 1) * vsj;
        c->timed(DDAMG_KERNEL_DSLASH, nrhs, [&] {
          if constexpr (std::is_same<T, double>::value)
            launch_dslash<double, double, double, double>(wk, zk, g64, g, nrhs, DS_FULL, 0, -1, n, n, st);
          else
            launch_dslash<float, double, double, double>(wk, zk, g64, g, nrhs, DS_FULL, 0, -1, n, n, st);
        });
        c->timed(DDAMG_KERNEL_OUTER_GS, nrhs, [&] { cgs2(V, vsj, k, nrhs, v32); });
        launch_arnoldi_column(ok.st, k, ok.h1.get<cx<double>>(), ok.h2.get<cx<double>>(), ok.ldh,
                              ok.n2.get<cx<double>>(), 1, nrhs, st);
        ++its;
        if (!read_any_active(ok, nrhs)) {
          ++k;
          break;
        }
      }
      launch_arnoldi_solve(ok.st, nrhs, st);
      launch_maxpy<double, T>(u, n, Z, vsj, n, k, ok.y.get<cx<double>>(), m, 1.0, n, nrhs, nullptr, st);
      ++restarts;
    }
    launch_spinor_to_canonical<double>(reinterpret_cast<cx<double>*>(u_canon), u, g, nrhs, st);
    check_launch("solve");
    c->sync();
    ddamg_stats& s = c->stats;
    s.outer_iterations = its;
    s.outer_restarts = restarts;
    s.nrhs = nrhs;
    s.converged = converged ? 1 : 0;
    for (int r = 0; r < 64; ++r) s.relres[r] = r < nrhs ? relres[r] : 0.0;
    return converged ? DDAMG_OK : DDAMG_NOT_CONVERGED;
  }
};

int fail_to_code(ddamg_ctx* c, const Fail& f) {
  if (c) c->err = f.msg;
  return f.code;
}

bool is_even_split(const ddamg_params* p, int mu) { return (p->L[mu] / p->block[mu]) % 2 == 0; }

int validate(const ddamg_params* p, std::string& why) {
  if (!p) {
    why = "params is NULL";
    return DDAMG_EARG;
  }
  int64_t V = 1, vb = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (p->L[mu] < 1 || p->block[mu] < 1) {
      why = "lattice and block extents must be positive";
      return DDAMG_EARG;
    }
    if (p->L[mu] % p->block[mu]) {
      why = "block extent must divide the lattice extent in direction " + std::to_string(mu);
      return DDAMG_EARG;
    }
    if (!is_even_split(p, mu)) {
      why = "the number of blocks in direction " + std::to_string(mu) +
            " must be even (red/black SAP and coarse even/odd)";
      return DDAMG_EARG;
    }
    V *= p->L[mu];
    vb *= p->block[mu];
  }
  if (V > (int64_t)1 << 28) {
    why = "lattice volume too large";
    return DDAMG_EARG;
  }
  if (vb > 256) {
    why = "block volume must be at most 256 sites";
    return DDAMG_EARG;
  }
  if (p->ntv < 1 || p->ntv > 32) {
    why = "ntv must be in [1, 32]";
    return DDAMG_EARG;
  }
  if (6 * vb < p->ntv) {
    why = "aggregates too small: 6 * block volume < ntv";
    return DDAMG_EARG;
  }
  if (p->n_setup < 0 || p->nu < 0 || p->n_mr < 0) {
    why = "n_setup, nu and n_mr must be non-negative";
    return DDAMG_EARG;
  }
  if (p->init_passes < 0 || p->init_passes > 16) {
    why = "init_passes must be in [0, 16]";
    return DDAMG_EARG;
  }
  if (p->coarse_restart < 1 || p->coarse_restart > 64 || p->outer_restart < 1 || p->outer_restart > 64) {
    why = "restart lengths must be in [1, 64]";
    return DDAMG_EARG;
  }
  if (p->coarse_maxit < 1 || p->outer_maxit < 1 || p->coarse_fixed_its < 0) {
    why = "iteration limits must be positive";
    return DDAMG_EARG;
  }
  if (p->coarse_fixed_its == 0 && !(p->coarse_tol > 0.0)) {
    why = "coarse_tol must be positive";
    return DDAMG_EARG;
  }
  if (p->prec != DDAMG_FP64 && p->prec != DDAMG_FP32 && p->prec != DDAMG_MIXED16) {
    why = "unknown precision";
    return DDAMG_EARG;
  }
  if (p->max_rhs < 1 || p->max_rhs > 64) {
    why = "max_rhs must be in [1, 64]";
    return DDAMG_EARG;
  }
  if (!std::isfinite(p->m0) || !std::isfinite(p->csw)) {
    why = "m0 and csw must be finite";
    return DDAMG_EARG;
  }
  return DDAMG_OK;
}

void build_tables(ddamg_ctx* c) {
  Geom& g = c->g;
  g.neven = g.nblocks / 2;
  std::vector<int> nbr((size_t)g.nblocks * 9);
  for (int ci = 0; ci < g.nblocks; ++ci) {
    int bc[4];
    int_block_coords(g, ci, bc);
    nbr[(size_t)ci * 9] = ci;
    for (int mu = 0; mu < 4; ++mu)
      for (int d = 0; d < 2; ++d) {
        int e[4] = {bc[0], bc[1], bc[2], bc[3]};
        e[mu] = (e[mu] + (d == 0 ? 1 : -1) + g.NB[mu]) % g.NB[mu];
        nbr[(size_t)ci * 9 + 1 + 2 * mu + d] = block_to_int(g, e);
      }
  }
  c->nbr.alloc<int>(nbr.size());
  GateExclusive lk(g_capture_gate);
  HIPCK(hipMemcpy(c->nbr.get<int>(), nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice));
}

}  // namespace

// ======================================== learned test-vector network
// A gauge-covariant network (k_learn.hip) that maps random fields to
// proposed test vectors, with its Adam state and a training set: per sample
// the FP32 links and the target aggregate basis of a finished setup.
struct NetSample {
  DevBuf U;  // FP32 links, internal layout [4][9][V]
  DevBuf T;  // FP32 target basis, internal layout [ntv][12][V]
};

// Work buffers of the network on one lattice: the input fields and every
// layer's pre-gate output, and (training only) gradients and partial sums.
struct NetWork {
  Geom g{};
  bool have = false;
  DevBuf act, gam0, gam1, lagg, part;
};

struct ddamg_net {
  std::vector<int> ch;        // channels C_0 .. C_L
  std::vector<size_t> woff;   // offset (complex weights) of every layer
  size_t nw = 0;              // complex weights
  hipStream_t st = nullptr;
  std::string err;
  DevBuf W, Wb, m, v, grad, loss, status;
  NetWork tw;                 // training (the samples' lattice)
  NetWork pw;                 // proposals on any lattice
  std::vector<std::unique_ptr<NetSample>> samples;
  int64_t step = 0;
  double* h_loss = nullptr;   // pinned
  int* h_stat = nullptr;      // pinned

  int nl() const { return (int)ch.size() - 1; }
  int cmax() const { return *std::max_element(ch.begin(), ch.end()); }
  // activations: [C_0 input | output of layer 0 | ... | output of layer L-1]
  cx<float>* act_ptr(NetWork& w, int l) const {
    size_t o = 0;
    for (int k = 0; k < l; ++k) o += (size_t)ch[k];
    return w.act.get<cx<float>>() + o * 12 * (size_t)w.g.V;
  }
  cx<float>* wl(int l) { return W.get<cx<float>>() + woff[l]; }

  static bool same_lattice(const Geom& a, const Geom& b) {
    for (int m = 0; m < 4; ++m)
      if (a.L[m] != b.L[m] || a.bs[m] != b.bs[m]) return false;
    return a.ntv == b.ntv;
  }
  void ensure(NetWork& w, const Geom& gl, bool training) {
    if (w.have && same_lattice(w.g, gl)) return;
    w.g = gl;
    w.have = true;
    const size_t V = gl.V;
    size_t tot = 0;
    for (int c : ch) tot += (size_t)c;
    w.act.alloc<cx<float>>(tot * 12 * V);
    if (!training) return;
    w.gam0.alloc<cx<float>>((size_t)cmax() * 12 * V);
    w.gam1.alloc<cx<float>>((size_t)cmax() * 12 * V);
    w.lagg.alloc<double>((size_t)2 * gl.nblocks);
    size_t pmax = 0;
    for (int l = 0; l < nl(); ++l) pmax = std::max(pmax, (size_t)ch[l] * ch[l + 1] * NET_NFEAT);
    w.part.alloc<cx<double>>((size_t)net_wgrad_chunks(gl) * pmax);
  }
  void sync() { HIPCK(hipStreamSynchronize(st)); }

  // forward on links gv: the input (canonical fields, or drawn from seed)
  // into act(0), every layer's pre-gate output into act(l + 1)
  void forward(NetWork& w, const GaugeView<float>& gv, const double* noise, uint64_t seed) {
    if (noise)
      launch_spinor_to_internal<float>(act_ptr(w, 0), reinterpret_cast<const cx<double>*>(noise), w.g, ch[0], st);
    else
      launch_gaussian_fields<float>(act_ptr(w, 0), w.g, ch[0], seed, st);
    for (int l = 0; l < nl(); ++l)
      launch_net_layer(act_ptr(w, l + 1), act_ptr(w, l), wl(l), ch[l], ch[l + 1], l > 0, nullptr, gv, w.g, st);
    check_launch("network forward");
  }

  // span loss against the target of sample k and the gradient of every
  // weight into grad; returns the loss
  double loss_grad(int k, const double* noise, uint64_t seed) {
    NetSample& smp = *samples[k];
    NetWork& w = tw;
    const GaugeView<float> gv{smp.U.get<cx<float>>(), nullptr, nullptr, nullptr};
    forward(w, gv, noise, seed);
    const int L = nl();
    HIPCK(hipMemsetAsync(status.get<int>(), 0, sizeof(int), st));
    cx<float>* gcur = w.gam0.get<cx<float>>();
    cx<float>* gnext = w.gam1.get<cx<float>>();
    launch_net_span_loss(gcur, w.lagg.get<double>(), loss.get<double>(), act_ptr(w, L), smp.T.get<cx<float>>(), w.g,
                         ch[L], status.get<int>(), st);
    for (int l = L - 1; l >= 0; --l) {
      cx<float>* gw = grad.get<cx<float>>() + woff[l];
      launch_net_wgrad(gw, w.part.get<cx<double>>(), act_ptr(w, l), l > 0, gcur, ch[l], ch[l + 1], gv, w.g, st);
      if (l > 0) {
        // input gradient: the transposed layer, then back through the gate
        launch_net_transpose(Wb.get<cx<float>>(), wl(l), ch[l], ch[l + 1], st);
        launch_net_layer(gnext, gcur, Wb.get<cx<float>>(), ch[l + 1], ch[l], false, act_ptr(w, l), gv, w.g, st);
        std::swap(gcur, gnext);
      }
    }
    check_launch("network backward");
    HIPCK(hipMemcpyAsync(h_loss, loss.get<double>(), sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(h_stat, status.get<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    sync();
    if (*h_stat) throw Fail{DDAMG_ENUMERIC, "proposal of rank below N_tv on an aggregate (span loss undefined)"};
    if (!std::isfinite(*h_loss)) throw Fail{DDAMG_ENUMERIC, "non-finite span loss"};
    return *h_loss;
  }

  ~ddamg_net() {
    pinned_free(h_loss);
    pinned_free(h_stat);
  }
};

// ================================================================== C ABI
namespace {
// A pool of host threads serving independent instances: each thread takes
// the next instance index and runs one(i); the calling thread is one of the
// workers.  If a thread cannot be started, the ones that did (at least the
// caller) serve every instance.  rc[i] and the times are written by the
// thread that ran instance i.
template <typename F>
int serve_batch(ddamg_ctx* const* ctx, int n, int workers, const std::vector<int>& order, int32_t* rc,
                double* begin_ms, double* end_ms, F&& one) {
  // Each worker takes the first instance in `order` whose stream has no
  // other instance in flight: contexts may share a stream (a stream pool
  // hands out a limited number), and two calls on one stream from two
  // threads would interleave their work, or put one's launches into the
  // other's graph capture.  Such instances run one after the other.
  std::mutex mx;
  std::condition_variable freed;
  std::vector<char> taken(n, 0);
  std::vector<hipStream_t> busy;
  int head = 0, left = n;
  const auto start = std::chrono::steady_clock::now();
  auto ms = [&] { return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - start).count(); };
  auto work = [&] {
    for (;;) {
      int i = -1;
      {
        std::unique_lock<std::mutex> lk(mx);
        for (;;) {
          if (left == 0) return;
          for (int q = head; q < n && i < 0; ++q) {
            const int j = order[q];
            if (!taken[j] && std::find(busy.begin(), busy.end(), ctx[j]->st) == busy.end()) i = j;
          }
          if (i >= 0) break;
          freed.wait(lk);
        }
        taken[i] = 1;
        --left;
        busy.push_back(ctx[i]->st);
        while (head < n && taken[order[head]]) ++head;
      }
      const double a = ms();
      const int r = one(i);
      const double b = ms();
      rc[i] = r;
      if (begin_ms) begin_ms[i] = a;
      if (end_ms) end_ms[i] = b;
      {
        std::lock_guard<std::mutex> lk(mx);
        busy.erase(std::find(busy.begin(), busy.end(), ctx[i]->st));
      }
      freed.notify_all();
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < std::min(workers, n); ++w) {
    try {
      pool.emplace_back(work);
    } catch (const std::exception&) {
      break;
    }
  }
  work();
  for (auto& t : pool) t.join();
  int first_neg = 0, any_nc = 0;
  for (int i = 0; i < n; ++i) {
    if (rc[i] < 0 && first_neg == 0) first_neg = rc[i];
    if (rc[i] == DDAMG_NOT_CONVERGED) any_nc = 1;
  }
  return first_neg ? first_neg : (any_nc ? DDAMG_NOT_CONVERGED : DDAMG_OK);
}

std::vector<int> array_order(int n) {
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  return order;
}

int check_batch(ddamg_ctx* const* ctx, int n, int workers, const int32_t* rc) {
  if (!ctx || n < 0 || !rc) return DDAMG_EARG;
  if (workers < 1 || workers > 64) return DDAMG_EARG;
  std::unordered_set<const ddamg_ctx*> seen;
  for (int i = 0; i < n; ++i)
    if (!ctx[i] || !seen.insert(ctx[i]).second) return DDAMG_EARG;
  return DDAMG_OK;
}
}  // namespace

extern "C" {

void ddamg_default_params(ddamg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  for (int mu = 0; mu < 4; ++mu) {
    p->L[mu] = 8;
    p->block[mu] = 4;
  }
  p->m0 = 0.0;
  p->csw = 1.0;
  p->ntv = 24;
  p->n_setup = 3;
  p->nu = 3;
  p->n_mr = 4;
  p->coarse_tol = 0.05;
  p->coarse_restart = 30;
  p->coarse_maxit = 300;
  p->coarse_fixed_its = 0;
  p->outer_restart = 20;
  p->outer_maxit = 2000;
  p->prec = DDAMG_MIXED16;
  p->max_rhs = 12;
  p->init_passes = 3;
  p->seed = 0;
}

int ddamg_validate_params(const ddamg_params* p, char* msg, size_t msg_len) {
  std::string why;
  int rc = validate(p, why);
  if (msg && msg_len) {
    std::snprintf(msg, msg_len, "%s", why.c_str());
  }
  return rc;
}

int ddamg_create(const ddamg_params* p, const double* gauge, void* stream, ddamg_ctx** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return DDAMG_EARG;
  }
  *out = nullptr;
  std::string why;
  int rc = validate(p, why);
  if (rc) {
    g_create_error = why;
    return rc;
  }
  if (!gauge) {
    g_create_error = "gauge is NULL";
    return DDAMG_EARG;
  }
  std::unique_ptr<ddamg_ctx> c(new ddamg_ctx());
  try {
    c->p = *p;
    c->st = static_cast<hipStream_t>(stream);
    c->scratch = resolve_scratch();
    preload_dslash_code();
    Geom& g = c->g;
    g.V = 1;
    g.vblock = 1;
    g.nblocks = 1;
    for (int mu = 0; mu < 4; ++mu) {
      g.L[mu] = p->L[mu];
      g.bs[mu] = p->block[mu];
      g.NB[mu] = p->L[mu] / p->block[mu];
      g.V *= g.L[mu];
      g.vblock *= g.bs[mu];
      g.nblocks *= g.NB[mu];
    }
    g.ntv = p->ntv;
    g.nc = 2 * p->ntv;
    g.lstr[0] = 1;
    for (int mu = 1; mu < 4; ++mu) g.lstr[mu] = g.lstr[mu - 1] * g.bs[mu - 1];
    build_tables(c.get());
    c->h_flags = static_cast<int*>(pinned_alloc(64 * sizeof(int)));
    c->h_ring = static_cast<int*>(pinned_alloc(2 * 64 * sizeof(int)));
    for (auto& e : c->ring_ev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->h_dbl = static_cast<double*>(pinned_alloc(128 * sizeof(double)));
    c->h_cx = static_cast<cx<double>*>(pinned_alloc(128 * sizeof(cx<double>)));
    c->status.alloc<int>(1);
    const size_t V = g.V;
    c->U64.alloc<cx<double>>(36 * V);
    c->A64.alloc<cx<double>>(2 * CLOVER_PAIRS * V);
    c->U32.alloc<cx<float>>(36 * V);
    c->A32.alloc<cx<float>>(2 * CLOVER_PAIRS * V);
    c->Uh.alloc<__half2>(36 * V);
    c->Uhs.alloc<float>(V);
    c->Ah.alloc<__half2>(2 * CLOVER_PAIRS * V);
    c->Ahs.alloc<float>(V);
    launch_gauge_import(c->U64.get<cx<double>>(), reinterpret_cast<const cx<double>*>(gauge), g, c->st);
    launch_clover_build(c->A64.get<cx<double>>(), c->U64.get<cx<double>>(), g, p->m0, p->csw, c->st);
    launch_quantize_gauge<float>(c->U32.get<cx<float>>(), nullptr, c->A32.get<cx<float>>(), nullptr,
                                 c->U64.get<cx<double>>(), c->A64.get<cx<double>>(), g, c->st);
    launch_quantize_gauge<__half>(c->Uh.get<__half2>(), c->Uhs.get<float>(), c->Ah.get<__half2>(),
                                  c->Ahs.get<float>(), c->U64.get<cx<double>>(), c->A64.get<cx<double>>(), g, c->st);
    check_launch("create");
    switch (p->prec) {
      case DDAMG_FP64:
        c->sol.reset(new Solver<double, double>(c.get(), c->gv64(), c->gv64()));
        break;
      case DDAMG_FP32:
        c->sol.reset(new Solver<float, float>(c.get(), c->gv32(), c->gv32()));
        break;
      default:
        c->sol.reset(new Solver<float, __half>(c.get(), c->gvh(), c->gv32()));
        break;
    }
    c->sync();
  } catch (const Fail& f) {
    g_create_error = f.msg;
    c->free_pinned();
    return f.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    c->free_pinned();
    return DDAMG_ENOMEM;
  }
  *out = c.release();
  return DDAMG_OK;
}

int ddamg_destroy(ddamg_ctx* c) {
  if (!c) return DDAMG_EARG;
  (void)hipStreamSynchronize(c->st);
  c->sol.reset();
  c->free_pinned();
  delete c;
  return DDAMG_OK;
}

const char* ddamg_last_error(const ddamg_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

#define GUARD_BEGIN try {
#define GUARD_END                            \
  }                                          \
  catch (const Fail& f) {                    \
    return fail_to_code(c, f);               \
  }                                          \
  catch (const std::exception& e) {          \
    c->err = e.what();                       \
    return DDAMG_ENOMEM;                     \
  }

static int need_setup(ddamg_ctx* c) {
  if (!c->setup_done) {
    c->err = "call mg_setup (or ddamg_import_basis) first";
    return DDAMG_ESTATE;
  }
  return 0;
}
static int check_rhs(ddamg_ctx* c, int nrhs) {
  if (nrhs < 1 || nrhs > c->p.max_rhs) {
    c->err = "nrhs must be in [1, max_rhs]";
    return DDAMG_EARG;
  }
  return 0;
}

int mg_setup(ddamg_ctx* c, const double* tv_init) {
  if (!c) return DDAMG_EARG;
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  c->setup_done = false;
  c->sol->setup(tv_init);
  c->setup_done = true;
  c->stats.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return DDAMG_OK;
  GUARD_END
}

int ddamg_import_basis(ddamg_ctx* c, const double* W) {
  if (!c) return DDAMG_EARG;
  if (!W) {
    c->err = "W is NULL";
    return DDAMG_EARG;
  }
  GUARD_BEGIN
  c->setup_done = false;
  c->sol->import_basis(W);
  c->setup_done = true;
  return DDAMG_OK;
  GUARD_END
}

int ddamg_export_basis(ddamg_ctx* c, double* W) {
  if (!c || !W) return DDAMG_EARG;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->export_basis(W);
  return DDAMG_OK;
  GUARD_END
}

int ddamg_export_tv(ddamg_ctx* c, double* tv) {
  if (!c || !tv) return DDAMG_EARG;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->export_tv(tv);
  return DDAMG_OK;
  GUARD_END
}

int ddamg_import_tv(ddamg_ctx* c, const double* tv) {
  if (!c) return DDAMG_EARG;
  if (!tv) {
    c->err = "tv is NULL";
    return DDAMG_EARG;
  }
  GUARD_BEGIN
  c->setup_done = false;
  c->sol->import_tv(tv);
  c->setup_done = true;
  return DDAMG_OK;
  GUARD_END
}

int ddamg_import_coarse(ddamg_ctx* c, const double* Dc) {
  if (!c) return DDAMG_EARG;
  if (!Dc) {
    c->err = "Dc is NULL";
    return DDAMG_EARG;
  }
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->import_coarse(Dc);
  return DDAMG_OK;
  GUARD_END
}

int ddamg_set_allocator(ddamg_alloc_fn alloc, ddamg_free_fn free_fn, void* user) {
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    g_create_error = "ddamg_set_allocator: alloc and free_fn must both be set or both be NULL";
    return DDAMG_EARG;
  }
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_user = alloc ? user : nullptr;
  return DDAMG_OK;
}

int ddamg_export_coarse(ddamg_ctx* c, double* Dc) {
  if (!c || !Dc) return DDAMG_EARG;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->export_coarse(Dc);
  return DDAMG_OK;
  GUARD_END
}

int ddamg_export_clover(ddamg_ctx* c, double* A) {
  if (!c || !A) return DDAMG_EARG;
  GUARD_BEGIN
  launch_clover_export(reinterpret_cast<cx<double>*>(A), c->A64.get<cx<double>>(), c->g, c->st);
  check_launch("export clover");
  c->sync();
  return DDAMG_OK;
  GUARD_END
}

int mg_apply(ddamg_ctx* c, double* x, const double* y, int nrhs) {
  if (!c) return DDAMG_EARG;
  if (!x || !y || x == y) {
    c->err = "x and y must be distinct non-NULL pointers";
    return DDAMG_EARG;
  }
  if (int e = check_rhs(c, nrhs)) return e;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->vcycle_canon(x, y, nrhs);
  check_launch("mg_apply");
  return DDAMG_OK;
  GUARD_END
}

int dirac_apply_internal(ddamg_ctx* c, void* out, const void* in, int nrhs, int prec) {
  if (!c) return DDAMG_EARG;
  if (!out || !in || out == in) {
    c->err = "out and in must be distinct non-NULL pointers";
    return DDAMG_EARG;
  }
  if (nrhs < 1 || nrhs > 65535) {
    c->err = "nrhs out of range";
    return DDAMG_EARG;
  }
  GUARD_BEGIN
  const Geom& g = c->g;
  const size_t n = (size_t)12 * g.V;
  switch (prec) {
    case DDAMG_FP64:
      launch_dslash<double, double, double, double>(static_cast<cx<double>*>(out), static_cast<const cx<double>*>(in),
                                                    c->gv64(), g, nrhs, DS_FULL, 0, -1, n, n, c->st);
      break;
    case DDAMG_FP32:
      launch_dslash<float, float, float, float>(static_cast<cx<float>*>(out), static_cast<const cx<float>*>(in),
                                                c->gv32(), g, nrhs, DS_FULL, 0, -1, n, n, c->st);
      break;
    case DDAMG_MIXED16:
      launch_dslash<float, float, __half, float>(static_cast<cx<float>*>(out), static_cast<const cx<float>*>(in),
                                                 c->gvh(), g, nrhs, DS_FULL, 0, -1, n, n, c->st);
      break;
    default:
      c->err = "unknown precision";
      return DDAMG_EARG;
  }
  check_launch("dirac_apply_internal");
  return DDAMG_OK;
  GUARD_END
}

// out = D in on canonical fields through internal-layout copies a (of in)
// and b (of out), each nrhs * 12 * V elements of the precision's type
static int dirac_apply_staged(ddamg_ctx* c, double* out, const double* in, int nrhs, int prec, void* a, void* b) {
  const Geom& g = c->g;
  const cx<double>* cin = reinterpret_cast<const cx<double>*>(in);
  cx<double>* cout = reinterpret_cast<cx<double>*>(out);
  if (prec == DDAMG_FP64) {
    launch_spinor_to_internal<double>(static_cast<cx<double>*>(a), cin, g, nrhs, c->st);
    int rc = dirac_apply_internal(c, b, a, nrhs, prec);
    if (rc) return rc;
    launch_spinor_to_canonical<double>(cout, static_cast<cx<double>*>(b), g, nrhs, c->st);
  } else {
    launch_spinor_to_internal<float>(static_cast<cx<float>*>(a), cin, g, nrhs, c->st);
    int rc = dirac_apply_internal(c, b, a, nrhs, prec);
    if (rc) return rc;
    launch_spinor_to_canonical<float>(cout, static_cast<cx<float>*>(b), g, nrhs, c->st);
  }
  check_launch("dirac_apply");
  return DDAMG_OK;
}

static int dirac_apply_args(ddamg_ctx* c, double* out, const double* in, int nrhs, int prec) {
  if (!out || !in || out == in) {
    c->err = "out and in must be distinct non-NULL pointers";
    return DDAMG_EARG;
  }
  if (int e = check_rhs(c, nrhs)) return e;
  if (prec != DDAMG_FP64 && prec != DDAMG_FP32 && prec != DDAMG_MIXED16) {
    c->err = "unknown precision";
    return DDAMG_EARG;
  }
  return DDAMG_OK;
}

int dirac_apply(ddamg_ctx* c, double* out, const double* in, int nrhs, int prec) {
  if (!c) return DDAMG_EARG;
  if (int e = dirac_apply_args(c, out, in, nrhs, prec)) return e;
  GUARD_BEGIN
  c->ensure_stage(nrhs);
  return dirac_apply_staged(c, out, in, nrhs, prec, c->stage_in.p, c->stage_out.p);
  GUARD_END
}

int dirac_apply_noalloc(ddamg_ctx* c, double* out, const double* in, int nrhs, int prec) {
  if (!c) return DDAMG_EARG;
  if (int e = dirac_apply_args(c, out, in, nrhs, prec)) return e;
  const size_t es = prec == DDAMG_FP64 ? sizeof(cx<double>) : sizeof(cx<float>);
  const size_t half = ((size_t)nrhs * 12 * c->g.V * es + 255) / 256 * 256;
  if (2 * half > DDAMG_NOALLOC_SCRATCH_BYTES) {
    c->err = "dirac_apply_noalloc: 2 * nrhs * 12 * V * " + std::to_string(es) + " bytes of staging exceed "
             "DDAMG_NOALLOC_SCRATCH_BYTES (" + std::to_string((size_t)DDAMG_NOALLOC_SCRATCH_BYTES) + ")";
    return DDAMG_EARG;
  }
  if (!c->scratch) {
    c->err = "dirac_apply_noalloc: no staging array on this device";
    return DDAMG_ESTATE;
  }
  GUARD_BEGIN
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  return dirac_apply_staged(c, out, in, nrhs, prec, base, base + half);
  GUARD_END
}

int coarse_apply(ddamg_ctx* c, double* out, const double* in, int nrhs) {
  if (!c) return DDAMG_EARG;
  if (!out || !in || out == in) {
    c->err = "out and in must be distinct non-NULL pointers";
    return DDAMG_EARG;
  }
  if (int e = check_rhs(c, nrhs)) return e;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->coarse_canon(out, in, nrhs);
  check_launch("coarse_apply");
  return DDAMG_OK;
  GUARD_END
}

int coarse_apply_internal(ddamg_ctx* c, void* out, const void* in, int nrhs) {
  if (!c) return DDAMG_EARG;
  if (!out || !in || out == in) {
    c->err = "out and in must be distinct non-NULL pointers";
    return DDAMG_EARG;
  }
  if (nrhs < 1 || nrhs > 65535) {
    c->err = "nrhs out of range";
    return DDAMG_EARG;
  }
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->coarse_internal(out, in, nrhs);
  check_launch("coarse_apply_internal");
  return DDAMG_OK;
  GUARD_END
}

int mg_restrict(ddamg_ctx* c, double* yc, const double* y, int nrhs) {
  if (!c) return DDAMG_EARG;
  if (!yc || !y) {
    c->err = "NULL pointer";
    return DDAMG_EARG;
  }
  if (int e = check_rhs(c, nrhs)) return e;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->restrict_canon(yc, y, nrhs);
  check_launch("mg_restrict");
  return DDAMG_OK;
  GUARD_END
}

int mg_prolong(ddamg_ctx* c, double* x, const double* xc, int nrhs) {
  if (!c) return DDAMG_EARG;
  if (!x || !xc) {
    c->err = "NULL pointer";
    return DDAMG_EARG;
  }
  if (int e = check_rhs(c, nrhs)) return e;
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  c->sol->prolong_canon(x, xc, nrhs);
  check_launch("mg_prolong");
  return DDAMG_OK;
  GUARD_END
}

int solve(ddamg_ctx* c, double* u, const double* f, int nrhs, double tol, ddamg_stats* st) {
  if (!c) return DDAMG_EARG;
  if (!u || !f || u == f) {
    c->err = "u and f must be distinct non-NULL pointers";
    return DDAMG_EARG;
  }
  if (int e = check_rhs(c, nrhs)) return e;
  if (!(tol > 0.0) || !(tol < 1.0)) {
    c->err = "tol must be in (0, 1)";
    return DDAMG_EARG;
  }
  if (int e = need_setup(c)) return e;
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  int rc = c->sol->solve(u, f, nrhs, tol);
  c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) ddamg_get_stats(c, st);
  return rc;
  GUARD_END
}

int ddamg_get_stats(const ddamg_ctx* c, ddamg_stats* st) {
  if (!c || !st) return DDAMG_EARG;
  *st = c->stats;
  if (c->sol) c->sol->coarse_stats(st->coarse_solves, st->coarse_iterations, st->coarse_iterations_max);
  return DDAMG_OK;
}

int ddamg_reset_stats(ddamg_ctx* c) {
  if (!c) return DDAMG_EARG;
  if (c->sol) c->sol->reset_coarse_stats();
  return DDAMG_OK;
}

int ddamg_set_coarse_host_sync(ddamg_ctx* c, int each_iteration) {
  if (!c) return DDAMG_EARG;
  if (each_iteration != 0 && each_iteration != 1) {
    c->err = "each_iteration must be 0 or 1";
    return DDAMG_EARG;
  }
  c->sol->set_coarse_host_sync(each_iteration == 1);
  return DDAMG_OK;
}

int ddamg_set_graphs(ddamg_ctx* c, int on) {
  if (!c) return DDAMG_EARG;
  if (on != 0 && on != 1) {
    c->err = "on must be 0 or 1";
    return DDAMG_EARG;
  }
  c->sol->set_graphs(on == 1);
  return DDAMG_OK;
}

int ddamg_set_coarse_single_kernel(ddamg_ctx* c, int on) {
  if (!c) return DDAMG_EARG;
  if (on != 0 && on != 1) {
    c->err = "on must be 0 or 1";
    return DDAMG_EARG;
  }
  c->sol->set_small_coarse(on == 1);
  return DDAMG_OK;
}

int ddamg_batch_setup(ddamg_ctx* const* ctx, int n, int workers, int32_t* rc, double* begin_ms, double* end_ms) {
  if (int e = check_batch(ctx, n, workers, rc)) return e;
  return serve_batch(ctx, n, workers, array_order(n), rc, begin_ms, end_ms,
                     [&](int i) { return mg_setup(ctx[i], nullptr); });
}

int ddamg_batch_solve(ddamg_ctx* const* ctx, int n, double* const* u, const double* const* f, const int32_t* nrhs,
                      double tol, int workers, int32_t* rc, double* begin_ms, double* end_ms) {
  if (int e = check_batch(ctx, n, workers, rc)) return e;
  if (n > 0 && (!u || !f || !nrhs)) return DDAMG_EARG;
  // the per-instance arguments are checked here, before any instance starts
  for (int i = 0; i < n; ++i) {
    ddamg_ctx* c = ctx[i];
    if (!u[i] || !f[i] || u[i] == f[i]) {
      c->err = "u and f must be distinct non-NULL pointers";
      return DDAMG_EARG;
    }
    if (int e = check_rhs(c, nrhs[i])) return e;
    if (!(tol > 0.0) || !(tol < 1.0)) {
      c->err = "tol must be in (0, 1)";
      return DDAMG_EARG;
    }
    if (int e = need_setup(c)) return e;
  }
  return serve_batch(ctx, n, workers, array_order(n), rc, begin_ms, end_ms,
                     [&](int i) { return solve(ctx[i], u[i], f[i], nrhs[i], tol, nullptr); });
}

int ddamg_set_kernel_timing(ddamg_ctx* c, int on) {
  if (!c) return DDAMG_EARG;
  GUARD_BEGIN
  c->sync();
  c->kt.reset();
  c->kt.on = on != 0;
  return DDAMG_OK;
  GUARD_END
}

int ddamg_get_kernel_times(ddamg_ctx* c, double* ms, int64_t* count, int64_t* rhs, int n) {
  if (!c || !ms || !count || !rhs || n < 1) return DDAMG_EARG;
  GUARD_BEGIN
  c->sync();
  for (int k = 0; k < n; ++k) {
    ms[k] = k < DDAMG_NKERNEL_KINDS ? c->kt.ms[k] : 0.0;
    count[k] = k < DDAMG_NKERNEL_KINDS ? c->kt.count[k] : 0;
    rhs[k] = k < DDAMG_NKERNEL_KINDS ? c->kt.rhs[k] : 0;
  }
  return DDAMG_OK;
  GUARD_END
}

// ------------------------------------------------ learned proposal (C ABI)
int ddamg_net_create(const int32_t* channels, int32_t nlayers, void* stream, ddamg_net** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return DDAMG_EARG;
  }
  *out = nullptr;
  if (!channels || nlayers < 1 || nlayers > 8) {
    g_create_error = "channels must be given for 1 to 8 layers";
    return DDAMG_EARG;
  }
  for (int l = 0; l <= nlayers; ++l)
    if (channels[l] < 1 || channels[l] > 32) {
      g_create_error = "channel counts must be in [1, 32]";
      return DDAMG_EARG;
    }
  std::unique_ptr<ddamg_net> n(new ddamg_net());
  try {
    n->ch.assign(channels, channels + nlayers + 1);
    n->st = static_cast<hipStream_t>(stream);
    for (int l = 0; l < nlayers; ++l) {
      n->woff.push_back(n->nw);
      n->nw += (size_t)channels[l] * channels[l + 1] * NET_NFEAT;
    }
    size_t wbmax = 0;
    for (int l = 0; l < nlayers; ++l) wbmax = std::max(wbmax, (size_t)channels[l] * channels[l + 1] * NET_NFEAT);
    n->W.alloc<cx<float>>(n->nw);
    n->Wb.alloc<cx<float>>(wbmax);
    n->m.alloc<cx<float>>(n->nw);
    n->v.alloc<cx<float>>(n->nw);
    n->grad.alloc<cx<float>>(n->nw);
    n->loss.alloc<double>(1);
    n->status.alloc<int>(1);
    HIPCK(hipMemsetAsync(n->W.p, 0, sizeof(cx<float>) * n->nw, n->st));
    HIPCK(hipMemsetAsync(n->m.p, 0, sizeof(cx<float>) * n->nw, n->st));
    HIPCK(hipMemsetAsync(n->v.p, 0, sizeof(cx<float>) * n->nw, n->st));
    n->h_loss = static_cast<double*>(pinned_alloc(sizeof(double)));
    n->h_stat = static_cast<int*>(pinned_alloc(sizeof(int)));
    n->sync();
  } catch (const Fail& f) {
    g_create_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return DDAMG_ENOMEM;
  }
  *out = n.release();
  return DDAMG_OK;
}

int ddamg_net_destroy(ddamg_net* n) {
  if (!n) return DDAMG_EARG;
  (void)hipStreamSynchronize(n->st);
  delete n;
  return DDAMG_OK;
}

const char* ddamg_net_last_error(const ddamg_net* n) { return n ? n->err.c_str() : g_create_error.c_str(); }

int64_t ddamg_net_num_weights(const ddamg_net* n) { return n ? (int64_t)n->nw : -1; }

#define NET_GUARD_BEGIN try {
#define NET_GUARD_END                        \
  }                                          \
  catch (const Fail& f) {                    \
    n->err = f.msg;                          \
    return f.code;                           \
  }                                          \
  catch (const std::exception& e) {          \
    n->err = e.what();                       \
    return DDAMG_ENOMEM;                     \
  }

int ddamg_net_set_weights(ddamg_net* n, const float* w) {
  if (!n || !w) return DDAMG_EARG;
  NET_GUARD_BEGIN
  HIPCK(hipMemcpyAsync(n->W.p, w, sizeof(cx<float>) * n->nw, hipMemcpyDeviceToDevice, n->st));
  HIPCK(hipMemsetAsync(n->m.p, 0, sizeof(cx<float>) * n->nw, n->st));
  HIPCK(hipMemsetAsync(n->v.p, 0, sizeof(cx<float>) * n->nw, n->st));
  n->step = 0;
  n->sync();
  return DDAMG_OK;
  NET_GUARD_END
}

int ddamg_net_get_weights(ddamg_net* n, float* w) {
  if (!n || !w) return DDAMG_EARG;
  NET_GUARD_BEGIN
  HIPCK(hipMemcpyAsync(w, n->W.p, sizeof(cx<float>) * n->nw, hipMemcpyDeviceToDevice, n->st));
  n->sync();
  return DDAMG_OK;
  NET_GUARD_END
}

int ddamg_net_add_sample(ddamg_net* n, ddamg_ctx* c, int32_t* index) {
  if (!n || !c) return DDAMG_EARG;
  if (!c->setup_done) {
    n->err = "the lattice context has no aggregate basis yet (mg_setup first)";
    return DDAMG_ESTATE;
  }
  if (c->g.ntv != n->ch.back()) {
    n->err = "the network's output channels differ from the context's ntv";
    return DDAMG_EARG;
  }
  if (!n->samples.empty() && !ddamg_net::same_lattice(n->tw.g, c->g)) {
    n->err = "all training samples must be on one lattice and blocking";
    return DDAMG_EARG;
  }
  NET_GUARD_BEGIN
  n->ensure(n->tw, c->g, true);
  std::unique_ptr<NetSample> smp(new NetSample());
  const size_t V = c->g.V;
  smp->U.alloc<cx<float>>((size_t)36 * V);
  smp->T.alloc<cx<float>>((size_t)c->g.ntv * 12 * V);
  HIPCK(hipMemcpyAsync(smp->U.p, c->U32.p, sizeof(cx<float>) * 36 * V, hipMemcpyDeviceToDevice, c->st));
  c->sol->basis_f32(smp->T.get<cx<float>>());
  check_launch("network sample");
  c->sync();
  n->samples.push_back(std::move(smp));
  if (index) *index = (int32_t)n->samples.size() - 1;
  return DDAMG_OK;
  NET_GUARD_END
}

int ddamg_net_loss_grad(ddamg_net* n, int32_t sample, const double* noise, uint64_t seed, double* loss, float* grad) {
  if (!n) return DDAMG_EARG;
  if (sample < 0 || sample >= (int32_t)n->samples.size()) {
    n->err = "no such sample";
    return DDAMG_EARG;
  }
  NET_GUARD_BEGIN
  const double l = n->loss_grad(sample, noise, seed);
  if (loss) *loss = l;
  if (grad) {
    HIPCK(hipMemcpyAsync(grad, n->grad.p, sizeof(cx<float>) * n->nw, hipMemcpyDeviceToDevice, n->st));
    n->sync();
  }
  return DDAMG_OK;
  NET_GUARD_END
}

int ddamg_net_train_step(ddamg_net* n, int32_t sample, uint64_t seed, float lr, double* loss) {
  if (!n) return DDAMG_EARG;
  if (sample < 0 || sample >= (int32_t)n->samples.size()) {
    n->err = "no such sample";
    return DDAMG_EARG;
  }
  if (!(lr > 0.f)) {
    n->err = "lr must be positive";
    return DDAMG_EARG;
  }
  NET_GUARD_BEGIN
  const double l = n->loss_grad(sample, nullptr, seed);
  n->step += 1;
  launch_adam(n->W.get<float>(), n->m.get<float>(), n->v.get<float>(), n->grad.get<float>(), 2 * n->nw, lr, n->step,
              n->st);
  check_launch("network Adam step");
  if (loss) *loss = l;
  return DDAMG_OK;
  NET_GUARD_END
}

int ddamg_net_propose(ddamg_net* n, ddamg_ctx* c, const double* noise, uint64_t seed, double* out) {
  if (!n || !c || !out) return DDAMG_EARG;
  NET_GUARD_BEGIN
  if (c->g.ntv != n->ch.back()) {
    n->err = "the network's output channels differ from the context's ntv";
    return DDAMG_EARG;
  }
  if (n->st != c->st) HIPCK(hipStreamSynchronize(c->st));
  n->ensure(n->pw, c->g, false);
  n->forward(n->pw, c->gv32(), noise, seed);
  launch_spinor_to_canonical<float>(reinterpret_cast<cx<double>*>(out), n->act_ptr(n->pw, n->nl()), n->pw.g,
                                    n->ch.back(), n->st);
  check_launch("network proposal");
  n->sync();
  return DDAMG_OK;
  NET_GUARD_END
}

int64_t ddamg_volume(const ddamg_ctx* c) { return c ? (int64_t)c->g.V : -1; }
int32_t ddamg_nblocks(const ddamg_ctx* c) { return c ? c->g.nblocks : -1; }

}  // extern "C"
