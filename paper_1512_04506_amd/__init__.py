"""Python binding of libddamg.so, the gfx950 two-level DD-alpha-AMG library.

Thin ctypes marshalling only: every step of the method runs in the HIP
kernels behind the C ABI declared in include/ddamg.h.  The functions keep the
ABI's names (mg_setup, mg_apply, dirac_apply, coarse_apply, solve, ...).
PyTorch provides device memory and the stream: arguments are complex128
CUDA/HIP tensors in the canonical layouts of the header, for example spinor
fields of shape (nrhs, Lt, Lz, Ly, Lx, 4, 3).

Importing this package fails loudly when the library is not built; there is
no CPU fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddamg.so")

ABI_VERSION = 2  # DDAMG_ABI_VERSION of include/ddamg.h this binding follows
FP64, FP32, MIXED16 = 0, 1, 2
OK, NOT_CONVERGED = 0, 1
ERRORS = {-1: "invalid argument", -2: "wrong state", -3: "HIP error", -4: "out of memory", -5: "numerical failure"}

EXPORTS = (
    "ddamg_default_params", "ddamg_validate_params", "ddamg_create", "ddamg_destroy", "ddamg_last_error",
    "mg_setup", "ddamg_import_basis", "ddamg_export_basis", "ddamg_export_tv", "ddamg_export_coarse",
    "ddamg_export_clover", "mg_apply", "dirac_apply", "coarse_apply", "mg_restrict", "mg_prolong", "solve",
    "ddamg_get_stats", "ddamg_reset_stats", "dirac_apply_internal", "coarse_apply_internal", "ddamg_volume",
    "ddamg_nblocks", "ddamg_set_kernel_timing", "ddamg_get_kernel_times", "ddamg_import_tv",
    "ddamg_import_coarse", "ddamg_set_allocator", "dirac_apply_noalloc", "ddamg_set_coarse_host_sync",
    "ddamg_net_create", "ddamg_net_destroy", "ddamg_net_last_error", "ddamg_net_num_weights",
    "ddamg_net_set_weights", "ddamg_net_get_weights", "ddamg_net_add_sample", "ddamg_net_loss_grad",
    "ddamg_net_train_step", "ddamg_net_propose", "ddamg_batch_setup", "ddamg_batch_solve", "ddamg_set_graphs",
    "ddamg_set_coarse_single_kernel",
)
KERNEL_KINDS = ("sap", "dslash", "restrict", "prolong", "coarse", "coarse_gs", "outer_gs", "setup_qr",
                "setup_galerkin", "residual")


class DDAMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ddamg error %d (%s): %s" % (code, ERRORS.get(code, "?"), msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32 * 4), ("block", ctypes.c_int32 * 4), ("m0", ctypes.c_double),
        ("csw", ctypes.c_double), ("ntv", ctypes.c_int32), ("n_setup", ctypes.c_int32),
        ("nu", ctypes.c_int32), ("n_mr", ctypes.c_int32), ("coarse_tol", ctypes.c_double),
        ("coarse_restart", ctypes.c_int32), ("coarse_maxit", ctypes.c_int32),
        ("coarse_fixed_its", ctypes.c_int32), ("outer_restart", ctypes.c_int32),
        ("outer_maxit", ctypes.c_int32), ("prec", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
        ("init_passes", ctypes.c_int32), ("seed", ctypes.c_uint64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_iterations", ctypes.c_int32), ("outer_restarts", ctypes.c_int32),
        ("coarse_solves", ctypes.c_int32), ("coarse_iterations_max", ctypes.c_int32),
        ("coarse_iterations", ctypes.c_int64), ("nrhs", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("relres", ctypes.c_double * 64), ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "relres"}
        d["relres"] = list(self.relres[: max(self.nrhs, 0)])
        return d


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libddamg.so is not built (run paper_1512_04506_amd/build.py); "
                          "there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int
    sig = {
        "ddamg_default_params": (None, [ctypes.POINTER(Params)]),
        "ddamg_validate_params": (i32, [ctypes.POINTER(Params), ctypes.c_char_p, ctypes.c_size_t]),
        "ddamg_create": (i32, [ctypes.POINTER(Params), dp, vp, ctypes.POINTER(vp)]),
        "ddamg_destroy": (i32, [vp]),
        "ddamg_last_error": (ctypes.c_char_p, [vp]),
        "mg_setup": (i32, [vp, dp]),
        "ddamg_import_basis": (i32, [vp, dp]),
        "ddamg_export_basis": (i32, [vp, dp]),
        "ddamg_export_tv": (i32, [vp, dp]),
        "ddamg_export_coarse": (i32, [vp, dp]),
        "ddamg_import_tv": (i32, [vp, dp]),
        "ddamg_import_coarse": (i32, [vp, dp]),
        "ddamg_set_allocator": (i32, [ALLOC_FN, FREE_FN, vp]),
        "ddamg_export_clover": (i32, [vp, dp]),
        "mg_apply": (i32, [vp, dp, dp, i32]),
        "dirac_apply": (i32, [vp, dp, dp, i32, i32]),
        "dirac_apply_noalloc": (i32, [vp, dp, dp, i32, i32]),
        "coarse_apply": (i32, [vp, dp, dp, i32]),
        "mg_restrict": (i32, [vp, dp, dp, i32]),
        "mg_prolong": (i32, [vp, dp, dp, i32]),
        "solve": (i32, [vp, dp, dp, i32, ctypes.c_double, ctypes.POINTER(Stats)]),
        "ddamg_get_stats": (i32, [vp, ctypes.POINTER(Stats)]),
        "ddamg_reset_stats": (i32, [vp]),
        "dirac_apply_internal": (i32, [vp, vp, vp, i32, i32]),
        "coarse_apply_internal": (i32, [vp, vp, vp, i32]),
        "ddamg_volume": (ctypes.c_int64, [vp]),
        "ddamg_nblocks": (ctypes.c_int32, [vp]),
        "ddamg_set_kernel_timing": (i32, [vp, i32]),
        "ddamg_set_coarse_host_sync": (i32, [vp, i32]),
        "ddamg_set_graphs": (i32, [vp, i32]),
        "ddamg_set_coarse_single_kernel": (i32, [vp, i32]),
        "ddamg_net_create": (i32, [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, vp, ctypes.POINTER(vp)]),
        "ddamg_net_destroy": (i32, [vp]),
        "ddamg_net_last_error": (ctypes.c_char_p, [vp]),
        "ddamg_net_num_weights": (ctypes.c_int64, [vp]),
        "ddamg_net_set_weights": (i32, [vp, vp]),
        "ddamg_net_get_weights": (i32, [vp, vp]),
        "ddamg_net_add_sample": (i32, [vp, vp, ctypes.POINTER(ctypes.c_int32)]),
        "ddamg_net_loss_grad": (i32, [vp, ctypes.c_int32, dp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), vp]),
        "ddamg_net_train_step": (i32, [vp, ctypes.c_int32, ctypes.c_uint64, ctypes.c_float,
                                       ctypes.POINTER(ctypes.c_double)]),
        "ddamg_net_propose": (i32, [vp, vp, dp, ctypes.c_uint64, dp]),
        "ddamg_get_kernel_times": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64), i32]),
        "ddamg_batch_setup": (i32, [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "ddamg_batch_solve": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_double, i32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


_allocator_refs = []  # every installed pair stays alive: buffers free through the pair they came from


def set_allocator(alloc=None, free=None):
    """ddamg_set_allocator: alloc(nbytes) -> device address (int, 0 on
    failure) and free(address) own the workspace of contexts created from
    now on; set_allocator() restores hipMalloc / hipFree.  Both are called
    from the library's thread while it holds no Python state."""
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must both be given or both be None")
    if alloc is None:
        rc = lib.ddamg_set_allocator(ALLOC_FN(), FREE_FN(), None)
    else:
        a = ALLOC_FN(lambda n, user: alloc(int(n)) or None)
        f = FREE_FN(lambda ptr, user: free(int(ptr)))
        _allocator_refs.append((a, f))
        rc = lib.ddamg_set_allocator(a, f, None)
    if rc != 0:
        raise DDAMGError(rc, lib.ddamg_last_error(None).decode())


def default_params(**kw):
    """ddamg_default_params, then keyword overrides (L and block as 4-tuples
    in x, y, z, t order)."""
    p = Params()
    lib.ddamg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("L", "block"):
            arr = getattr(p, k)
            for i in range(4):
                arr[i] = int(v[i])
        else:
            setattr(p, k, v)
    return p


def validate_params(p):
    """(code, message) of ddamg_validate_params; touches no GPU."""
    buf = ctypes.create_string_buffer(256)
    rc = lib.ddamg_validate_params(ctypes.byref(p), buf, 256)
    return rc, buf.value.decode()


def _ptr(t, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() * t.element_size() != numel:
        raise ValueError("%s has %d bytes, expected %d" % (name, t.numel() * t.element_size(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One ddamg_ctx on the current device and torch's current stream."""

    def __init__(self, params, gauge, stream=None):
        import torch
        self.params = params
        self.L = tuple(params.L)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.nblocks = 1
        for m in range(4):
            self.nblocks *= self.L[m] // params.block[m]
        self.ntv = params.ntv
        if gauge.dtype != torch.complex128:
            raise TypeError("gauge must be complex128")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.ddamg_create(ctypes.byref(params), _ptr(gauge, "gauge", self.V * 36 * 16),
                              ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise DDAMGError(rc, lib.ddamg_last_error(None).decode())
        self.h = h

    # -- helpers -----------------------------------------------------------
    def _check(self, rc):
        if rc < 0:
            raise DDAMGError(rc, lib.ddamg_last_error(self.h).decode())
        return rc

    def fine_bytes(self, nrhs):
        return nrhs * self.V * 12 * 16

    def coarse_bytes(self, nrhs):
        return nrhs * self.nblocks * 2 * self.ntv * 16

    def close(self):
        if getattr(self, "h", None):
            lib.ddamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI -----------------------------------------------------------
    def mg_setup(self, tv_init=None):
        """tv_init None: the library draws the starting vectors from params.seed."""
        if tv_init is None:
            return self._check(lib.mg_setup(self.h, None))
        return self._check(lib.mg_setup(self.h, _ptr(tv_init, "tv_init", self.fine_bytes(self.ntv))))

    def import_basis(self, W):
        return self._check(lib.ddamg_import_basis(self.h, _ptr(W, "W", self.fine_bytes(self.ntv))))

    def export_basis(self, W):
        return self._check(lib.ddamg_export_basis(self.h, _ptr(W, "W", self.fine_bytes(self.ntv))))

    def export_tv(self, tv):
        return self._check(lib.ddamg_export_tv(self.h, _ptr(tv, "tv", self.fine_bytes(self.ntv))))

    def export_coarse(self, Dc):
        n = self.nblocks * 9 * (2 * self.ntv) ** 2 * 16
        return self._check(lib.ddamg_export_coarse(self.h, _ptr(Dc, "Dc", n)))

    def import_tv(self, tv):
        return self._check(lib.ddamg_import_tv(self.h, _ptr(tv, "tv", self.fine_bytes(self.ntv))))

    def import_coarse(self, Dc):
        n = self.nblocks * 9 * (2 * self.ntv) ** 2 * 16
        return self._check(lib.ddamg_import_coarse(self.h, _ptr(Dc, "Dc", n)))

    def export_clover(self, A):
        return self._check(lib.ddamg_export_clover(self.h, _ptr(A, "A", self.V * 72 * 16)))

    def mg_apply(self, x, y, nrhs):
        b = self.fine_bytes(nrhs)
        return self._check(lib.mg_apply(self.h, _ptr(x, "x", b), _ptr(y, "y", b), nrhs))

    def dirac_apply(self, out, inp, nrhs, prec=FP64):
        b = self.fine_bytes(nrhs)
        return self._check(lib.dirac_apply(self.h, _ptr(out, "out", b), _ptr(inp, "in", b), nrhs, prec))

    def dirac_apply_noalloc(self, out, inp, nrhs, prec=FP64):
        b = self.fine_bytes(nrhs)
        return self._check(lib.dirac_apply_noalloc(self.h, _ptr(out, "out", b), _ptr(inp, "in", b), nrhs, prec))

    def dirac_apply_internal(self, out, inp, nrhs, prec):
        es = 16 if prec == FP64 else 8
        b = nrhs * self.V * 12 * es
        return self._check(lib.dirac_apply_internal(self.h, _ptr(out, "out", b), _ptr(inp, "in", b), nrhs, prec))

    def coarse_apply(self, out, inp, nrhs):
        b = self.coarse_bytes(nrhs)
        return self._check(lib.coarse_apply(self.h, _ptr(out, "out", b), _ptr(inp, "in", b), nrhs))

    def coarse_apply_internal(self, out, inp, nrhs):
        es = 16 if self.params.prec == FP64 else 8
        b = nrhs * self.nblocks * 2 * self.ntv * es
        return self._check(lib.coarse_apply_internal(self.h, _ptr(out, "out", b), _ptr(inp, "in", b), nrhs))

    def mg_restrict(self, yc, y, nrhs):
        return self._check(lib.mg_restrict(self.h, _ptr(yc, "yc", self.coarse_bytes(nrhs)),
                                           _ptr(y, "y", self.fine_bytes(nrhs)), nrhs))

    def mg_prolong(self, x, xc, nrhs):
        return self._check(lib.mg_prolong(self.h, _ptr(x, "x", self.fine_bytes(nrhs)),
                                          _ptr(xc, "xc", self.coarse_bytes(nrhs)), nrhs))

    def solve(self, u, f, nrhs, tol=1e-10):
        """Returns (code, stats dict); code 0 = converged, 1 = not converged."""
        st = Stats()
        b = self.fine_bytes(nrhs)
        rc = self._check(lib.solve(self.h, _ptr(u, "u", b), _ptr(f, "f", b), nrhs, tol, ctypes.byref(st)))
        return rc, st.as_dict()

    def stats(self):
        st = Stats()
        self._check(lib.ddamg_get_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        return self._check(lib.ddamg_reset_stats(self.h))

    def set_coarse_host_sync(self, each_iteration):
        """ddamg_set_coarse_host_sync: True makes the host wait for the coarse
        convergence flags after every coarse iteration (timing comparison)."""
        return self._check(lib.ddamg_set_coarse_host_sync(self.h, 1 if each_iteration else 0))

    def set_graphs(self, on):
        """ddamg_set_graphs: capture and replay each coarse GMRES iteration as
        a HIP graph (default on; contexts on the null stream stay eager)."""
        return self._check(lib.ddamg_set_graphs(self.h, 1 if on else 0))

    def set_coarse_single_kernel(self, on):
        """ddamg_set_coarse_single_kernel: the whole coarse solve in one launch
        per rhs on coarse lattices of at most 64 sites and 1.5 MiB of coarse
        operator (default on)."""
        return self._check(lib.ddamg_set_coarse_single_kernel(self.h, 1 if on else 0))

    def set_kernel_timing(self, on):
        return self._check(lib.ddamg_set_kernel_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        """{kind: (total ms, launch groups, rhs summed over them)} of the
        per-kernel-class event timers."""
        n = len(KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        rhs = (ctypes.c_int64 * n)()
        self._check(lib.ddamg_get_kernel_times(self.h, ms, cnt, rhs, n))
        return {k: (ms[i], cnt[i], rhs[i]) for i, k in enumerate(KERNEL_KINDS)}


def _batch_result(rc, ctxs, codes, t0, t1):
    out = {"rc": [int(x) for x in codes], "begin_ms": list(t0), "end_ms": list(t1)}
    if rc < 0:
        bad = next((i for i, x in enumerate(codes) if x < 0), None)
        msg = lib.ddamg_last_error(ctxs[bad].h).decode() if bad is not None else "invalid batch arguments"
        raise DDAMGError(rc, msg)
    return rc, out


def batch_setup(ctxs, workers=8):
    """ddamg_batch_setup: mg_setup(ctx, NULL) for every context, `workers`
    instances at a time.  Returns (code, {"rc", "begin_ms", "end_ms"})."""
    n = len(ctxs)
    hs = (ctypes.c_void_p * max(n, 1))(*[c.h.value for c in ctxs])
    codes = (ctypes.c_int32 * max(n, 1))()
    t0 = (ctypes.c_double * max(n, 1))()
    t1 = (ctypes.c_double * max(n, 1))()
    rc = lib.ddamg_batch_setup(hs, n, workers, codes, t0, t1)
    return _batch_result(rc, ctxs, codes[:n], t0[:n], t1[:n])


def batch_solve(ctxs, us, fs, nrhs, tol=1e-10, workers=8):
    """ddamg_batch_solve: solve(ctx[i], us[i], fs[i], nrhs[i], tol) for every
    instance, `workers` at a time.  nrhs: an int or one per instance.
    Returns (code, {"rc", "begin_ms", "end_ms"}); per-instance statistics
    come from each context's stats()."""
    n = len(ctxs)
    if isinstance(nrhs, int):
        nrhs = [nrhs] * n
    if not (len(us) == len(fs) == len(nrhs) == n):
        raise ValueError("one u, f and nrhs per context")
    hs = (ctypes.c_void_p * max(n, 1))(*[c.h.value for c in ctxs])
    up = (ctypes.c_void_p * max(n, 1))(*[_ptr(u, "u", c.fine_bytes(k)).value for u, c, k in zip(us, ctxs, nrhs)])
    fp = (ctypes.c_void_p * max(n, 1))(*[_ptr(f, "f", c.fine_bytes(k)).value for f, c, k in zip(fs, ctxs, nrhs)])
    nr = (ctypes.c_int32 * max(n, 1))(*nrhs)
    codes = (ctypes.c_int32 * max(n, 1))()
    t0 = (ctypes.c_double * max(n, 1))()
    t1 = (ctypes.c_double * max(n, 1))()
    rc = lib.ddamg_batch_solve(hs, n, up, fp, nr, tol, workers, codes, t0, t1)
    return _batch_result(rc, ctxs, codes[:n], t0[:n], t1[:n])


class Net:
    """ddamg_net: the gauge-covariant network that proposes test vectors
    (channels C_0 .. C_L, C_L = ntv), trained on the device.  Weights are a
    complex64 device tensor, the layers' [C_out][C_in][18] arrays one after
    the other."""

    def __init__(self, channels, stream=None):
        import torch
        self.channels = tuple(int(c) for c in channels)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        arr = (ctypes.c_int32 * len(self.channels))(*self.channels)
        h = ctypes.c_void_p()
        rc = lib.ddamg_net_create(arr, len(self.channels) - 1, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise DDAMGError(rc, lib.ddamg_net_last_error(None).decode())
        self.h = h
        self.nw = lib.ddamg_net_num_weights(h)

    def _check(self, rc):
        if rc < 0:
            raise DDAMGError(rc, lib.ddamg_net_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib.ddamg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        return self._check(lib.ddamg_net_set_weights(self.h, _ptr(w, "w", self.nw * 8)))

    def get_weights(self):
        import torch
        w = torch.zeros(self.nw, dtype=torch.complex64, device="cuda")
        self._check(lib.ddamg_net_get_weights(self.h, _ptr(w, "w", self.nw * 8)))
        return w

    def add_sample(self, ctx):
        idx = ctypes.c_int32()
        self._check(lib.ddamg_net_add_sample(self.h, ctx.h, ctypes.byref(idx)))
        return idx.value

    def loss_grad(self, sample, noise=None, seed=0):
        """(loss, gradient dL/dRe w + i dL/dIm w as a complex64 tensor)."""
        import torch
        g = torch.zeros(self.nw, dtype=torch.complex64, device="cuda")
        loss = ctypes.c_double()
        nz = None if noise is None else _ptr(noise, "noise")
        self._check(lib.ddamg_net_loss_grad(self.h, sample, nz, seed, ctypes.byref(loss), _ptr(g, "grad")))
        return loss.value, g

    def train_step(self, sample, seed, lr):
        loss = ctypes.c_double()
        self._check(lib.ddamg_net_train_step(self.h, sample, seed, lr, ctypes.byref(loss)))
        return loss.value

    def propose(self, ctx, out, noise=None, seed=0):
        nz = None if noise is None else _ptr(noise, "noise")
        return self._check(lib.ddamg_net_propose(self.h, ctx.h, nz, seed, _ptr(out, "out", ctx.fine_bytes(ctx.ntv))))
