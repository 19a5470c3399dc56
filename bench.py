"""Benchmark: time-to-solution of the two-level DD-alpha-AMG solve on one
MI355X, mixed precision vs the plain FP64 path, plus the HBM roofline of the
Wilson-clover dslash and the coarse stencil D_c.

One step = the whole hot path on one batch: the adaptive setup (Alg. 4/5,
24 test vectors) and the FGMRES(20) solve of the 12 point-source right-hand
sides of the 32^3 x 64 workload (eps 0.5, m0 -0.2, c_sw 1, 4^4 blocks) to
relative residual 1e-10, all inputs resident in HBM before the timed region.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1] [--workload c3|c2|c1]

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: L (x, y, z, t), block, eps, m0, ntv, nrhs, rhs kind, seeds (gauge, tv)
    "c3": dict(L=(32, 32, 32, 64), block=(4, 4, 4, 4), eps=0.5, m0=-0.2, ntv=24, nrhs=12, rhs="point",
               seeds=(301, 302), name="32^3x64 eps0.5 m0-0.2 csw1 blocks4^4 Ntv24 12 point sources"),
    "c2": dict(L=(16, 16, 16, 16), block=(4, 4, 4, 4), eps=0.5, m0=-0.2, ntv=20, nrhs=8, rhs="gauss",
               seeds=(201, 202), name="16^4 eps0.5 m0-0.2 csw1 blocks4^4 Ntv20 8 gaussian rhs"),
    "c1": dict(L=(4, 4, 4, 4), block=(2, 2, 2, 2), eps=0.3, m0=-0.1, ntv=8, nrhs=1, rhs="gauss",
               seeds=(101, 102), name="4^4 eps0.3 m0-0.1 csw1 blocks2^4 Ntv8 1 gaussian rhs"),
}
# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counter runs calibrated on a stream kernel of known size; the
# record names the sources it was taken from and is ignored once they change
TRAFFIC_RECORDS = os.path.join(ROOT, "profiles", "hbm_traffic_32x32x32x64.txt")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (counts packed dual FP32 issue)
FP32_UNPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz: the library is built without packed FP32
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(w):
    import numpy as np
    import synth
    L = w["L"]
    U = synth.su3_field(L, w["eps"], w["seeds"][0])
    tv = synth.gaussian_spinors(L, w["ntv"], w["seeds"][1])
    if w["rhs"] == "point":
        f = synth.point_sources(L)[: w["nrhs"]]
    else:
        f = synth.gaussian_spinors(L, w["nrhs"], 203)
    return U, np.ascontiguousarray(tv), np.ascontiguousarray(f)


def run_path(dd, torch, w, prec, U_d, tv_d, f_d, steps, warmup):
    p = dd.default_params(L=w["L"], block=w["block"], m0=w["m0"], csw=1.0, ntv=w["ntv"], prec=prec,
                          max_rhs=max(w["nrhs"], 1), outer_restart=20)
    ctx = dd.Context(p, U_d)
    nrhs = w["nrhs"]
    u = torch.zeros_like(f_d)
    res = {"setup_ms": [], "solve_ms": [], "step_ms": []}
    st = None
    for it in range(warmup + steps):
        if it == warmup:
            ctx.set_kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mg_setup(tv_d)
        t1 = time.perf_counter()
        u.zero_()
        ctx.reset_stats()
        rc, st = ctx.solve(u, f_d, nrhs, 1e-10)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rc != 0:
            raise RuntimeError("solve did not converge: %s" % st)
        if it >= warmup:
            res["setup_ms"].append((t1 - t0) * 1e3)
            res["solve_ms"].append((t2 - t1) * 1e3)
            res["step_ms"].append((t2 - t0) * 1e3)
        log("  prec %d step %d: setup %.1f ms solve %.1f ms outer its %d coarse its max %d" %
            (prec, it, (t1 - t0) * 1e3, (t2 - t1) * 1e3, st["outer_iterations"], st["coarse_iterations_max"]))
    res["kernel_times"] = ctx.kernel_times()
    ctx.set_kernel_timing(False)
    res["stats"] = st
    res["ctx"] = ctx
    res["u"] = u
    return res


def time_kernel(torch, fn, reps):
    """Average duration of one launch of fn (a single kernel on torch's
    current stream) measured with HIP events around reps launches."""
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_rooflines(dd, torch, ctx, w, reps=50):
    V = 1
    for x in w["L"]:
        V *= x
    nb = ctx.nblocks
    nc = 2 * w["ntv"]
    out = {}
    # dslash, FP16 links/clover + per-site FP32 scales, FP32 spinors, 1 rhs
    a = torch.randn(12 * V * 2, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = time_kernel(torch, lambda: ctx.dirac_apply_internal(b, a, 1, dd.MIXED16), reps)
    bytes_site = 96 + 96 + (36 * 4 + 4) + (72 * 2 + 4)
    out["dslash_mixed16"] = dict(ms=ms, bytes=bytes_site * V, gbs=bytes_site * V / ms / 1e6)
    a64 = torch.randn(12 * V * 2, dtype=torch.float64, device="cuda")
    b64 = torch.empty_like(a64)
    ms = time_kernel(torch, lambda: ctx.dirac_apply_internal(b64, a64, 1, dd.FP64), reps)
    bytes_site = 192 + 192 + 576 + 576
    out["dslash_fp64"] = dict(ms=ms, bytes=bytes_site * V, gbs=bytes_site * V / ms / 1e6)
    # stream kernel dst = 1 * src over 2 GiB: the HBM rate this machine reaches,
    # and the known-size reference for the traffic counters
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = time_kernel(torch, lambda: torch.mul(src, 1.0, out=dst), 10)
    out["stream_2GiB"] = dict(ms=ms, bytes=2 << 31, gbs=(2 << 31) / ms / 1e6)
    del src, dst
    # coarse stencil (FP16 D_c + per-(site, slot) scale, FP32 vectors)
    for nr in (1, w["nrhs"]):
        x = torch.randn(nr * nb * nc * 2, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        ms = time_kernel(torch, lambda: ctx.coarse_apply_internal(y, x, nr), reps)
        by = nb * (9 * nc * nc * 4 + 9 * 4 + nr * 2 * nc * 8)
        out["coarse_mixed16_%drhs" % nr] = dict(ms=ms, bytes=by, gbs=by / ms / 1e6)
    return out


def coarse_iteration_cost(dd, torch, w, U_d, tv_d, f_d, its=(5, 30), reps=5):
    """Wall-clock cost of one coarse GMRES iteration (Alg. 2) inside the
    V-cycle at the workload, in deterministic mode (a fixed number of coarse
    iterations, no tolerance test): (T(its[1]) - T(its[0])) / (its[1] -
    its[0]) for V-cycles of all rhs, with the host reading the convergence
    flags after every iteration ("sync_each", the device idles meanwhile)
    and with the pipelined test ("pipelined": nothing read with a fixed
    count).  Also the device time of the coarse kernels per iteration."""
    nrhs = w["nrhs"]
    out = {"coarse_fixed_its": list(its), "nrhs": nrhs}
    times = {}
    for n_its in its:
        p = dd.default_params(L=w["L"], block=w["block"], m0=w["m0"], csw=1.0, ntv=w["ntv"], prec=dd.MIXED16,
                              max_rhs=nrhs, coarse_fixed_its=n_its, coarse_restart=max(its))
        ctx = dd.Context(p, U_d)
        ctx.mg_setup(tv_d)
        x = torch.zeros_like(f_d)
        for mode in ("sync_each", "pipelined"):
            ctx.set_coarse_host_sync(mode == "sync_each")
            ctx.mg_apply(x, f_d, nrhs)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                ctx.mg_apply(x, f_d, nrhs)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            times[(mode, n_its)] = sorted(ts)[len(ts) // 2]
        ctx.set_coarse_host_sync(False)
        ctx.set_kernel_timing(True)
        ctx.mg_apply(x, f_d, nrhs)
        kt = ctx.kernel_times()
        ctx.set_kernel_timing(False)
        if n_its == its[1]:
            out["device_ms_per_iteration_at_%d" % n_its] = (kt["coarse"][0] + kt["coarse_gs"][0]) / n_its
        ctx.close()
        del x
        torch.cuda.empty_cache()
    d = its[1] - its[0]
    for mode in ("sync_each", "pipelined"):
        out["ms_per_iteration_" + mode] = (times[(mode, its[1])] - times[(mode, its[0])]) / d
        out["vcycle_ms_%s_%d_its" % (mode, its[1])] = times[(mode, its[1])]
    return out


def _field_worker(a):
    import synth
    L, eps, seed = a
    return synth.su3_field(L, eps, seed)


def generated_fields(L, eps, seeds, workers):
    """Seeded gauge fields drawn on the host in a process pool (children
    started fresh: they import only numpy and the input generators)."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_field_worker, [(L, eps, s) for s in seeds])


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=float), q))


def batched_serving(dd, torch, n=64, seed=401, workers=(1, 2, 4, 8, 16), field_workers=16, setup_workers=8):
    """Batched serving of uneven instances: n independent lattices of the
    uneven-instance recipe (8^4, 8^3 x 16, 12^4 with 2^4 blocks, 16^4; N_tv
    16; FP32 preconditioner, FP64 outer; one Gaussian rhs each), every
    context on a stream of its own.  Setup of all instances by the worker
    pool, then the n solves served with 1, 2, 4, ... workers; the worker
    count with the highest throughput is the one reported (a one-parameter
    tuner of the concurrency).  Latency of a solve = its own call time
    (service); completion = from the start of the batch to its return."""
    import synth
    insts = synth.uneven_instances(n, seed)
    t0 = time.perf_counter()
    U = generated_fields_for([(i["L"], i["eps"], i["gauge_seed"]) for i in insts], field_workers)
    f = [synth.gaussian_spinors(i["L"], 1, i["rhs_seed"]) for i in insts]
    gen_s = time.perf_counter() - t0
    ctxs, fd, ud = [], [], []
    for i, u, ff in zip(insts, U, f):
        p = dd.default_params(L=i["L"], block=i["block"], m0=i["m0"], csw=i["csw"], ntv=i["ntv"], prec=dd.FP32,
                              max_rhs=1, seed=i["setup_seed"])
        Ud = torch.from_numpy(u).cuda()
        torch.cuda.synchronize()
        ctxs.append(dd.Context(p, Ud, stream=torch.cuda.Stream()))
        del Ud
        fd.append(torch.from_numpy(ff).cuda())
        ud.append(torch.zeros_like(fd[-1]))
    del U
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, sinfo = dd.batch_setup(ctxs, workers=setup_workers)
    setup_ms = (time.perf_counter() - t0) * 1e3
    if rc != 0:
        raise RuntimeError("batched setup: rc %d %s" % (rc, sinfo["rc"]))
    runs = {}
    ref = None
    for wk in workers:
        for x in ud:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = dd.batch_solve(ctxs, ud, fd, 1, 1e-10, workers=wk)
        span = (time.perf_counter() - t0) * 1e3
        if rc != 0:
            raise RuntimeError("batched solve: rc %d %s" % (rc, info["rc"]))
        sols = [x.cpu() for x in ud]
        same = None
        if ref is None:
            ref = sols
        else:
            same = all(torch.equal(a, b) for a, b in zip(ref, sols))
        svc = [e - b for b, e in zip(info["begin_ms"], info["end_ms"])]
        runs[wk] = {"makespan_ms": span, "solves_per_s": n / span * 1e3,
                    "latency_ms_p50": _pct(svc, 50), "latency_ms_p99": _pct(svc, 99),
                    "completion_ms_p50": _pct(info["end_ms"], 50), "completion_ms_p99": _pct(info["end_ms"], 99),
                    "solutions_equal_to_1_worker": same}
        log("batched serving, %d workers: %s" % (wk, json.dumps(runs[wk])))
    its = [c.stats()["outer_iterations"] for c in ctxs]
    relres = max(c.stats()["relres"][0] for c in ctxs)
    for c in ctxs:
        c.close()
    best = max(runs, key=lambda k: runs[k]["solves_per_s"])
    shapes = {}
    for i in insts:
        k = "x".join(str(x) for x in i["L"])
        shapes[k] = shapes.get(k, 0) + 1
    return {"instances": n, "seed": seed, "shapes": shapes, "ntv": 16, "prec": "FP32 preconditioner, FP64 outer",
            "nrhs_per_instance": 1, "tol": 1e-10, "input_generation_s": gen_s, "setup_workers": setup_workers,
            "setup_makespan_ms": setup_ms,
            "outer_iterations_min_max": [min(its), max(its)], "relres_max": relres,
            "by_workers": {str(k): v for k, v in runs.items()}, "best_workers": best,
            "speedup_best_vs_1_worker": runs[best]["solves_per_s"] / runs[1]["solves_per_s"] if 1 in runs else None}


def generated_fields_for(specs, workers):
    """Seeded gauge fields for (L, eps, seed) triples, in a process pool."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_field_worker, specs)


def _gamma5(torch, X):
    """gamma5 = diag(-1, -1, 1, 1) on the spin index of canonical fields."""
    Y = X.clone(memory_format=torch.contiguous_format)
    Y[..., :2, :] *= -1
    return Y


def _orthonormal_rows(torch, X):
    """The fields X[i] made orthonormal (Cholesky QR, twice)."""
    n = X.shape[0]
    M = X.reshape(n, -1)
    for _ in range(2):
        G = torch.matmul(M, M.conj().transpose(0, 1))  # G_ij = <M_j, M_i> = L L^H
        L = torch.linalg.cholesky(G)
        M = torch.linalg.solve_triangular(L, M, upper=False)
    return M.contiguous().reshape(X.shape)


def low_modes(dd, torch, w, U_d, nmodes=20, iters=6, seed=11):
    """nmodes vectors spanning (approximately) the right singular vectors of
    D with the smallest singular values on the workload's field: block
    inverse iteration on D^dag D, (D^dag D)^-1 = D^-1 g5 D^-1 g5 (D^dag =
    g5 D g5), each D^-1 a solve of all nmodes rhs to 1e-8 by the library
    (its own plain setup, FGMRES(8) to bound the Krylov basis), then
    Rayleigh-Ritz with D in FP64.  Returns the Ritz vectors (device,
    canonical) and their singular-value estimates |D v|."""
    p = dd.default_params(L=w["L"], block=w["block"], m0=w["m0"], csw=1.0, ntv=w["ntv"], prec=dd.MIXED16,
                          max_rhs=nmodes, outer_restart=8, seed=302)
    ctx = dd.Context(p, U_d)
    ctx.mg_setup()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    shape = (nmodes,) + tuple(reversed(w["L"])) + (4, 3)
    V = torch.randn(shape, dtype=torch.complex128, device="cuda", generator=gen)
    for _ in range(iters):
        V = _orthonormal_rows(torch, V)
        Y = torch.zeros(shape, dtype=torch.complex128, device="cuda")
        ctx.solve(Y, _gamma5(torch, V), nmodes, 1e-8)
        X = _gamma5(torch, Y)
        del Y
        V = torch.zeros(shape, dtype=torch.complex128, device="cuda")
        ctx.solve(V, X, nmodes, 1e-8)
        del X
    V = _orthonormal_rows(torch, V)
    W = torch.empty(shape, dtype=torch.complex128, device="cuda")
    ctx.dirac_apply(W, V, nmodes, dd.FP64)
    Wm = W.reshape(nmodes, -1)
    H = torch.matmul(Wm.conj(), Wm.transpose(0, 1))
    del W, Wm
    ev, Q = torch.linalg.eigh(H)
    V = torch.matmul(Q.transpose(0, 1), V.reshape(nmodes, -1)).contiguous().reshape(shape)
    ctx.close()
    return V, [float(x) for x in torch.sqrt(ev.clamp(min=0)).cpu()]


def low_mode_capture(torch, ctx, V):
    """|(1 - P R) v| for every (normalised) low mode v: how much of the
    near-null space the setup's aggregates miss."""
    n = V.shape[0]
    yc = torch.empty((ctx.coarse_bytes(n) // 16,), dtype=torch.complex128, device="cuda")
    X = torch.empty(V.shape, dtype=torch.complex128, device="cuda")
    ctx.mg_restrict(yc, V, n)
    ctx.mg_prolong(X, yc, n)
    d = (V - X).reshape(n, -1).norm(dim=1) / V.reshape(n, -1).norm(dim=1)
    return [float(x) for x in d.cpu()]


def learned_eval(dd, torch, w, args):
    """The learned test-vector proposal: train the network on the aggregate
    bases of plain setups on generated 16^4 fields (eps 0.5, m0 -0.2, 4^4
    blocks, N_tv of the workload), then on the workload compare setups:
    plain (Alg. 4: three smoother passes, n_setup V-cycle passes), learned
    (the network's proposal, no smoother passes, fewer V-cycle passes) and
    the same short setup from random vectors (what the network adds)."""
    import numpy as np
    from paper_1512_04506_amd import learned_setup as ls
    ntv = w["ntv"]
    Lt = (16, 16, 16, 16)
    t0 = time.perf_counter()
    nf = args.train_fields
    fields = generated_fields(Lt, 0.5, [700 + k for k in range(nf + 1)], 16)
    log("learned: %d training fields and one held-out field generated in %.1f s" % (nf, time.perf_counter() - t0))
    net = dd.Net(ls.channels_for(ntv))
    net.set_weights(torch.from_numpy(ls.smoother_init(ls.channels_for(ntv), 0.1, 0.01, 7)).cuda())
    pt = dd.default_params(L=Lt, block=(4, 4, 4, 4), m0=-0.2, csw=1.0, ntv=ntv, prec=dd.MIXED16, max_rhs=ntv)
    samples = []
    for k in range(nf + 1):
        Ud = torch.from_numpy(fields[k]).cuda()
        s, _ = ls.training_samples(net, [Ud], pt, seed0=1000 + k)
        samples += s
        del Ud
    del fields
    held_out = samples.pop()
    loss0, _ = net.loss_grad(held_out, seed=4242)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ls.train(net, samples, args.train_epochs, args.train_lr, decay=0.5,
                    decay_every=max(1, args.train_epochs // 3), log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loss1, _ = net.loss_grad(held_out, seed=4242)
    log("learned: held-out span loss %.4f untrained, %.4f trained" % (loss0, loss1))
    res = {"train_fields": nf, "epochs": args.train_epochs, "lr": args.train_lr, "train_s": train_s,
           "held_out_span_loss": {"untrained": loss0, "trained": loss1},
           "steps": nf * args.train_epochs, "ms_per_step": train_s * 1e3 / (nf * args.train_epochs),
           "loss_per_epoch": hist, "channels": list(ls.channels_for(ntv)), "weights": int(net.nw)}
    # the workload: plain against learned and random short setups
    U, tv, f = make_inputs(w)
    U_d = torch.from_numpy(U).cuda()
    f_d = torch.from_numpy(f).cuda()
    del U, tv
    nrhs = w["nrhs"]
    rows = []
    modes = None
    if args.low_modes > 0:
        t0 = time.perf_counter()
        modes, sig = low_modes(dd, torch, w, U_d, nmodes=args.low_modes)
        res["low_modes"] = {"n": args.low_modes, "method": "6 steps of block inverse iteration on D^dag D, "
                            "Rayleigh-Ritz", "singular_values": sig, "s": time.perf_counter() - t0}
        log("learned: %d low modes, singular values %.3g .. %.3g" % (args.low_modes, sig[0], sig[-1]))
        torch.cuda.empty_cache()
    for name, init_passes, n_setup, start in [("plain", 3, 3, "random"), ("learned", 0, 0, "net"),
                                              ("random_short", 0, 0, "random"), ("learned", 0, 1, "net"),
                                              ("random_short", 0, 1, "random"), ("plain_short", 1, 0, "random")]:
        p = dd.default_params(L=w["L"], block=w["block"], m0=w["m0"], csw=1.0, ntv=ntv, prec=dd.MIXED16,
                              max_rhs=max(nrhs, ntv), init_passes=init_passes, n_setup=n_setup, seed=302)
        ctx = dd.Context(p, U_d)
        setups = []
        for rep_ in range(3):
            if start == "net":
                prop_ms, set_ms = ls.propose_setup(net, ctx, seed=5000 + rep_)
            else:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.mg_setup()
                torch.cuda.synchronize()
                prop_ms, set_ms = 0.0, (time.perf_counter() - t0) * 1e3
            setups.append((prop_ms, set_ms))
        u = torch.zeros_like(f_d)
        r = {"setup": name, "init_passes": init_passes, "n_setup": n_setup,
             "proposal_ms": min(x[0] for x in setups), "setup_ms": min(x[1] for x in setups)}
        if modes is not None:
            cap = low_mode_capture(torch, ctx, modes)
            r["low_mode_residual"] = {"mean": float(np.mean(cap)), "max": max(cap), "lowest5_mean": float(np.mean(cap[:5]))}
        try:
            solve_ms = []
            for _ in range(2):  # the first solve of a context also grows its Krylov basis
                u.zero_()
                rc, st = ctx.solve(u, f_d, nrhs, 1e-10)
                solve_ms.append(st["solve_ms"])
            r.update(outer_iterations=st["outer_iterations"], solve_ms=min(solve_ms), converged=rc == 0)
        except dd.DDAMGError as e:  # a setup too poor for the outer solve: it diverges
            r.update(outer_iterations=None, solve_ms=None, converged=False, error=str(e)[:120])
        r["setup_total_ms"] = r["proposal_ms"] + r["setup_ms"]
        rows.append(r)
        log("learned eval:", json.dumps(r))
        ctx.close()
        del u
        torch.cuda.empty_cache()
    res["workload"] = w["name"]
    res["setups"] = rows
    net.close()
    return res


def sap_flops_per_site(block, n_mr):
    """Algorithmic flops of one SAP colour phase per site of that colour and
    rhs: residual y - D x (1320 hop + 504 clover + 24), n_mr MR steps each
    with B rho (clover 504 + the in-block share of the 1320 hop flops) and
    two inner products and two axpys (336), and the update x += e (24)."""
    inblock = sum((b - 1) / b for b in block) / 4.0
    return 1320 + 504 + 24 + n_mr * (504 + 1320 * inblock + 336) + 24


def dominant_roofline(w, kt, prec):
    """Roofline record of the kernel class with the largest total time in
    the timed steps, from the library's per-launch HIP events.  Algorithmic
    work per class (each datum counted once per launch):
      sap      flops: rhs x V/2 x sap_flops_per_site      (FP32 ALU bound)
      dslash   bytes: launches x V x 1152 (FP64 links + clover)
                      + rhs x V x (12 x 8 in + 12 x 16 out)  (HBM bound)
      restrict / prolong bytes: launches x V x ntv x (12 x w + s)
                      + rhs x V x 12 x 8   (w = 4, s = 4 for FP16 + scale)
    Other classes are reported in kernel_times only."""
    V = 1
    for x in w["L"]:
        V *= x
    ntv = w["ntv"]
    sb = 8 if prec != 0 else 16
    wb, ws = (4, 4) if prec == 2 else ((8, 0) if prec == 1 else (16, 0))
    cand = {}
    for kind, (ms, cnt, rhs) in kt.items():
        if cnt == 0 or ms <= 0:
            continue
        if kind == "sap":
            work = rhs * (V / 2) * sap_flops_per_site(w["block"], 4)
            cand[kind] = dict(bound="alu", achieved=work / (ms * 1e-3) / 1e12,
                              peak=FP32_PEAK_TFLOPS if prec != 0 else FP64_PEAK_TFLOPS, unit="TFLOP/s",
                              per_launch=work / cnt, ms=ms, launches=cnt)
        elif kind == "dslash":
            work = cnt * V * 1152 + rhs * V * (12 * sb + 192)
            cand[kind] = dict(bound="hbm", achieved=work / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                              per_launch=work / cnt, ms=ms, launches=cnt)
        elif kind in ("restrict", "prolong"):
            work = cnt * V * ntv * (12 * wb + ws) + rhs * V * 12 * sb
            cand[kind] = dict(bound="hbm", achieved=work / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                              per_launch=work / cnt, ms=ms, launches=cnt)
    kind = max(cand, key=lambda k: cand[k]["ms"])
    r = cand[kind]
    out = {"bound": r["bound"], "kernel": kind, "achieved": r["achieved"], "peak": r["peak"], "unit": r["unit"],
           "frac": r["achieved"] / r["peak"], "traffic": None,
           "avg_launch_ms": r["ms"] / r["launches"], "launches": r["launches"],
           "algorithmic_per_launch": r["per_launch"]}
    if kind == "sap" and prec != 0:
        out["peak_unpacked"] = FP32_UNPACKED_TFLOPS
        out["frac_unpacked"] = r["achieved"] / FP32_UNPACKED_TFLOPS
    return out


def sources_digest(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1512_04506_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kind, workload):
    """HBM bytes per launch of kernel class `kind` on `workload`, or None if
    no counter record exists for the sources as they are now."""
    try:
        with open(TRAFFIC_RECORDS) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    for line in lines:
        if not line.startswith("record: "):
            continue
        r = json.loads(line[len("record: "):])
        if r["class"] == kind and r["workload"] == workload and r["sources_sha256"] == sources_digest(r["sources"]):
            return r["bytes_per_launch"]
    return None


def _host_cpu():
    """(cores this process may use, CPU model name)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


_ORACLE_CHILD = r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import multiprocessing as mp
import synth
from oracle import mg, dirac

def solve_one(args):
    M, f = args
    t = time.perf_counter()
    u, st = M.solve(f)
    return time.perf_counter() - t, st["iterations"], mg.true_relres(M.D, u, f)

def run(L, block, eps, m0, ntv, seeds, rhs, nrhs, workers):
    U = synth.su3_field(L, eps, seeds[0])
    p = mg.Params(L, block, m0, 1.0, ntv)
    M = mg.MG(p, U)
    t0 = time.perf_counter()
    M.setup(synth.gaussian_spinors(L, ntv, seeds[1]))
    t1 = time.perf_counter()
    f = synth.point_sources(L)[:nrhs] if rhs == "point" else synth.gaussian_spinors(L, nrhs, 103)
    with mp.get_context("fork").Pool(min(workers, nrhs)) as pool:
        out = pool.map(solve_one, [(M, f[r]) for r in range(nrhs)])
    t2 = time.perf_counter()
    return dict(setup_s=t1 - t0, solve_s=t2 - t1, solve_cpu_s=sum(o[0] for o in out),
                outer_its=[o[1] for o in out], relres_max=max(o[2] for o in out))

if __name__ == "__main__":
    cfg = json.loads(sys.argv[1])
    print(json.dumps(run(**cfg)))
"""


def _oracle_run(cfg, cores, timeout):
    """One oracle run in a fresh interpreter (no GPU in it): the setup in
    one process (the oracle's setup is serial; numpy on more BLAS threads
    made it slower: 201 s against 81 s on 8 threads for the 8^4 sample),
    the right-hand sides solved in a process pool of min(cores, nrhs)
    workers, every process on one BLAS thread."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = _ORACLE_CHILD % ROOT
    p = subprocess.run([sys.executable, "-c", code, json.dumps(cfg)], capture_output=True, text=True, env=env,
                       timeout=timeout)
    if p.returncode != 0:
        raise RuntimeError(p.stderr[-500:])
    return json.loads(p.stdout.strip().splitlines()[-1])


def cpu_baseline(w):
    """The oracle (numpy, FP64) timed on this host's cores: the 4^4
    workload measured in full (setup + solve), and the same parameters as
    the workload on the 8^4 lattice (the smallest with an even number of
    4^4 blocks per direction: setup + all rhs), which is scaled by the
    volume ratio to the workload (an extrapolation, stated as such)."""
    cores, model = _host_cpu()
    t = time.perf_counter()
    c1 = WORKLOADS["c1"]
    m1 = _oracle_run(dict(L=c1["L"], block=c1["block"], eps=c1["eps"], m0=c1["m0"], ntv=c1["ntv"],
                          seeds=c1["seeds"], rhs=c1["rhs"], nrhs=c1["nrhs"], workers=cores), cores, 600)
    ms = _oracle_run(dict(L=(8, 8, 8, 8), block=w["block"], eps=w["eps"], m0=w["m0"], ntv=w["ntv"],
                          seeds=w["seeds"], rhs=w["rhs"], nrhs=w["nrhs"], workers=cores), cores, 900)
    V = 1
    for x in w["L"]:
        V *= x
    scale = V / 8 ** 4
    est = (ms["setup_s"] + ms["solve_s"]) * scale
    return dict(value=est, unit="s", cores=min(cores, w["nrhs"]), host_cores=cores, cpu_model=model, kind="oracle",
                cores_note="setup on 1 core (the oracle's setup is serial), rhs on a pool of min(cores, nrhs)",
                sample="8^4 lattice with the workload's eps/m0/csw/blocks/Ntv: setup %.1f s (1 core) + %d rhs %.1f s "
                       "(%d processes) measured, scaled x%d by volume to the workload (extrapolated); 4^4 workload "
                       "measured in full: setup %.2f s + solve %.2f s; %.0f s wall in all"
                       % (ms["setup_s"], w["nrhs"], ms["solve_s"], min(cores, w["nrhs"]), scale, m1["setup_s"],
                          m1["solve_s"], time.perf_counter() - t),
                measured={"c1_4x4x4x4": m1, "sample_8x8x8x8": ms}, extrapolated_to=w["name"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-coarse-cost", action="store_true")
    ap.add_argument("--batched-only", type=int, default=0, metavar="WORKERS",
                    help="serve only the 64 uneven instances with this many workers and print their JSON (for "
                         "profiling the small-instance path); no step is timed")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched serving of 64 uneven instances")
    ap.add_argument("--learned", action="store_true",
                    help="train the test-vector network and compare learned and plain setups (prints its own line)")
    ap.add_argument("--train-fields", type=int, default=256)
    ap.add_argument("--train-epochs", type=int, default=12)
    ap.add_argument("--train-lr", type=float, default=2e-3)
    ap.add_argument("--low-modes", type=int, default=20,
                    help="low modes of D for the |(1-PR)v| comparison of --learned (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a multi-GPU run would split "
              "the lattice along t, with halo exchanges and all-reduced inner products). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1512_04506_amd as dd
    w = WORKLOADS[args.workload]
    log("workload", w["name"])
    if args.learned:
        print(json.dumps({"learned_setup": learned_eval(dd, torch, w, args)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_uneven": batched_serving(dd, torch, workers=(args.batched_only,),
                                                            setup_workers=args.batched_only)}), flush=True)
        return
    t = time.perf_counter()
    U, tv, f = make_inputs(w)
    log("inputs generated in %.1f s" % (time.perf_counter() - t))
    U_d = torch.from_numpy(U).cuda()
    tv_d = torch.from_numpy(tv).cuda()
    f_d = torch.from_numpy(f).cuda()
    del U, tv
    mixed = run_path(dd, torch, w, dd.MIXED16, U_d, tv_d, f_d, args.steps, args.warmup)
    roof = kernel_rooflines(dd, torch, mixed["ctx"], w)
    log("kernels:", json.dumps(roof))
    # the solve with the host reading the coarse convergence flags after
    # every coarse iteration, against the pipelined test (tolerance mode)
    solve_sync = {}
    for mode in ("sync_each", "pipelined"):
        mixed["ctx"].set_coarse_host_sync(mode == "sync_each")
        ts = []
        for _ in range(2):
            mixed["u"].zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mixed["ctx"].solve(mixed["u"], f_d, w["nrhs"], 1e-10)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        solve_sync[mode] = min(ts)
    mixed["ctx"].set_coarse_host_sync(False)
    log("solve ms by coarse convergence test:", json.dumps(solve_sync))
    st = mixed["stats"]
    mixed["ctx"].close()
    del mixed["ctx"], mixed["u"]
    torch.cuda.empty_cache()
    coarse_cost = None
    if not args.no_coarse_cost:
        coarse_cost = coarse_iteration_cost(dd, torch, w, U_d, tv_d, f_d)
        coarse_cost["solve_ms_sync_each"] = solve_sync["sync_each"]
        coarse_cost["solve_ms_pipelined"] = solve_sync["pipelined"]
        log("coarse iteration cost:", json.dumps(coarse_cost))
    batched = None
    if not args.no_batched:
        try:
            batched = batched_serving(dd, torch)
        except Exception as e:  # reported, the workload's figures stand on their own
            batched = {"error": str(e)[:300]}
        torch.cuda.empty_cache()
    fp64 = None
    if not args.no_fp64:
        fp64 = run_path(dd, torch, w, dd.FP64, U_d, tv_d, f_d, max(1, args.steps // 2), args.warmup)
        fp64["ctx"].close()
        del fp64["ctx"], fp64["u"]
        torch.cuda.empty_cache()
    ms = sum(mixed["step_ms"]) / len(mixed["step_ms"])
    line = {
        "metric": "time-to-solution (rel.res 1e-10) 32^3x64, mixed vs FP64; dslash/D_c HBM GB/s",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (fp16 storage), f64 outer",
        "data": "synthetic seeded SU(3) field and point sources",
        "config": {"workload": w["name"], "nrhs": w["nrhs"], "outer": "FGMRES(20)", "tol": 1e-10},
        "setup_ms": sum(mixed["setup_ms"]) / len(mixed["setup_ms"]),
        "solve_ms": sum(mixed["solve_ms"]) / len(mixed["solve_ms"]),
        "outer_iterations": st["outer_iterations"],
        "coarse_iterations_max": st["coarse_iterations_max"],
        "relres_max": max(st["relres"]),
        "kernel_times_ms": {k: round(v[0] / args.steps, 3) for k, v in mixed["kernel_times"].items()},
        "kernels_isolated": roof,
        "roofline": dominant_roofline(w, mixed["kernel_times"], dd.MIXED16),
        "coarse_iteration_cost": coarse_cost,
        "batched_uneven": batched,
    }
    line["roofline"]["traffic"] = measured_traffic(line["roofline"]["kernel"], w["name"])
    if fp64:
        f64ms = sum(fp64["step_ms"]) / len(fp64["step_ms"])
        line["fp64"] = {"ms_per_step": f64ms, "setup_ms": sum(fp64["setup_ms"]) / len(fp64["setup_ms"]),
                        "solve_ms": sum(fp64["solve_ms"]) / len(fp64["solve_ms"]),
                        "outer_iterations": fp64["stats"]["outer_iterations"],
                        "kernel_times_ms": {k: round(v[0] / max(1, args.steps // 2), 3)
                                            for k, v in fp64["kernel_times"].items()}}
        line["speedup_mixed_vs_fp64"] = f64ms / ms
    if not args.no_cpu:
        try:
            line["cpu_baseline"] = cpu_baseline(w)
        except Exception as e:  # the GPU figures stand on their own
            line["cpu_baseline"] = {"error": str(e)[:200]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
