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


def cpu_baseline(w):
    """Time the oracle (numpy, one thread) on a bounded sample and scale it to
    the workload: the full setup + one-rhs solve on the 8^4 lattice with the
    same parameters (smallest lattice with an even number of 4^4 blocks per
    direction), scaled by the volume ratio (setup) and by volume ratio x nrhs
    (solve; the oracle solves right-hand sides one after another)."""
    code = r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import synth
from oracle import mg
L = (8, 8, 8, 8)
U = synth.su3_field(L, %r, 301)
p = mg.Params(L, %r, %r, 1.0, %d)
M = mg.MG(p, U)
t0 = time.perf_counter()
M.setup(synth.gaussian_spinors(L, %d, 302))
t1 = time.perf_counter()
f = synth.point_sources(L)[0]
u, st = M.solve(f)
t2 = time.perf_counter()
print(json.dumps(dict(setup=t1 - t0, solve=t2 - t1, its=st["iterations"], relres=st["relres"])))
""" % (ROOT, w["eps"], tuple(w["block"]), w["m0"], w["ntv"], w["ntv"])
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    t = time.perf_counter()
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if p.returncode != 0:
        raise RuntimeError(p.stderr)
    r = json.loads(p.stdout.strip().splitlines()[-1])
    V = 1
    for x in w["L"]:
        V *= x
    scale = V / 8 ** 4
    est = r["setup"] * scale + r["solve"] * scale * w["nrhs"]
    return dict(value=est, unit="s", cores=1, kind="oracle",
                sample="oracle setup + 1-rhs solve on 8^4 (same eps/m0/csw/blocks/Ntv, %.1f s wall, %d outer its, "
                       "relres %.1e), scaled x%d volume for setup and x%d volume x %d rhs for the solve"
                       % (time.perf_counter() - t, r["its"], r["relres"], scale, scale, w["nrhs"]),
                sample_setup_s=r["setup"], sample_solve_s=r["solve"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
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
    st = mixed["stats"]
    mixed["ctx"].close()
    del mixed["ctx"], mixed["u"]
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
