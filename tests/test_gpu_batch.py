"""Batched serving of uneven instances (ddamg_batch_setup / ddamg_batch_solve
through the C ABI): several independent lattices of the uneven-instance
recipe (8^4, 8^3 x 16, 12^4 with 2^4 blocks, 16^4; N_tv 16; FP32
preconditioner, FP64 outer), each context on a stream of its own, set up and
solved by a pool of host workers.  Every instance must get bit for bit the
basis, D_c and solution of the same instance served alone, and every
solution's residual, recomputed by the oracle's D, must be below the
tolerance."""
import sys

import numpy as np
import pytest

import synth
from oracle import dirac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_04506_amd as dd
    return dd


def _pick():
    """Two instances of every shape from the recipe (seed 11)."""
    by = {}
    for inst in synth.uneven_instances(64, 11):
        by.setdefault(inst["L"], []).append(inst)
    out = []
    for L in synth.UNEVEN_SHAPES:
        out += by[L][:2]
    return out


def _ctx(dd, inst, U):
    p = dd.default_params(L=inst["L"], block=inst["block"], m0=inst["m0"], csw=inst["csw"], ntv=inst["ntv"],
                          prec=dd.FP32, max_rhs=1, seed=inst["setup_seed"])
    Ud = dev(U)
    torch.cuda.synchronize()  # the context reads the field on a stream of its own
    return dd.Context(p, Ud, stream=torch.cuda.Stream())


@pytest.fixture(scope="module")
def batch():
    dd = _gpu()
    insts = _pick()
    say("batch: %d instances, shapes %s" % (len(insts), [i["L"] for i in insts]))
    U = [synth.su3_field(i["L"], i["eps"], i["gauge_seed"]) for i in insts]
    f = [synth.gaussian_spinors(i["L"], 1, i["rhs_seed"]) for i in insts]
    ctxs = [_ctx(dd, i, u) for i, u in zip(insts, U)]
    torch.cuda.synchronize()
    rc, info = dd.batch_setup(ctxs, workers=4)
    say("batch setup rc %d, per instance %s" % (rc, info["rc"]))
    assert rc == 0
    fd = [dev(x) for x in f]
    ud = [torch.zeros_like(x) for x in fd]
    torch.cuda.synchronize()
    rc, sinfo = dd.batch_solve(ctxs, ud, fd, 1, TOL, workers=4)
    say("batch solve rc %d, per instance %s" % (rc, sinfo["rc"]))
    assert rc == 0
    yield dd, insts, U, f, ctxs, [host(u) for u in ud], info, sinfo
    for c in ctxs:
        c.close()


def test_batch_matches_single_instance_calls(batch):
    dd, insts, U, f, ctxs, ub, info, sinfo = batch
    for k, inst in enumerate(insts):
        c = _ctx(dd, inst, U[k])
        c.mg_setup()
        nb, n = c.nblocks, 2 * inst["ntv"]
        W1 = torch.zeros((inst["ntv"],) + tuple(reversed(inst["L"])) + (4, 3), dtype=torch.complex128,
                         device="cuda")
        W2 = torch.zeros_like(W1)
        torch.cuda.synchronize()
        c.export_basis(W1)
        ctxs[k].export_basis(W2)
        D1 = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
        D2 = torch.zeros_like(D1)
        torch.cuda.synchronize()
        c.export_coarse(D1)
        ctxs[k].export_coarse(D2)
        fk = dev(f[k])
        u = torch.zeros_like(fk)
        torch.cuda.synchronize()
        rc, st = c.solve(u, fk, 1, TOL)
        assert rc == 0
        same = (np.array_equal(host(W1), host(W2)), np.array_equal(host(D1), host(D2)), np.array_equal(host(u), ub[k]))
        say("instance %d %s: basis / D_c / solution bitwise equal to the single call: %s, outer its %d" %
            (k, inst["L"], same, st["outer_iterations"]))
        assert all(same)
        c.close()


def test_batch_solutions_residual_by_oracle(batch):
    dd, insts, U, f, ctxs, ub, info, sinfo = batch
    for k, inst in enumerate(insts):
        A = dirac.clover_term(U[k], inst["m0"], inst["csw"])
        r = np.linalg.norm(f[k][0] - dirac.apply_D(U[k], A, ub[k][0])) / np.linalg.norm(f[k][0])
        st = ctxs[k].stats()
        say("instance %d %s eps %.3f m0 %.3f: oracle residual %.2e, outer its %d, solve %.1f ms in the batch" %
            (k, inst["L"], inst["eps"], inst["m0"], r, st["outer_iterations"],
             sinfo["end_ms"][k] - sinfo["begin_ms"][k]))
        assert r <= TOL


def test_batch_timings_are_consistent(batch):
    dd, insts, U, f, ctxs, ub, info, sinfo = batch
    for d in (info, sinfo):
        b, e = np.array(d["begin_ms"]), np.array(d["end_ms"])
        assert np.all(b >= 0) and np.all(e >= b)


def test_batch_serves_in_array_order(batch):
    """One worker starts the instances in array order; the solutions are bit
    for bit those of the batch above."""
    dd, insts, U, f, ctxs, ub, info, sinfo = batch
    fd = [dev(x) for x in f]
    ud = [torch.zeros_like(x) for x in fd]
    torch.cuda.synchronize()
    rc, out = dd.batch_solve(ctxs, ud, fd, 1, TOL, workers=1)
    assert rc == 0
    got = [int(i) for i in np.argsort(np.array(out["begin_ms"]), kind="stable")]
    assert got == list(range(len(insts)))
    for k in range(len(insts)):
        assert np.array_equal(host(ud[k]), ub[k])


def test_batch_concurrent_capture_and_allocation():
    """Fresh contexts served by 8 workers: while some instances capture
    their coarse iterations into graphs, others allocate and free their
    setup and Krylov buffers on other threads (HIP refuses a free during any
    capture of the process; the library keeps the two apart), and the 16
    contexts share 6 streams, as contexts drawn from a stream pool do: the
    pool never runs two instances of one stream at once (their calls do not
    overlap in time), and every instance's setup and solve succeed."""
    dd = _gpu()
    by = {}
    for inst in synth.uneven_instances(64, 23):
        by.setdefault(inst["L"], []).append(inst)
    insts = [i for L in synth.UNEVEN_SHAPES for i in by[L][:4]]
    U = [synth.su3_field(i["L"], i["eps"], i["gauge_seed"]) for i in insts]
    streams = [torch.cuda.Stream() for _ in range(6)]
    ctxs = []
    for k, (inst, u) in enumerate(zip(insts, U)):
        p = dd.default_params(L=inst["L"], block=inst["block"], m0=inst["m0"], csw=inst["csw"], ntv=inst["ntv"],
                              prec=dd.FP32, max_rhs=1, seed=inst["setup_seed"])
        Ud = dev(u)
        torch.cuda.synchronize()
        ctxs.append(dd.Context(p, Ud, stream=streams[k % 6]))
    torch.cuda.synchronize()
    say("concurrent capture: %d fresh contexts, 8 workers" % len(ctxs))
    rc, info = dd.batch_setup(ctxs, workers=8)
    assert rc == 0, info["rc"]
    fd = [dev(synth.gaussian_spinors(i["L"], 1, i["rhs_seed"])) for i in insts]
    ud = [torch.zeros_like(x) for x in fd]
    torch.cuda.synchronize()
    rc, sinfo = dd.batch_solve(ctxs, ud, fd, 1, TOL, workers=8)
    say("  setup rc %s, solve rc %s" % (info["rc"], sinfo["rc"]))
    assert rc == 0, sinfo["rc"]
    for d in (info, sinfo):
        for s0 in range(6):
            iv = sorted((d["begin_ms"][k], d["end_ms"][k]) for k in range(len(ctxs)) if k % 6 == s0)
            assert all(iv[q][1] <= iv[q + 1][0] for q in range(len(iv) - 1)), iv
    for c in ctxs:
        assert max(c.stats()["relres"][:1]) <= TOL
        c.close()


def test_batch_argument_errors(batch):
    dd, insts, U, f, ctxs, ub, info, sinfo = batch
    fd = [dev(x) for x in f[:2]]
    ud = [torch.zeros_like(x) for x in fd]
    torch.cuda.synchronize()
    with pytest.raises(dd.DDAMGError):      # the same context twice
        dd.batch_solve([ctxs[0], ctxs[0]], ud, [fd[0], fd[0]], 1, TOL)
    with pytest.raises(dd.DDAMGError):      # no workers
        dd.batch_solve(ctxs[:2], ud, fd, 1, TOL, workers=0)
    with pytest.raises(dd.DDAMGError):      # u == f
        dd.batch_solve(ctxs[:2], [fd[0], ud[1]], fd, 1, TOL)
    rc, out = dd.batch_solve([], [], [], [], TOL)
    assert rc == 0 and out["rc"] == []
