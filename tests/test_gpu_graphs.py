"""Graph replay of the coarse GMRES iterations (ddamg_set_graphs) against
eager launches: contexts on a stream of their own (the null stream cannot be
captured), the same solve and V-cycle with graphs off and on.  The graphs
are captured on the first use of every (iteration index, rhs count) and
replayed in every later coarse iteration; each replayed solve, with eager
work and synchronisations of the program in between, must equal the eager
result bit for bit."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_04506_amd as dd
    return dd


def _case(dd, prec, L, block, ntv, nrhs, **kw):
    U = torch.from_numpy(synth.su3_field(L, 0.5, 811)).cuda()
    p = dd.default_params(L=L, block=block, m0=-0.2, csw=1.0, ntv=ntv, prec=prec, max_rhs=nrhs, seed=812, **kw)
    torch.cuda.synchronize()
    ctx = dd.Context(p, U, stream=torch.cuda.Stream())
    ctx.mg_setup()
    f = torch.from_numpy(synth.gaussian_spinors(L, nrhs, 813)).cuda()
    torch.cuda.synchronize()
    return ctx, f


# coarse lattices of more than 64 sites: the multi-launch coarse solve, whose
# iterations are the graphs (smaller ones run the single-kernel solve)
@pytest.mark.parametrize("prec,L,block,ntv,nrhs", [(1, (8, 8, 8, 8), (2, 2, 2, 2), 8, 1),
                                                   (2, (8, 8, 8, 16), (2, 2, 2, 2), 8, 3),
                                                   (0, (12, 12, 12, 12), (3, 3, 3, 3), 8, 2)])
def test_graph_replays_equal_eager_solve(prec, L, block, ntv, nrhs):
    dd = _gpu()
    ctx, f = _case(dd, prec, L, block, ntv, nrhs)
    ctx.set_graphs(False)
    u0 = torch.zeros_like(f)
    torch.cuda.synchronize()
    rc, st0 = ctx.solve(u0, f, nrhs, 1e-10)
    assert rc == 0
    ref = u0.cpu()
    ctx.set_graphs(True)
    for rep in range(3):
        u = torch.zeros_like(f)
        torch.cuda.synchronize()
        rc, st = ctx.solve(u, f, nrhs, 1e-10)
        # eager work of the program between the replays
        w = torch.empty_like(f)
        ctx.dirac_apply(w, u, nrhs, dd.FP64)
        torch.cuda.synchronize()
        same = torch.equal(u.cpu(), ref)
        say("prec %d %s: graph solve %d equal to eager: %s (outer its %d / %d, coarse its %d / %d)" %
            (prec, L, rep, same, st["outer_iterations"], st0["outer_iterations"], st["coarse_iterations"],
             st0["coarse_iterations"]))
        assert rc == 0 and same
    ctx.close()


def test_graph_replays_equal_eager_vcycle_fixed_iterations():
    """With a fixed coarse iteration count (no host reads at all) the V-cycle
    replayed from graphs equals the eager one, for two rhs counts in turn
    (separate graphs per count)."""
    dd = _gpu()
    ctx, f = _case(dd, 1, (8, 8, 8, 8), (2, 2, 2, 2), 8, 4, coarse_fixed_its=7, coarse_restart=3)
    outs = {}
    for on in (False, True, True):
        ctx.set_graphs(on)
        for nr in (4, 1):
            x = torch.zeros_like(f[:nr])
            torch.cuda.synchronize()
            ctx.mg_apply(x, f[:nr].contiguous(), nr)
            torch.cuda.synchronize()
            key = (nr, on)
            if key in outs:
                assert torch.equal(outs[key], x.cpu())
            outs[key] = x.cpu()
    for nr in (4, 1):
        same = torch.equal(outs[(nr, False)], outs[(nr, True)])
        say("fixed-iteration V-cycle, %d rhs: graph equal to eager: %s" % (nr, same))
        assert same
    ctx.close()


def test_graph_switch_arguments():
    dd = _gpu()
    ctx, f = _case(dd, 1, (8, 8, 8, 8), (4, 4, 4, 4), 16, 1)
    assert dd.lib.ddamg_set_graphs(ctx.h, 2) == -1
    assert dd.lib.ddamg_set_graphs(None, 1) == -1
    ctx.close()


# coarse operators within the single-kernel bound: 8^3 x 16 / 4^4 in FP64
# with N_tv = 8 (1.2 MiB), 8^4 / 4^4 in FP32 with N_tv = 16 (1.2 MiB),
# 8^3 x 16 / 4^4 with FP16 storage and N_tv = 16 (1.2 MiB)
@pytest.mark.parametrize("prec,L,ntv", [(0, (8, 8, 8, 16), 8), (1, (8, 8, 8, 8), 16), (2, (8, 8, 8, 16), 16)])
def test_single_kernel_coarse_solve_matches_multi_launch(prec, L, ntv):
    """Coarse lattices of at most 64 sites run the whole coarse solve in one
    workgroup per rhs: the V-cycle with a fixed number of coarse iterations
    (and a restart inside them) equals the multi-launch one to rounding
    (FP64 1e-12, FP32 1e-5, FP16 storage 1e-4 relative to the largest
    element), and the solve reaches 1e-10 both ways with the same number of
    outer iterations.  The per-class kernel timers show which path ran: the
    single kernel launches no coarse Gram-Schmidt."""
    dd = _gpu()
    tol = {0: 1e-12, 1: 1e-5, 2: 1e-4}[prec]
    ctx, f = _case(dd, prec, L, (4, 4, 4, 4), ntv, 3, coarse_fixed_its=9, coarse_restart=4)
    outs = {}
    for on in (True, False):
        ctx.set_coarse_single_kernel(on)
        x = torch.zeros_like(f)
        torch.cuda.synchronize()
        ctx.mg_apply(x, f, 3)
        torch.cuda.synchronize()
        outs[on] = x.cpu().numpy()
        ctx.set_kernel_timing(True)
        ctx.mg_apply(x, f, 3)
        gs_launches = ctx.kernel_times()["coarse_gs"][1]
        ctx.set_kernel_timing(False)
        assert (gs_launches == 0) == on
    d = np.abs(outs[True] - outs[False]).max() / np.abs(outs[False]).max()
    say("prec %d %s: single-kernel vs multi-launch coarse solve in the V-cycle: rel diff %.2e" % (prec, L, d))
    assert d <= tol
    ctx.close()
    ctx, f = _case(dd, prec, L, (4, 4, 4, 4), ntv, 2)
    its = {}
    for on in (True, False):
        ctx.set_coarse_single_kernel(on)
        ctx.reset_stats()
        u = torch.zeros_like(f)
        torch.cuda.synchronize()
        rc, st = ctx.solve(u, f, 2, 1e-10)
        assert rc == 0 and max(st["relres"]) <= 1e-10
        its[on] = (st["outer_iterations"], st["coarse_iterations"], st["coarse_iterations_max"])
    say("prec %d: outer / coarse its / coarse max, single kernel %s, multi-launch %s" % (prec, its[True], its[False]))
    assert its[True][0] == its[False][0]
    assert its[True][1] > 0 and its[True][2] > 0
    ctx.close()


def test_single_kernel_coarse_solve_bound():
    """A coarse operator above the byte bound (8^3 x 16 / 4^4 in FP32 with
    N_tv = 16: 2.4 MiB) keeps the multi-launch solve with the switch on."""
    dd = _gpu()
    ctx, f = _case(dd, 1, (8, 8, 8, 16), (4, 4, 4, 4), 16, 1)
    ctx.set_coarse_single_kernel(True)
    x = torch.zeros_like(f)
    ctx.set_kernel_timing(True)
    ctx.mg_apply(x, f, 1)
    assert ctx.kernel_times()["coarse_gs"][1] > 0
    ctx.set_kernel_timing(False)
    ctx.close()
