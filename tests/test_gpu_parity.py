"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances (relative, max-norm over the whole output unless stated):
operator applies 1e-12 in FP64, 1e-5 in FP32, 1e-2 with 16-bit storage;
composite V-cycle in deterministic mode (fixed coarse iterations) 1e-10 in
FP64; every solution reaches ||f - D u|| / ||f|| <= 1e-10 recomputed by the
oracle's own D.  Lattices are chosen to span several 256-thread tiles with
a ragged tail (V not a multiple of 256, block volumes not multiples of 64).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import dirac, sap, coarse, mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_04506_amd as dd
    return dd


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {
    # name: L, block, eps, m0, ntv
    "c1_4x4x4x4": ((4, 4, 4, 4), (2, 2, 2, 2), 0.3, -0.1, 8),
    "ragged_6x4x4x4": ((6, 4, 4, 4), (3, 2, 2, 2), 0.5, -0.2, 6),
    "tiles_8x8x4x8": ((8, 8, 4, 8), (4, 4, 2, 4), 0.5, -0.2, 12),
}
TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2}


def make_ctx(dd, L, block, eps, m0, ntv, prec, gauge_seed=7, **kw):
    """A context on a seeded gauge field; kw go to the parameters (seed =
    the key of the setup's own random start vectors)."""
    U = synth.su3_field(L, eps, gauge_seed)
    p = dd.default_params(L=L, block=block, m0=m0, csw=1.0, ntv=ntv, prec=prec, max_rhs=kw.pop("max_rhs", 4), **kw)
    ctx = dd.Context(p, dev(U))
    return ctx, U


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nrhs", [1, 3, 6])
def test_dirac_apply(case, prec, nrhs):
    # 1, 3 and 6 rhs: a lone rhs, and groups of 2 or 4 rhs per thread with a
    # ragged last group
    dd = _gpu()
    L, block, eps, m0, ntv = CASES[case]
    say("dirac_apply", case, "prec", prec, "nrhs", nrhs)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, max_rhs=6)
    A = dirac.clover_term(U, m0, 1.0)
    psi = synth.gaussian_spinors(L, nrhs, 11)
    out = torch.zeros_like(dev(psi))
    ctx.dirac_apply(out, dev(psi), nrhs, prec)
    got = host(out)
    ref = np.stack([dirac.apply_D(U, A, psi[r]) for r in range(nrhs)])
    assert rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("case", list(CASES))
def test_clover_export(case):
    dd = _gpu()
    L, block, eps, m0, ntv = CASES[case]
    say("clover", case)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 0)
    V = int(np.prod(L))
    out = torch.zeros((V, 2, 6, 6), dtype=torch.complex128, device="cuda")
    ctx.export_clover(out)
    A = dirac.clover_term(U, m0, 1.0).reshape(V, 12, 12)
    ref = np.stack([A[:, :6, :6], A[:, 6:, 6:]], axis=1)
    assert rel(host(out), ref) <= 1e-13


def _basis(L, block, ntv, seed=21):
    blk = sap.Blocking(L, block)
    W = coarse.orthonormalise(blk, synth.gaussian_spinors(L, ntv, seed))
    return blk, W


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_coarse_operator_restrict_prolong(case, prec):
    """Imported orthonormal basis: D_c (Eq. cgo, backward slots from
    Eq. dagger on the GPU, computed directly by the oracle), R y, P x_c and
    the stencil apply all match the oracle."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES[case]
    say("coarse operator", case, "prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, max_rhs=17)
    A = dirac.clover_term(U, m0, 1.0)
    blk, W = _basis(L, block, ntv)
    ctx.import_basis(dev(W))
    nb, n = blk.nblocks, 2 * ntv
    Dc_ref = coarse.coarse_operator(U, A, blk, W)
    Dc = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx.export_coarse(Dc)
    assert rel(host(Dc), Dc_ref) <= TOL[prec]
    # R y and P x_c
    y = synth.gaussian_spinors(L, 2, 31)
    yc = torch.zeros((2, nb, 2, ntv), dtype=torch.complex128, device="cuda")
    ctx.mg_restrict(yc, dev(y), 2)
    assert rel(host(yc), coarse.restrict(blk, W, y)) <= TOL[prec]
    # seventeen rhs: the matrix-core restriction (FP32 paths)
    y9 = synth.gaussian_spinors(L, 17, 33)
    yc9 = torch.zeros((17, nb, 2, ntv), dtype=torch.complex128, device="cuda")
    ctx.mg_restrict(yc9, dev(y9), 17)
    assert rel(host(yc9), coarse.restrict(blk, W, y9)) <= TOL[prec]
    xc = synth.gaussian_coarse(nb, ntv, 2, 32)
    x = torch.zeros_like(dev(y))
    ctx.mg_prolong(x, dev(xc), 2)
    assert rel(host(x), coarse.prolong(blk, W, xc)) <= TOL[prec]
    # seventeen rhs: a full pass of twelve and a ragged one
    xp17 = synth.gaussian_coarse(nb, ntv, 17, 36)
    x17 = torch.zeros_like(dev(y9))
    ctx.mg_prolong(x17, dev(xp17), 17)
    assert rel(host(x17), coarse.prolong(blk, W, xp17)) <= TOL[prec]
    # stencil apply
    out = torch.zeros_like(dev(xc))
    ctx.coarse_apply(out, dev(xc), 2)
    nbr = coarse.neighbour_table(blk)
    ref = coarse.coarse_apply(Dc_ref, nbr, xc.reshape(2, nb, n)).reshape(xc.shape)
    assert rel(host(out), ref) <= TOL[prec]
    # seventeen rhs: the matrix-core stencil (FP32 paths), a full and a
    # one-rhs tile
    xc17 = synth.gaussian_coarse(nb, ntv, 17, 34)
    out17 = torch.zeros_like(dev(xc17))
    ctx.coarse_apply(out17, dev(xc17), 17)
    ref17 = coarse.coarse_apply(Dc_ref, nbr, xc17.reshape(17, nb, n)).reshape(xc17.shape)
    assert rel(host(out17), ref17) <= TOL[prec]


@pytest.mark.parametrize("geom", [((4, 4, 4, 4), (2, 2, 2, 2), 20), ((8, 4, 4, 4), (4, 2, 2, 2), 16)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_coarse_operator_many_test_vectors(prec, geom):
    """ntv >= 16 (at least 16 columns per Galerkin pass): D_c assembled with
    the matrix-core restriction, summing the block-crossing pieces over the
    last layer of each block only, matches the oracle.  Blocks 4 wide in x
    take the four-site vector staging on every face but x."""
    dd = _gpu()
    L, block, ntv = geom
    eps, m0 = 0.3, -0.1
    say("coarse operator", L, block, "ntv", ntv, "prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, max_rhs=6)
    A = dirac.clover_term(U, m0, 1.0)
    blk, W = _basis(L, block, ntv)
    ctx.import_basis(dev(W))
    nb, n = blk.nblocks, 2 * ntv
    Dc_ref = coarse.coarse_operator(U, A, blk, W)
    Dc = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx.export_coarse(Dc)
    assert rel(host(Dc), Dc_ref) <= TOL[prec]
    # six rhs through the stencil (row tiles of 16 over 2 ntv = 40 or 32 rows)
    xc = synth.gaussian_coarse(nb, ntv, 6, 35)
    out = torch.zeros_like(dev(xc))
    ctx.coarse_apply(out, dev(xc), 6)
    ref = coarse.coarse_apply(Dc_ref, coarse.neighbour_table(blk), xc.reshape(6, nb, n)).reshape(xc.shape)
    assert rel(host(out), ref) <= TOL[prec]


@pytest.mark.parametrize("case", ["c1_4x4x4x4", "ragged_6x4x4x4"])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_vcycle_deterministic(case, prec):
    """Alg. 1 with a fixed number of coarse GMRES iterations (no tolerance
    test), imported basis: GPU V-cycle == oracle V-cycle."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES[case]
    say("vcycle", case, "prec", prec)
    its = 7
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, coarse_fixed_its=its, coarse_restart=5)
    blk, W = _basis(L, block, ntv)
    ctx.import_basis(dev(W))
    p = mg.Params(L, block, m0, 1.0, ntv, coarse_fixed_its=its, coarse_restart=5)
    M = mg.MG(p, U)
    M.set_basis(W)
    # three right-hand sides: the smoother pairs them, leaving a lone last one
    y = synth.gaussian_spinors(L, 3, 41)
    x = torch.zeros_like(dev(y))
    ctx.mg_apply(x, dev(y), 3)
    ref = np.stack([M.vcycle(y[r]) for r in range(3)])
    tol = {0: 1e-10, 1: 1e-5, 2: 2e-2}[prec]
    say("vcycle %s prec %d: rel err %.2e" % (case, prec, rel(host(x), ref)))
    assert rel(host(x), ref) <= tol
    # a lone right-hand side goes through the one-vector smoother kernel
    x1 = torch.zeros_like(dev(y[2:3]))
    ctx.mg_apply(x1, dev(y[2:3].copy()), 1)
    assert rel(host(x1)[0], ref[2]) <= tol


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_setup_deterministic(prec):
    """Alg. 4/5 end to end from the same random start vectors with fixed
    coarse iterations: the GPU aggregate basis and D_c match the oracle's."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    say("setup", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, coarse_fixed_its=6, coarse_restart=30, n_setup=2)
    tv = synth.gaussian_spinors(L, ntv, 102)
    ctx.mg_setup(dev(tv))
    p = mg.Params(L, block, m0, 1.0, ntv, coarse_fixed_its=6, n_setup=2)
    M = mg.MG(p, U)
    M.setup(tv)
    W = torch.zeros_like(dev(tv))
    ctx.export_basis(W)
    tol = {0: 1e-9, 1: 1e-4, 2: 5e-2}[prec]
    say("setup prec %d: basis rel err %.2e" % (prec, rel(host(W), M.W)))
    assert rel(host(W), M.W) <= tol
    nb, n = M.blk.nblocks, 2 * ntv
    Dc = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx.export_coarse(Dc)
    assert rel(host(Dc), M.Dc) <= tol


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_solve_residual(case, prec):
    """Every solution reaches 1e-10 relative residual, recomputed by the
    oracle's own FP64 D; it agrees with the oracle's solve."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES[case]
    say("solve", case, "prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, max_rhs=ntv)
    tv = synth.gaussian_spinors(L, ntv, 102)
    ctx.mg_setup(dev(tv))
    A = dirac.clover_term(U, m0, 1.0)
    f = synth.gaussian_spinors(L, 3, 103)
    u = torch.zeros_like(dev(f))
    rc, st = ctx.solve(u, dev(f), 3, 1e-10)
    assert rc == 0, st
    uh = host(u)
    for r in range(3):
        res = f[r] - dirac.apply_D(U, A, uh[r])
        assert np.linalg.norm(res) / np.linalg.norm(f[r]) <= 1e-10
        assert st["relres"][r] <= 1e-10
    if case == "c1_4x4x4x4":
        p = mg.Params(L, block, m0, 1.0, ntv)
        M = mg.MG(p, U)
        M.setup(tv)
        uo, _ = M.solve(f[0])
        assert rel(uh[0], uo) <= 1e-8


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_solve_long_outer_cycle(prec):
    """A deliberately weak preconditioner (N_tv 2, one SAP cycle of one MR
    step, no setup passes, one coarse iteration; the oracle needs 52 outer
    iterations on this field) with FGMRES(30): the first cycle runs all 30
    iterations, through the two-pass Gram-Schmidt with the deferred
    subtraction (k <= 22), the step that completes the last pending vector
    (k = 23) and the three-pass steps of a long basis (k >= 24), then
    restarts.  Both rhs reach 1e-10, recomputed by the oracle's FP64 D; in
    FP64 the oracle's own solve of the first rhs takes the same number of
    outer iterations (within one) and gives the same solution (1e-12;
    6e-16 measured)."""
    dd = _gpu()
    L, block, m0, ntv = (8, 8, 8, 8), (4, 4, 4, 4), -0.2, 2
    say("long outer cycle prec", prec)
    ctx, U = make_ctx(dd, L, block, 0.5, m0, ntv, prec, gauge_seed=61, max_rhs=2, n_setup=0, nu=1, n_mr=1,
                      coarse_fixed_its=1, outer_restart=30)
    ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 62)))
    A = dirac.clover_term(U, m0, 1.0)
    f = synth.gaussian_spinors(L, 2, 63)
    u = torch.zeros_like(dev(f))
    rc, st = ctx.solve(u, dev(f), 2, 1e-10)
    say("  outer iterations %d, restarts %d, relres %s" % (st["outer_iterations"], st["outer_restarts"],
                                                           st["relres"][:2]))
    assert rc == 0, st
    assert st["outer_iterations"] > 30 and st["outer_restarts"] >= 1
    uh = host(u)
    for r in range(2):
        res = f[r] - dirac.apply_D(U, A, uh[r])
        assert np.linalg.norm(res) / np.linalg.norm(f[r]) <= 1e-10
    ctx.close()
    if prec == 0:
        p = mg.Params(L, block, m0, 1.0, ntv, n_setup=0, nu=1, n_mr=1, coarse_fixed_its=1, outer_restart=30)
        M = mg.MG(p, U)
        M.setup(synth.gaussian_spinors(L, ntv, 62))
        uo, sto = M.solve(f[0])
        say("  oracle: %d outer iterations, solution rel diff %.2e" % (sto["iterations"], rel(uh[0], uo)))
        assert abs(sto["iterations"] - st["outer_iterations"]) <= 1
        assert rel(uh[0], uo) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("kind", ["free_field", "no_clover"])
def test_degenerate_operator(kind, prec):
    """Degenerate cases of the operator: the free field (every link the
    identity) and c_sw = 0 (the clover term is the mass term alone).  D
    applies within the parity bar of its precision, and the solve reaches
    1e-10, recomputed by the oracle's FP64 D."""
    dd = _gpu()
    L, block, ntv, m0 = (4, 4, 4, 4), (2, 2, 2, 2), 8, -0.1
    if kind == "free_field":
        U, csw = np.broadcast_to(np.eye(3, dtype=np.complex128), tuple(reversed(L)) + (4, 3, 3)).copy(), 1.0
    else:
        U, csw = synth.su3_field(L, 0.4, 7), 0.0
    say("degenerate operator", kind, "prec", prec)
    p = dd.default_params(L=L, block=block, m0=m0, csw=csw, ntv=ntv, prec=prec, max_rhs=ntv)
    ctx = dd.Context(p, dev(U))
    A = dirac.clover_term(U, m0, csw)
    psi = synth.gaussian_spinors(L, 2, 11)
    out = torch.zeros_like(dev(psi))
    ctx.dirac_apply(out, dev(psi), 2, prec)
    ref = np.stack([dirac.apply_D(U, A, psi[r]) for r in range(2)])
    assert rel(host(out), ref) <= TOL[prec]
    ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 102)))
    f = synth.gaussian_spinors(L, 2, 103)
    u = torch.zeros_like(dev(f))
    rc, st = ctx.solve(u, dev(f), 2, 1e-10)
    say("  outer iterations %d" % st["outer_iterations"])
    assert rc == 0, st
    uh = host(u)
    for r in range(2):
        res = f[r] - dirac.apply_D(U, A, uh[r])
        assert np.linalg.norm(res) / np.linalg.norm(f[r]) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_maximum_rhs_count(prec):
    """64 right-hand sides, the largest max_rhs: two 32-rhs tiles of the
    matrix-core restriction, four 16-rhs tiles of the coarse stencil, every
    lane of the 64-thread Arnoldi kernels.  D applies within the parity bar,
    and all 64 solutions reach 1e-10, recomputed by the oracle's FP64 D."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    n = 64
    say("maximum rhs count prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, max_rhs=n)
    A = dirac.clover_term(U, m0, 1.0)
    psi = synth.gaussian_spinors(L, n, 11)
    out = torch.zeros_like(dev(psi))
    ctx.dirac_apply(out, dev(psi), n, prec)
    ref = np.stack([dirac.apply_D(U, A, psi[r]) for r in range(n)])
    assert rel(host(out), ref) <= TOL[prec]
    ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 102)))
    f = synth.gaussian_spinors(L, n, 103)
    u = torch.zeros_like(dev(f))
    rc, st = ctx.solve(u, dev(f), n, 1e-10)
    say("  outer iterations %d" % st["outer_iterations"])
    assert rc == 0, st
    uh = host(u)
    for r in range(n):
        res = f[r] - dirac.apply_D(U, A, uh[r])
        assert np.linalg.norm(res) / np.linalg.norm(f[r]) <= 1e-10
        assert st["relres"][r] <= 1e-10
    ctx.close()


@pytest.mark.parametrize("prec", [0, 2])
def test_solve_initial_guess(prec):
    """The solve starts from the caller's u.  All three cases reach 1e-10
    (recomputed by the oracle's D): every guess zero (the first residual is f,
    no operator applied), every guess nonzero (the oracle's solution plus a
    perturbation: the first residual is f - D u), and a mix of both in one
    call; a guess equal to the oracle's solution needs at most one cycle."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    say("initial guess prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, max_rhs=ntv)
    tv = synth.gaussian_spinors(L, ntv, 102)
    ctx.mg_setup(dev(tv))
    A = dirac.clover_term(U, m0, 1.0)
    f = synth.gaussian_spinors(L, 3, 103)
    p = mg.Params(L, block, m0, 1.0, ntv)
    M = mg.MG(p, U)
    M.setup(tv)
    uo = np.stack([M.solve(f[r])[0] for r in range(3)])
    noise = synth.gaussian_spinors(L, 3, 104)
    guesses = {"zero": np.zeros_like(f), "near": uo + 1e-3 * noise,
               "mixed": np.stack([np.zeros_like(f[0]), uo[1] + 1e-3 * noise[1], noise[2]])}
    its = {}
    for name, g0 in guesses.items():
        u = dev(g0.copy())
        rc, st = ctx.solve(u, dev(f), 3, 1e-10)
        assert rc == 0, (name, st)
        uh = host(u)
        for r in range(3):
            res = f[r] - dirac.apply_D(U, A, uh[r])
            assert np.linalg.norm(res) / np.linalg.norm(f[r]) <= 1e-10, (name, r)
        its[name] = st["outer_iterations"]
    say("  outer iterations %s" % its)
    u = dev(uo.copy())
    rc, st = ctx.solve(u, dev(f), 3, 1e-10)
    assert rc == 0 and st["outer_iterations"] <= ctx.params.outer_restart
    ctx.close()


def test_solve_batching_invariance():
    """rhs k solved alone equals rhs k solved in a batch (independent Krylov
    per rhs, shared launches), up to the solver tolerance."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["ragged_6x4x4x4"]
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 1, max_rhs=ntv)
    ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 5)))
    f = synth.gaussian_spinors(L, 3, 6)
    u = torch.zeros_like(dev(f))
    ctx.solve(u, dev(f), 3, 1e-10)
    u1 = torch.zeros_like(dev(f[1:2]))
    ctx.solve(u1, dev(f[1:2].copy()), 1, 1e-10)
    assert rel(host(u)[1], host(u1)[0]) <= 1e-8


def test_solve_zero_and_point_sources():
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 2, max_rhs=12)
    ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 8)))
    f = synth.point_sources(L)
    f[3] = 0.0
    u = torch.ones_like(dev(f))
    rc, st = ctx.solve(u, dev(f), 12, 1e-10)
    assert rc == 0
    uh = host(u)
    assert np.all(uh[3] == 0)
    A = dirac.clover_term(U, m0, 1.0)
    for r in range(12):
        if r == 3:
            continue
        res = f[r] - dirac.apply_D(U, A, uh[r])
        assert np.linalg.norm(res) / np.linalg.norm(f[r]) <= 1e-10


def test_errors_before_setup_and_bad_args():
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 0)
    y = dev(synth.gaussian_spinors(L, 1, 1))
    x = torch.zeros_like(y)
    with pytest.raises(dd.DDAMGError) as e:
        ctx.mg_apply(x, y, 1)
    assert e.value.code == -2
    with pytest.raises(dd.DDAMGError) as e:
        ctx.dirac_apply(x, y, 1, prec=7)
    assert e.value.code == -1
    with pytest.raises(dd.DDAMGError) as e:
        ctx.dirac_apply(y, y, 1)
    assert e.value.code == -1


def test_import_tv_resumes_setup():
    """ddamg_export_tv of a finished setup, given to a fresh context through
    ddamg_import_tv, reproduces its D_c (same test vectors, same kernels)."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    say("import tv")
    ctx1, U = make_ctx(dd, L, block, eps, m0, ntv, 2)
    ctx1.mg_setup(dev(synth.gaussian_spinors(L, ntv, 77)))
    tv = torch.zeros((ntv,) + tuple(reversed(L)) + (4, 3), dtype=torch.complex128, device="cuda").reshape(ntv, -1)
    ctx1.export_tv(tv)
    nb, n = ctx1.nblocks, 2 * ntv
    D1 = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx1.export_coarse(D1)
    ctx2, _ = make_ctx(dd, L, block, eps, m0, ntv, 2)
    ctx2.import_tv(tv)
    D2 = torch.zeros_like(D1)
    ctx2.export_coarse(D2)
    assert rel(host(D2), host(D1)) <= 1e-12
    f = synth.gaussian_spinors(L, 1, 78)
    u = torch.zeros_like(dev(f))
    rc, st = ctx2.solve(u, dev(f), 1, 1e-10)
    assert rc == 0


@pytest.mark.parametrize("ntv", [4, 6, 12, 16, 20, 24, 28, 32])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_aggregate_orthonormalisation(prec, ntv):
    """Alg. 5 on the GPU (CholQR2 behind ddamg_import_tv) against the
    oracle's modified Gram-Schmidt of the same test vectors: every count of
    4-vector K steps of the X T^-1 update (ntv up to 32), with and without
    the second 16-column tile, on aggregates of 24 sites (ragged 16-site and
    8-site tiles)."""
    dd = _gpu()
    L, block = (6, 4, 4, 4), (3, 2, 2, 2)
    say("aggregate QR ntv", ntv, "prec", prec)
    ctx, U = make_ctx(dd, L, block, 0.5, -0.2, ntv, prec)
    tv = synth.gaussian_spinors(L, ntv, 90 + ntv)
    ctx.import_tv(dev(tv))
    W = torch.zeros_like(dev(tv))
    ctx.export_basis(W)
    ref = coarse.orthonormalise(sap.Blocking(L, block), tv)
    assert rel(host(W), ref) <= {0: 1e-11, 1: 1e-5, 2: 1e-2}[prec]


@pytest.mark.parametrize("prec", [0, 2])
def test_import_coarse_injection(prec):
    """A D_c injected with ddamg_import_coarse (the oracle's) is the one
    coarse_apply uses; before any setup the call is refused."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["ragged_6x4x4x4"]
    say("import coarse prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec)
    A = dirac.clover_term(U, m0, 1.0)
    blk, W = _basis(L, block, ntv)
    nb, n = blk.nblocks, 2 * ntv
    Dc_ref = coarse.coarse_operator(U, A, blk, W)
    with pytest.raises(dd.DDAMGError) as e:
        ctx.import_coarse(dev(Dc_ref))
    assert e.value.code == -2
    ctx.import_basis(dev(W))
    # perturb the self blocks so the injected operator differs from the built one
    Dc_inj = Dc_ref.copy()
    Dc_inj[:, 0] *= 1.25
    ctx.import_coarse(dev(Dc_inj))
    xc = synth.gaussian_coarse(nb, ntv, 2, 79)
    out = torch.zeros_like(dev(xc))
    ctx.coarse_apply(out, dev(xc), 2)
    nbr = coarse.neighbour_table(blk)
    ref = coarse.coarse_apply(Dc_inj, nbr, xc.reshape(2, nb, n)).reshape(xc.shape)
    assert rel(host(out), ref) <= TOL[prec]


def test_allocator_hook_owns_workspace():
    """With a caller's allocator installed (here torch's caching
    allocator), a context allocates through it and releases every block on
    destruction; the default is restored afterwards."""
    dd = _gpu()
    live = {}

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n)
        live[p] = n
        return p

    def free(p):
        assert p in live
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    say("allocator hook")
    dd.set_allocator(alloc, free)
    try:
        ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 2)
        ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 80)))
        f = synth.gaussian_spinors(L, 1, 81)
        u = torch.zeros_like(dev(f))
        rc, st = ctx.solve(u, dev(f), 1, 1e-10)
        assert rc == 0
        assert len(live) > 0
        ctx.close()
        assert len(live) == 0
    finally:
        dd.set_allocator()
    A = dirac.clover_term(U, m0, 1.0)
    res = f[0] - dirac.apply_D(U, A, host(u)[0])
    assert np.linalg.norm(res) / np.linalg.norm(f[0]) <= 1e-10


def test_kernel_timing_counts():
    """ddamg_set_kernel_timing / ddamg_get_kernel_times (what the benchmark's
    roofline reads): one outer Gram-Schmidt group and one w = D z per outer
    iteration with all rhs, one aggregate QR per basis build (1 + N_setup
    builds of N_tv vectors), positive times; enabling zeroes the sums and
    nothing is counted while timing is off."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    say("kernel timing")
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 2)
    n_setup = ctx.params.n_setup
    ctx.set_kernel_timing(True)
    ctx.mg_setup(dev(synth.gaussian_spinors(L, ntv, 91)))
    f = synth.gaussian_spinors(L, 2, 92)
    u = torch.zeros_like(dev(f))
    rc, st = ctx.solve(u, dev(f), 2, 1e-10)
    assert rc == 0
    kt = ctx.kernel_times()
    its = st["outer_iterations"]
    assert kt["outer_gs"][1:] == (its, 2 * its)
    assert kt["dslash"][1:] == (its, 2 * its)
    assert kt["setup_qr"][1:] == (1 + n_setup, (1 + n_setup) * ntv)
    for k in ("sap", "restrict", "prolong", "coarse", "outer_gs", "setup_qr", "setup_galerkin"):
        assert kt[k][0] > 0.0 and kt[k][1] > 0, (k, kt[k])
    ctx.set_kernel_timing(True)
    assert all(v == (0.0, 0, 0) for v in ctx.kernel_times().values())
    ctx.set_kernel_timing(False)
    u.zero_()
    rc, st = ctx.solve(u, dev(f), 2, 1e-10)
    assert rc == 0
    assert all(v == (0.0, 0, 0) for v in ctx.kernel_times().values())
    ctx.close()


def _internal_site_index(L, block):
    """Internal (block-major) site index of every canonical site, in the
    canonical order [t][z][y][x], from the order stated in the header."""
    NB = [L[m] // block[m] for m in range(4)]
    t, z, y, x = np.meshgrid(*[np.arange(L[m]) for m in (3, 2, 1, 0)], indexing="ij")
    c = [x, y, z, t]
    bc = [c[m] // block[m] for m in range(4)]
    lc = [c[m] % block[m] for m in range(4)]
    l = lc[0] + block[0] * (lc[1] + block[1] * (lc[2] + block[2] * lc[3]))
    lexb = bc[0] + NB[0] * (bc[1] + NB[1] * (bc[2] + NB[2] * bc[3]))
    nb = NB[0] * NB[1] * NB[2] * NB[3]
    ci = ((bc[0] + bc[1] + bc[2] + bc[3]) % 2) * (nb // 2) + lexb // 2
    vb = block[0] * block[1] * block[2] * block[3]
    return (ci * vb + l).reshape(-1), ci, lexb


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_internal_layout_applies(prec):
    """dirac_apply_internal and coarse_apply_internal on fields permuted into
    the internal order the header states match the oracle's D and D_c."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["ragged_6x4x4x4"]
    say("internal applies prec", prec)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec)
    A = dirac.clover_term(U, m0, 1.0)
    V = int(np.prod(L))
    S, _, _ = _internal_site_index(L, block)
    assert np.array_equal(np.sort(S), np.arange(V))
    ct = np.complex128 if prec == 0 else np.complex64
    psi = synth.gaussian_spinors(L, 2, 95)
    inner = np.zeros((2, 12, V), dtype=ct)
    inner[:, :, S] = psi.reshape(2, V, 12).transpose(0, 2, 1)
    out = torch.zeros_like(dev(inner))
    ctx.dirac_apply_internal(out, dev(inner), 2, prec)
    got = host(out)[:, :, S].transpose(0, 2, 1).reshape(psi.shape)
    ref = np.stack([dirac.apply_D(U, A, psi[r]) for r in range(2)])
    assert rel(got, ref) <= TOL[prec]
    # coarse fields: internal coarse site ci of every lexicographic block
    blk, W = _basis(L, block, ntv)
    ctx.import_basis(dev(W))
    nb, n = blk.nblocks, 2 * ntv
    Dc_ref = coarse.coarse_operator(U, A, blk, W)
    NB = [L[m] // block[m] for m in range(4)]
    bcs = np.array([[b % NB[0], (b // NB[0]) % NB[1], (b // (NB[0] * NB[1])) % NB[2], b // (NB[0] * NB[1] * NB[2])]
                    for b in range(nb)])
    cib = (bcs.sum(axis=1) % 2) * (nb // 2) + np.arange(nb) // 2
    assert np.array_equal(np.sort(cib), np.arange(nb))
    xc = synth.gaussian_coarse(nb, ntv, 2, 96).reshape(2, nb, n)
    cin = np.zeros((2, nb, n), dtype=ct)
    cin[:, cib, :] = xc
    cout = torch.zeros_like(dev(cin))
    ctx.coarse_apply_internal(cout, dev(cin), 2)
    gotc = host(cout)[:, cib, :]
    refc = coarse.coarse_apply(Dc_ref, coarse.neighbour_table(blk), xc)
    assert rel(gotc, refc) <= TOL[prec]
    ctx.close()


def test_rhs_count_rejected_before_any_work():
    """Every multi-rhs entry point returns -1 (bad argument) for nrhs = 0 and
    nrhs > max_rhs and leaves its output untouched (buffers are sized for
    max_rhs + 1, so nothing could run out of bounds either way)."""
    dd = _gpu()
    import ctypes
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, 2)
    blk, W = _basis(L, block, ntv)
    ctx.import_basis(dev(W))
    mr = ctx.params.max_rhs
    fine = dev(synth.gaussian_spinors(L, mr + 1, 97))
    crs = dev(synth.gaussian_coarse(blk.nblocks, ntv, mr + 1, 98))
    fo, co = torch.full_like(fine, 7.0), torch.full_like(crs, 7.0)
    fp, cp = ctypes.c_void_p(fine.data_ptr()), ctypes.c_void_p(crs.data_ptr())
    fop, cop = ctypes.c_void_p(fo.data_ptr()), ctypes.c_void_p(co.data_ptr())
    lib, h = dd.lib, ctx.h
    for n in (0, mr + 1):
        calls = {
            "dirac_apply": lambda: lib.dirac_apply(h, fop, fp, n, dd.MIXED16),
            "mg_apply": lambda: lib.mg_apply(h, fop, fp, n),
            "coarse_apply": lambda: lib.coarse_apply(h, cop, cp, n),
            "mg_restrict": lambda: lib.mg_restrict(h, cop, fp, n),
            "mg_prolong": lambda: lib.mg_prolong(h, fop, cp, n),
            "solve": lambda: lib.solve(h, fop, fp, n, 1e-10, ctypes.byref(dd.Stats())),
        }
        for name, call in calls.items():
            assert call() == -1, (name, n)
            assert b"nrhs" in lib.ddamg_last_error(h), name
    torch.cuda.synchronize()
    assert bool((fo == 7.0).all()) and bool((co == 7.0).all())
    ctx.close()


@pytest.mark.parametrize("prec", [0, 2])
def test_setup_seeded_start(prec):
    """mg_setup without start vectors draws them on the device from
    params.seed (Philox4x32-10 and Box-Muller, as the header states); the
    same vectors drawn on the host by an independent implementation of that
    generator give the same basis and D_c.  Another seed gives another
    basis."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["c1_4x4x4x4"]
    seed = (7 << 32) + 12345
    say("seeded setup prec", prec)
    kw = dict(coarse_fixed_its=6, n_setup=1)
    ctx1, U = make_ctx(dd, L, block, eps, m0, ntv, prec, seed=seed, **kw)
    ctx1.mg_setup()
    ctx2, _ = make_ctx(dd, L, block, eps, m0, ntv, prec, **kw)
    ctx2.mg_setup(dev(synth.philox_gaussian_spinors(L, ntv, seed)))
    ctx3, _ = make_ctx(dd, L, block, eps, m0, ntv, prec, seed=seed + 1, **kw)
    ctx3.mg_setup()
    shp = (ntv,) + tuple(reversed(L)) + (4, 3)
    W1, W2, W3 = (torch.zeros(shp, dtype=torch.complex128, device="cuda") for _ in range(3))
    ctx1.export_basis(W1)
    ctx2.export_basis(W2)
    ctx3.export_basis(W3)
    e = rel(host(W1), host(W2))
    say("seeded setup prec %d: basis rel diff %.2e" % (prec, e))
    assert e <= {0: 1e-10, 2: 1e-5}[prec]
    assert rel(host(W3), host(W2)) > 0.1
    nb, n = ctx1.nblocks, 2 * ntv
    D1, D2 = (torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda") for _ in range(2))
    ctx1.export_coarse(D1)
    ctx2.export_coarse(D2)
    assert rel(host(D1), host(D2)) <= {0: 1e-10, 2: 1e-5}[prec]
    for c in (ctx1, ctx2, ctx3):
        c.close()


@pytest.mark.parametrize("restart", [2, 30])
@pytest.mark.parametrize("prec", [0, 2])
def test_coarse_pipelined_convergence_test(prec, restart):
    """The pipelined convergence test of the coarse GMRES (flags read one
    iteration late, the extra iteration predicated away) gives bitwise the
    V-cycle of the per-iteration host read, with the same coarse iteration
    counts, with and without coarse restarts; a tight coarse tolerance
    makes the coarse solve run several iterations."""
    dd = _gpu()
    L, block, eps, m0, ntv = CASES["ragged_6x4x4x4"]
    say("coarse convergence test prec", prec, "restart", restart)
    ctx, U = make_ctx(dd, L, block, eps, m0, ntv, prec, coarse_tol=1e-4, coarse_restart=restart)
    # both variants of the multi-launch solve (this coarse lattice is small
    # enough for the single-kernel one, which the host-sync switch turns off)
    ctx.set_coarse_single_kernel(False)
    blk, W = _basis(L, block, ntv)
    ctx.import_basis(dev(W))
    y = dev(synth.gaussian_spinors(L, 3, 47))
    out = {}
    for each in (True, False):
        ctx.set_coarse_host_sync(each)
        ctx.reset_stats()
        x = torch.zeros_like(y)
        ctx.mg_apply(x, y, 3)
        out[each] = (host(x), ctx.stats())
    assert np.array_equal(out[True][0], out[False][0])
    for k in ("coarse_solves", "coarse_iterations", "coarse_iterations_max"):
        assert out[True][1][k] == out[False][1][k], k
    assert out[False][1]["coarse_iterations_max"] >= 4
    ctx.close()
