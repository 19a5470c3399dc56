"""Element-wise parity with the oracle in the benchmark's launch shapes.

The 32^3 x 64 benchmark runs 4^4 blocks (256 threads and four waves per SAP
workgroup, cross-wave reductions), N_tv = 24 (coarse blocks of 48 x 48:
three 16-row tiles of the matrix-core stencil), 12 right-hand sides in the
solve and 24 in the setup's V-cycles (matrix-core restriction).  These
tests run exactly those shapes on the smallest lattice that holds them,
8^4 (a 2^4 block lattice), against the FP64 oracle element by element:

* D_c = R D P (Eq. cgo) from an imported basis, and the 12-rhs stencil;
* the V-cycle (Alg. 1) with a fixed number of coarse iterations, 12 and
  24 rhs, FP64 / FP32 / FP16 storage;
* the whole setup (Alg. 4, Alg. 5) from the same random start vectors with
  one iterative pass and fixed coarse iterations;

and the 16^4 workload (4^4 blocks, N_tv 20, FP32 preconditioner, 8
Gaussian rhs) through setup and solve, every residual recomputed by the
oracle's D.  Tolerances are relative to the largest element of the oracle's
output: 1e-12 / 1e-5 / 1e-2 (FP64 / FP32 / FP16 storage, the parity bars) for
the operator applies and the V-cycle, 1e-11 / 1e-5 / 1e-2 for the setup.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import dirac, sap, coarse, mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L = (8, 8, 8, 8)
BLOCK = (4, 4, 4, 4)
EPS, M0, CSW, NTV = 0.5, -0.2, 1.0, 24
FIXED_ITS, COARSE_RESTART = 6, 4  # a restart inside the fixed coarse iterations
NRHS_MAX = 24
# operator applies (the parity bars): FP64 1e-12, FP32 1e-5, 16-bit storage 1e-2
TOL_OP = {0: 1e-12, 1: 1e-5, 2: 1e-2}
# composites: V-cycle and setup chain dozens of applies and inner products;
# measured here 8e-16 / 3.4e-7 / 3.0e-4 (V-cycle) and 1.1e-15 / 3.1e-7 /
# 8.3e-4 (setup basis), so the same bars hold for them as well
TOL_VCYCLE = {0: 1e-12, 1: 1e-5, 2: 1e-2}
TOL_SETUP = {0: 1e-11, 1: 1e-5, 2: 1e-2}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_04506_amd as dd
    return dd


@pytest.fixture(scope="module")
def ref():
    """The oracle's D_c, 24-rhs V-cycle and one-pass setup on the 8^4
    lattice (about a minute of CPU work, shared by all precisions)."""
    _gpu()
    U = synth.su3_field(L, EPS, 401)
    blk = sap.Blocking(L, BLOCK)
    W = coarse.orthonormalise(blk, synth.gaussian_spinors(L, NTV, 402))
    say("bench shape: oracle D_c (N_tv 24)")
    p = mg.Params(L, BLOCK, M0, CSW, NTV, coarse_fixed_its=FIXED_ITS, coarse_restart=COARSE_RESTART)
    M = mg.MG(p, U)
    M.set_basis(W)
    y = synth.gaussian_spinors(L, NRHS_MAX, 403)
    say("bench shape: oracle V-cycle of 24 rhs")
    x = np.stack([M.vcycle(y[r]) for r in range(NRHS_MAX)])
    xc = synth.gaussian_coarse(blk.nblocks, NTV, 12, 404)
    nbr = coarse.neighbour_table(blk)
    dcx = coarse.coarse_apply(M.Dc, nbr, xc.reshape(12, blk.nblocks, 2 * NTV)).reshape(xc.shape)
    return dict(U=U, blk=blk, W=W, Dc=M.Dc, y=y, x=x, xc=xc, dcx=dcx)


@pytest.fixture(scope="module")
def ref_setup():
    _gpu()
    U = synth.su3_field(L, EPS, 411)
    tv = synth.gaussian_spinors(L, NTV, 412)
    say("bench shape: oracle setup (3 smoother passes + 1 V-cycle pass, N_tv 24)")
    p = mg.Params(L, BLOCK, M0, CSW, NTV, n_setup=1, coarse_fixed_its=FIXED_ITS, coarse_restart=COARSE_RESTART)
    M = mg.MG(p, U)
    M.setup(tv)
    return dict(U=U, tv=tv, W=M.W, Dc=M.Dc)


def _ctx(dd, U, prec, **kw):
    p = dd.default_params(L=L, block=BLOCK, m0=M0, csw=CSW, ntv=NTV, prec=prec, max_rhs=NRHS_MAX,
                          coarse_fixed_its=FIXED_ITS, coarse_restart=COARSE_RESTART, **kw)
    return dd.Context(p, dev(U))


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_benchshape_coarse_operator_and_stencil(ref, prec):
    """D_c at N_tv = 24 (nc = 48) from an imported basis, and the 12-rhs
    stencil apply (the matrix-core path of the FP32 arithmetic)."""
    dd = _gpu()
    ctx = _ctx(dd, ref["U"], prec)
    ctx.import_basis(dev(ref["W"]))
    nb, n = ref["blk"].nblocks, 2 * NTV
    Dc = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx.export_coarse(Dc)
    e = rel(host(Dc), ref["Dc"])
    say("bench shape prec %d: D_c rel err %.2e" % (prec, e))
    assert e <= TOL_OP[prec]
    out = torch.zeros_like(dev(ref["xc"]))
    ctx.coarse_apply(out, dev(ref["xc"]), 12)
    e = rel(host(out), ref["dcx"])
    say("bench shape prec %d: 12-rhs D_c x rel err %.2e" % (prec, e))
    assert e <= TOL_OP[prec]
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_benchshape_vcycle(ref, prec):
    """Alg. 1 with 4^4 blocks and N_tv 24 at 24 rhs (the setup's V-cycles:
    matrix-core restriction) and 12 rhs (the solve's), fixed coarse
    iterations, against the oracle element by element."""
    dd = _gpu()
    ctx = _ctx(dd, ref["U"], prec)
    ctx.import_basis(dev(ref["W"]))
    for nrhs in (24, 12):
        y = ref["y"][:nrhs]
        x = torch.zeros_like(dev(y))
        ctx.mg_apply(x, dev(y), nrhs)
        e = rel(host(x), ref["x"][:nrhs])
        say("bench shape prec %d: V-cycle %d rhs rel err %.2e" % (prec, nrhs, e))
        assert e <= TOL_VCYCLE[prec]
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_benchshape_setup(ref_setup, prec):
    """Alg. 4 / Alg. 5 end to end at 4^4 blocks and N_tv 24 (24-rhs smoother
    passes and V-cycles, FP64 aggregate Gram-Schmidt, D_c assembly) from
    the same start vectors, one iterative pass, fixed coarse iterations."""
    dd = _gpu()
    r = ref_setup
    ctx = _ctx(dd, r["U"], prec, n_setup=1)
    ctx.mg_setup(dev(r["tv"]))
    W = torch.zeros_like(dev(r["tv"]))
    ctx.export_basis(W)
    e_w = rel(host(W), r["W"])
    nb, n = ctx.nblocks, 2 * NTV
    Dc = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx.export_coarse(Dc)
    e_d = rel(host(Dc), r["Dc"])
    say("bench shape prec %d: setup basis rel err %.2e, D_c rel err %.2e" % (prec, e_w, e_d))
    assert e_w <= TOL_SETUP[prec] and e_d <= TOL_SETUP[prec]
    ctx.close()


def test_workload_16x16x16x16_fp32():
    """The 16^4 workload: eps 0.5, m0 -0.2, c_sw 1, 4^4 blocks, N_tv 20, FP32
    smoother and coarse solve in the FP64 outer FGMRES, 8 Gaussian rhs as one
    block vector (seeds 201 / 202 / 203).  Setup and solve on the GPU; the
    oracle's own D recomputes every residual."""
    dd = _gpu()
    Lw = (16, 16, 16, 16)
    U = synth.su3_field(Lw, 0.5, 201)
    p = dd.default_params(L=Lw, block=(4, 4, 4, 4), m0=-0.2, csw=1.0, ntv=20, prec=dd.FP32, max_rhs=8)
    ctx = dd.Context(p, dev(U))
    say("16^4: setup")
    ctx.mg_setup(dev(synth.gaussian_spinors(Lw, 20, 202)))
    f = synth.gaussian_spinors(Lw, 8, 203)
    u = torch.zeros_like(dev(f))
    say("16^4: solve of 8 rhs")
    rc, st = ctx.solve(u, dev(f), 8, 1e-10)
    assert rc == 0, st
    uh = host(u)
    A = dirac.clover_term(U, -0.2, 1.0)
    for r in range(8):
        res = np.linalg.norm(f[r] - dirac.apply_D(U, A, uh[r])) / np.linalg.norm(f[r])
        say("16^4: rhs %d oracle residual %.2e (library %.2e), outer its %d" %
            (r, res, st["relres"][r], st["outer_iterations"]))
        assert res <= 1e-10
    ctx.close()


@pytest.mark.parametrize("nrhs", [1, 3, 12, 17])
def test_benchshape_fp16_stencil_arithmetic(ref, nrhs):
    """The stencil with D_c stored in FP16 (per-block FP32 scales) against
    the oracle applying the library's own stored D_c (exported, dequantised)
    in FP64: this isolates the arithmetic error of the apply from the
    storage rounding, and it must be at FP32 level (1e-5).  1 and 3 rhs take
    the vector kernel, 12 and 17 the f16 matrix-core kernel with its
    two-part split of the input vectors (a full tile of 16 rhs and a ragged
    one)."""
    dd = _gpu()
    ctx = _ctx(dd, ref["U"], 2)
    ctx.import_basis(dev(ref["W"]))
    nb, n = ref["blk"].nblocks, 2 * NTV
    Dc = torch.zeros((nb, 9, n, n), dtype=torch.complex128, device="cuda")
    ctx.export_coarse(Dc)
    Dq = host(Dc)
    xc = synth.gaussian_coarse(nb, NTV, nrhs, 405)
    # input entries over several orders of magnitude (rhs k scaled by 10^(k-6))
    xc = xc * (10.0 ** (np.arange(nrhs) - 6.0)).reshape(-1, 1, 1, 1)
    out = torch.zeros_like(dev(xc))
    ctx.coarse_apply(out, dev(xc), nrhs)
    want = coarse.coarse_apply(Dq, coarse.neighbour_table(ref["blk"]), xc.reshape(nrhs, nb, n)).reshape(xc.shape)
    got = host(out)
    e = max(rel(got[r], want[r]) for r in range(nrhs))
    say("bench shape: FP16-stored D_c, %d rhs, arithmetic rel err %.2e (per rhs, worst)" % (nrhs, e))
    assert e <= 1e-5
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("Lr", [(8, 8, 8, 8), (8, 8, 8, 16), (16, 8, 8, 8)])
def test_benchshape_dirac_one_rhs(prec, Lr):
    """D psi for one rhs on 4^4 blocks against the oracle: with FP32 inputs
    the kernel that also stages the x and y faces of the neighbour blocks
    in LDS (two blocks in a direction: both neighbours are the same block;
    four blocks in x)."""
    dd = _gpu()
    U = synth.su3_field(Lr, EPS, 421)
    A = dirac.clover_term(U, M0, CSW)
    psi = synth.gaussian_spinors(Lr, 1, 422)
    want = dirac.apply_D(U, A, psi[0])
    p = dd.default_params(L=Lr, block=BLOCK, m0=M0, csw=CSW, ntv=NTV, prec=prec, max_rhs=1)
    ctx = dd.Context(p, dev(U))
    out = torch.zeros_like(dev(psi))
    ctx.dirac_apply(out, dev(psi), 1, prec)
    e = rel(host(out)[0], want)
    say("one-rhs D on %s, prec %d: rel err %.2e" % (Lr, prec, e))
    assert e <= TOL_OP[prec]
    ctx.close()
