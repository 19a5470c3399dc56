"""The 32^3 x 64 benchmark configuration on the GPU (4^4 blocks, N_tv = 24,
FP16 storage with FP32 arithmetic, the launch shapes bench.py times),
checked against the oracle on sampled outputs and through properties that
hold at any size:

* D psi at 256 sampled sites against the oracle's site-local D (FP64 storage
  1e-12, FP16 storage 1e-2, relative to the sampled output's max);
* R P x_c = x_c for 24 rhs (matrix-core restriction) and 12 rhs (VALU
  restriction) up to the FP16 rounding of the stored basis (1e-2);
* D_c x_c = R D P x_c with the FP32 operator D_c is assembled from, up to the
  FP16 rounding of D_c (1e-2);
* the 12 point-source solve converges to 1e-10, and the oracle's site-local
  residual at sampled sites stays below 1e-10 ||f|| for two of the rhs.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import dirac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L = (32, 32, 32, 64)
BLOCK = (4, 4, 4, 4)
EPS, M0, CSW, NTV = 0.5, -0.2, 1.0, 24


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def sample_sites(n, seed, extra=()):
    rng = np.random.default_rng(seed)
    s = np.stack([rng.integers(0, l, n) for l in L], axis=1)
    if extra:
        s = np.concatenate([s, np.array(extra, dtype=s.dtype)], axis=0)
    return s


def at_sites(field, sites):
    return np.array([field[t, z, y, x] for x, y, z, t in sites])


@pytest.fixture(scope="module")
def c3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_04506_amd as dd
    say("full size: generating the 32^3x64 field and test vectors")
    U = synth.su3_field(L, EPS, 301)
    p = dd.default_params(L=L, block=BLOCK, m0=M0, csw=CSW, ntv=NTV, prec=dd.MIXED16, max_rhs=24)
    ctx = dd.Context(p, dev(U))
    tv = dev(synth.gaussian_spinors(L, NTV, 302))
    say("full size: setup")
    ctx.mg_setup(tv)
    del tv
    torch.cuda.empty_cache()
    yield dd, ctx, U
    ctx.close()
    torch.cuda.empty_cache()


def test_fullsize_dirac_sampled(c3):
    dd, ctx, U = c3
    psi = synth.gaussian_spinors(L, 1, 303)
    sites = sample_sites(256, 7, extra=[(0, 0, 0, 0), (31, 31, 31, 63), (3, 4, 5, 63), (31, 0, 4, 0)])
    ref = dirac.apply_D_sites(U, M0, CSW, psi[0], sites)
    out = torch.zeros_like(dev(psi))
    for prec, tol in ((dd.FP64, 1e-12), (dd.MIXED16, 1e-2)):
        say("full size: dirac_apply prec", prec)
        ctx.dirac_apply(out, dev(psi), 1, prec)
        got = at_sites(host(out)[0], sites)
        assert rel(got, ref) <= tol


@pytest.mark.parametrize("nrhs", [24, 12])
def test_fullsize_restrict_prolong_roundtrip(c3, nrhs):
    dd, ctx, U = c3
    nb = ctx.nblocks
    say("full size: R P x_c, nrhs", nrhs)
    xc = synth.gaussian_coarse(nb, NTV, nrhs, 304)
    x = torch.zeros((nrhs,) + tuple(reversed(L)) + (4, 3), dtype=torch.complex128, device="cuda")
    ctx.mg_prolong(x, dev(xc), nrhs)
    yc = torch.zeros_like(dev(xc))
    ctx.mg_restrict(yc, x, nrhs)
    del x
    torch.cuda.empty_cache()
    assert rel(host(yc), xc) <= 1e-2


def test_fullsize_galerkin_consistency(c3):
    dd, ctx, U = c3
    nb = ctx.nblocks
    say("full size: D_c x_c against R D P x_c")
    xc = dev(synth.gaussian_coarse(nb, NTV, 2, 305))
    x = torch.zeros((2,) + tuple(reversed(L)) + (4, 3), dtype=torch.complex128, device="cuda")
    ctx.mg_prolong(x, xc, 2)
    y = torch.zeros_like(x)
    ctx.dirac_apply(y, x, 2, dd.FP32)
    yc = torch.zeros_like(xc)
    ctx.mg_restrict(yc, y, 2)
    dc = torch.zeros_like(xc)
    ctx.coarse_apply(dc, xc, 2)
    del x, y
    torch.cuda.empty_cache()
    assert rel(host(dc), host(yc)) <= 1e-2


def test_fullsize_point_source_solve(c3):
    dd, ctx, U = c3
    say("full size: solve of the 12 point sources")
    f = synth.point_sources(L)
    fd = dev(f)
    u = torch.zeros_like(fd)
    rc, st = ctx.solve(u, fd, 12, 1e-10)
    assert rc == 0
    assert max(st["relres"][:12]) <= 1e-10
    src = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 0, 0, 1), (31, 0, 0, 0), (0, 0, 0, 63)]
    sites = sample_sites(200, 11, extra=src)
    for r in (0, 7):
        ur = host(u[r])
        res = at_sites(f[r], sites) - dirac.apply_D_sites(U, M0, CSW, ur, sites)
        fn = np.linalg.norm(f[r])
        say("full size: sampled residual of rhs", r, np.abs(res).max() / fn)
        assert np.abs(res).max() <= 1e-10 * fn * (1 + 1e-6)
