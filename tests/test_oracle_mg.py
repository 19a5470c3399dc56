"""Pins of the oracle's V-cycle, setup and outer FGMRES (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import dirac, coarse, mg
from helpers import dense_from_apply, relerr

L = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def c1():
    """The 4^4 configuration: eps 0.3, m0 -0.1, c_sw 1, 2^4 blocks, Ntv 8,
    3 setup iterations, SAP with 4 MR steps."""
    U = synth.su3_field(L, 0.3, 101)
    p = mg.Params(L, (2, 2, 2, 2), -0.1, 1.0, 8, n_setup=3)
    M = mg.MG(p, U)
    M.setup(synth.gaussian_spinors(L, 8, 102))
    return M


def test_setup_produces_orthonormal_basis(c1):
    M = c1
    shp = (L[3], L[2], L[1], L[0], 4, 3)
    R = dense_from_apply(lambda y: coarse.restrict(M.blk, M.W, y), shp)
    assert np.abs(R @ R.conj().T - np.eye(R.shape[0])).max() < 1e-13
    # the final test vectors lie in the span of the prolongation
    P = R.conj().T
    for j in range(8):
        v = M.V[j].reshape(-1)
        assert relerr(P @ (R @ v), v) < 1e-12


def test_vcycle_homogeneous(c1):
    M = c1
    y = synth.gaussian_spinors(L, 1, 141)[0]
    a = M.vcycle(y)
    b = M.vcycle((0.5 + 2j) * y)
    assert relerr(b, (0.5 + 2j) * a) < 1e-12


def test_vcycle_is_good_preconditioner(c1):
    M = c1
    y = synth.gaussian_spinors(L, 1, 142)[0]
    x = M.vcycle(y)
    r = y - M.D(x)
    assert np.linalg.norm(r) < 0.2 * np.linalg.norm(y)


def test_solve_reaches_tolerance_and_dense_solution(c1):
    M = c1
    f = synth.gaussian_spinors(L, 1, 103)[0]
    u, st = M.solve(f, tol=1e-10)
    assert mg.true_relres(M.D, u, f) <= 1e-10
    shp = f.shape
    D = dense_from_apply(M.D, shp)
    ud = np.linalg.solve(D, f.reshape(-1))
    kappa = np.linalg.cond(D)
    assert relerr(u.reshape(-1), ud) <= kappa * 1e-10
    assert st['iterations'] < 30


def test_solve_zero_rhs(c1):
    f = np.zeros((L[3], L[2], L[1], L[0], 4, 3), dtype=complex)
    u, st = c1.solve(f)
    assert np.all(u == 0) and st['relres'] == 0.0


def test_fgmres_textbook_minimal_residual():
    """With a fixed linear right preconditioner, FGMRES after k iterations
    minimises ||b - A u|| over u in M^{-1} K_k(A M^{-1}, b)."""
    rng = np.random.default_rng(3)
    n = 50
    A = np.eye(n) * 2 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    Minv = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    k = 6
    u, st = mg.fgmres(lambda v: A @ v, lambda v: Minv @ v, b, None, 0.0, 20, 100, fixed_its=k)
    AM = A @ Minv
    K = np.array([np.linalg.matrix_power(AM, j) @ b for j in range(k)]).T
    c, *_ = np.linalg.lstsq(AM @ K, b, rcond=None)
    assert relerr(u, Minv @ K @ c) < 1e-10
    # the Givens estimate at a normal stop equals the true residual
    u2, st2 = mg.fgmres(lambda v: A @ v, lambda v: Minv @ v, b, None, 1e-12, 20, 200)
    assert np.linalg.norm(b - A @ u2) <= 1e-12 * np.linalg.norm(b)


def test_solve_with_point_sources_and_restart():
    """A point source and a short restart still reach 1e-10 (true residual)."""
    U = synth.su3_field(L, 0.5, 301)
    p = mg.Params(L, (2, 2, 2, 2), -0.2, 1.0, 8, n_setup=1, outer_restart=3)
    M = mg.MG(p, U)
    M.setup(synth.gaussian_spinors(L, 8, 302))
    f = synth.point_sources(L)[7]
    u, st = M.solve(f)
    assert mg.true_relres(M.D, u, f) <= 1e-10
    assert st['restarts'] >= 2


def test_setup_composition_with_decoupled_blocks():
    """Pin of the order of Alg. 4's passes.  With the links across block faces
    cut, D is block diagonal; with the block MR run to convergence every SAP
    cycle returns the block solve, so each smoother pass from zero and each
    V-cycle (whatever the coarse correction gave as start) returns D^{-1} y.
    Alg. 4 then leaves every test vector at D^{-N_setup} x3 with x3 =
    D^{-3} v / |D^{-3} v| for its start vector v (three smoother passes, the
    one normalisation after the initial setup, N_setup V-cycle passes), and
    the basis is their aggregate Gram-Schmidt.  A pass too many or too few
    changes the power, and a normalisation after the last pass changes the
    length: either fails the check."""
    Ls, bs, ntv, n_setup = (4, 4, 2, 2), (2, 2, 1, 1), 4, 2
    U = synth.su3_field(Ls, 0.5, 61)
    c = dirac.coords(Ls)
    for mu in range(4):
        U[..., mu, :, :][(c[mu] % bs[mu]) == bs[mu] - 1] = 0.0
    p = mg.Params(Ls, bs, -0.2, 1.0, ntv, n_setup=n_setup, n_mr=80)
    M = mg.MG(p, U)
    v0 = synth.gaussian_spinors(Ls, ntv, 62)
    V = M.setup(v0)
    shp = (Ls[3], Ls[2], Ls[1], Ls[0], 4, 3)
    D = dense_from_apply(M.D, shp)
    for j in range(ntv):
        x = v0[j].reshape(-1)
        for _ in range(3):
            x = np.linalg.solve(D, x)
        x /= np.linalg.norm(x)
        for _ in range(n_setup):
            x = np.linalg.solve(D, x)
        assert relerr(V[j].reshape(-1), x) < 1e-9
        # one power fewer is far off, and so is the unit vector along x (the
        # check has teeth for the passes and for where the normalisation is)
        assert relerr(V[j].reshape(-1), D @ x) > 1e-3
        assert abs(np.linalg.norm(x) - 1.0) > 1e-3
        assert relerr(V[j].reshape(-1), x / np.linalg.norm(x)) > 1e-3
    assert relerr(M.W, coarse.orthonormalise(M.blk, V)) < 1e-12


def _dense_vcycle_case(nu):
    """A small lattice where the V-cycle's pieces are exact: block solves by
    many MR steps (to rounding), coarse solve to 1e-14.  Returns the oracle
    MG object and the dense D, B, R, P it is checked against."""
    Ls, bs, ntv = (4, 4, 2, 2), (2, 2, 1, 1), 4
    U = synth.su3_field(Ls, 0.5, 63)
    p = mg.Params(Ls, bs, -0.2, 1.0, ntv, nu=nu, n_mr=80, coarse_tol=1e-14, coarse_restart=64,
                  coarse_maxit=640)
    M = mg.MG(p, U)
    M.set_basis(coarse.orthonormalise(M.blk, synth.gaussian_spinors(Ls, ntv, 64)))
    shp = (Ls[3], Ls[2], Ls[1], Ls[0], 4, 3)
    D = dense_from_apply(M.D, shp)
    B = dense_from_apply(lambda q: dirac.apply_B(U, M.A, q, Ls, bs), shp)
    R = dense_from_apply(lambda q: coarse.restrict(M.blk, M.W, q), shp)
    P = R.conj().T
    return M, shp, D, B, R, P


def _schwarz(blk, D, B, y, x0, nu):
    """nu red/black multiplicative Schwarz cycles with exact block inverses
    (dense algebra), started from x0."""
    x = x0.copy()
    masks = [blk.colour_mask_field(c).reshape(-1).astype(bool) for c in (0, 1)]
    for _ in range(nu):
        for m in masks:
            r = y - D @ x
            e = np.zeros_like(x)
            e[m] = np.linalg.solve(B[np.ix_(m, m)], r[m])
            x = x + e
    return x


@pytest.mark.parametrize("nu", [1, 3])
def test_vcycle_composition_dense(nu):
    """Pin of Alg. 1 (with Alg. 2 and Alg. 3): the coarse-grid correction
    is x0 = P (R D P)^{-1} R y, and the smoother starts from it:
    x = S^nu(y; x0).  Both checked against dense algebra with exact block
    and coarse solves.  Two wrong compositions miss by far: the smoother
    from zero without the correction, and the correction applied after the
    smoother instead of before it."""
    M, shp, D, B, R, P = _dense_vcycle_case(nu)
    y = synth.gaussian_spinors(M.p.L, 1, 65)[0]
    yv = y.reshape(-1)
    Dc = R @ D @ P
    x0 = P @ np.linalg.solve(Dc, R @ yv)
    assert relerr(M.cgc(y).reshape(-1), x0) < 1e-11
    want = _schwarz(M.blk, D, B, yv, x0, nu)
    got = M.vcycle(y).reshape(-1)
    assert relerr(got, want) < 1e-10
    # teeth: no coarse-grid correction at all
    no_cgc = _schwarz(M.blk, D, B, yv, np.zeros_like(yv), nu)
    assert relerr(got, no_cgc) > 1e-3
    # teeth: the correction after the smoother (post- instead of pre-smoothing order)
    post = no_cgc + P @ np.linalg.solve(Dc, R @ (yv - D @ no_cgc))
    assert relerr(got, post) > 1e-3
