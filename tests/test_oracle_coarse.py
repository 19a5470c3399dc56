"""Pins of the oracle's aggregates, R/P, D_c and coarse solve (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import dirac, sap, coarse
from helpers import dense_from_apply, relerr

L = (4, 4, 4, 4)
BLK = (2, 2, 2, 2)
NTV = 6


@pytest.fixture(scope="module")
def c1():
    U = synth.su3_field(L, 0.3, 101)
    A = dirac.clover_term(U, -0.1, 1.0)
    blk = sap.Blocking(L, BLK)
    V = synth.gaussian_spinors(L, NTV, 102)
    W = coarse.orthonormalise(blk, V)
    Dc = coarse.coarse_operator(U, A, blk, W)
    return U, A, blk, V, W, Dc


def _RP_dense(blk, W):
    shp = (L[3], L[2], L[1], L[0], 4, 3)
    R = dense_from_apply(lambda y: coarse.restrict(blk, W, y), shp)
    P = dense_from_apply(lambda xc: coarse.prolong(blk, W, xc), (blk.nblocks, 2, W.shape[0]))
    return R, P


def test_orthonormalise_equals_numpy_qr(c1):
    U, A, blk, V, W, Dc = c1
    X = np.moveaxis(coarse.chirality_split(blk, V), 0, -1)    # (Nb, 2, n, Ntv)
    Wa = np.moveaxis(coarse.chirality_split(blk, W), 0, -1)
    for b in (0, 5, blk.nblocks - 1):
        for h in (0, 1):
            Q, T = np.linalg.qr(X[b, h])
            ph = np.diag(T) / np.abs(np.diag(T))                # fix diag(T) > 0
            Q = Q * ph[None, :]
            assert np.abs(Q - Wa[b, h]).max() < 1e-13


def test_chirality_split_layout(c1):
    _, _, blk, V, _, _ = c1
    s = coarse.chirality_split(blk, V)
    bv = blk.block_view(V)                                      # (Ntv, Nb, Vb, 4, 3)
    # element n = (site_in_block * 2 + spin_within_h) * 3 + colour
    assert s[2, 7, 1, (5 * 2 + 1) * 3 + 2] == bv[2, 7, 5, 3, 2]
    assert s[2, 7, 0, (5 * 2 + 0) * 3 + 1] == bv[2, 7, 5, 0, 1]
    assert np.array_equal(coarse.chirality_merge(blk, s), V)


def test_R_P_identities(c1):
    U, A, blk, V, W, Dc = c1
    R, P = _RP_dense(blk, W)
    nc = blk.nblocks * 2 * NTV
    assert np.abs(P - R.conj().T).max() == 0.0
    assert np.abs(R @ P - np.eye(nc)).max() < 1e-13
    PR = P @ R
    assert np.abs(PR - PR.conj().T).max() < 1e-14
    assert np.abs(PR @ PR - PR).max() < 1e-13
    for j in range(NTV):
        v = V[j].reshape(-1)
        assert relerr(PR @ v, v) < 1e-13


def test_coarse_operator_equals_dense_galerkin(c1):
    U, A, blk, V, W, Dc = c1
    R, P = _RP_dense(blk, W)
    shp = (L[3], L[2], L[1], L[0], 4, 3)
    nc = P.shape[1]
    # D P column by column, then R: the dense Galerkin product R D P
    DP = np.array([dirac.apply_D(U, A, P[:, k].reshape(shp)).reshape(-1) for k in range(nc)]).T
    G = R @ DP
    nbr = coarse.neighbour_table(blk)
    Cd = dense_from_apply(lambda x: coarse.coarse_apply(Dc, nbr, x.reshape(blk.nblocks, -1)),
                          (blk.nblocks, 2 * NTV))
    assert np.abs(G - Cd).max() < 1e-12 * np.abs(G).max()


def test_coarse_operator_dagger_symmetry(c1):
    """Eq. (dagger): backward couplings are the Gamma5_c-adjoint of forward ones."""
    U, A, blk, V, W, Dc = c1
    nbr = coarse.neighbour_table(blk)
    g5c = np.diag(np.r_[-np.ones(NTV), np.ones(NTV)])
    for mu in range(4):
        for i in range(blk.nblocks):
            j = nbr[i, 1 + 2 * mu]
            fwd = Dc[i, 1 + 2 * mu]
            bwd = Dc[j, 2 + 2 * mu]
            assert np.abs(bwd - g5c @ fwd.conj().T @ g5c).max() < 1e-13
    # self blocks: same-chirality parts Hermitian, and Gamma5_c-Hermitian overall
    for i in range(blk.nblocks):
        S = Dc[i, 0]
        assert np.abs(S[:NTV, :NTV] - S[:NTV, :NTV].conj().T).max() < 1e-13
        assert np.abs(S - g5c @ S.conj().T @ g5c).max() < 1e-13


def test_coarse_operator_zero_beyond_neighbours(c1):
    """Blocks that are not face neighbours do not couple: the dense Galerkin
    product vanishes outside the 9-slot pattern (checked on a lattice with
    block-lattice extent 4 in x so that x-next-nearest blocks exist)."""
    Lb = (8, 4, 4, 4)
    U = synth.su3_field(Lb, 0.3, 111)
    A = dirac.clover_term(U, -0.1, 1.0)
    blk = sap.Blocking(Lb, BLK)
    W = coarse.orthonormalise(blk, synth.gaussian_spinors(Lb, 2, 112))
    shp = (Lb[3], Lb[2], Lb[1], Lb[0], 4, 3)
    nbr = coarse.neighbour_table(blk)
    Dc = coarse.coarse_operator(U, A, blk, W)
    for j in (0, 3):
        for col in range(4):
            e = np.zeros((blk.nblocks, 2, 2), dtype=complex)
            e.reshape(blk.nblocks, 4)[j, col] = 1.0
            out = coarse.restrict(blk, W, dirac.apply_D(U, A, coarse.prolong(blk, W, e)))
            out = out.reshape(blk.nblocks, 4)
            touched = set(np.nonzero(np.abs(out).max(axis=1) > 1e-14)[0])
            allowed = set(int(i) for i in range(blk.nblocks) if j in nbr[i])
            assert touched <= allowed
            ref = coarse.coarse_apply(Dc, nbr, e.reshape(blk.nblocks, 4))
            assert np.abs(out - ref).max() < 1e-13


def test_coarse_solve_exact_matches_dense(c1):
    U, A, blk, V, W, Dc = c1
    nbr = coarse.neighbour_table(blk)
    n = 2 * NTV
    Cd = dense_from_apply(lambda x: coarse.coarse_apply(Dc, nbr, x.reshape(blk.nblocks, -1)),
                          (blk.nblocks, n))
    yc = synth.gaussian_coarse(blk.nblocks, NTV, 1, 121)[0]
    cs = coarse.CoarseSolver(blk, Dc, tol=1e-14, restart=30, maxit=500)
    xc = cs.solve(yc)
    xd = np.linalg.solve(Cd, yc.reshape(-1))
    assert relerr(xc.reshape(-1), xd) < 1e-10


def test_coarse_solve_tolerance_and_schur_identity(c1):
    """With x_e from the back-substitution the full coarse residual equals
    (0, b_o - S x_o) and the stop rule bounds it by 0.05 ||y_c||."""
    U, A, blk, V, W, Dc = c1
    nbr = coarse.neighbour_table(blk)
    yc = synth.gaussian_coarse(blk.nblocks, NTV, 1, 122)[0]
    cs = coarse.CoarseSolver(blk, Dc, tol=0.05)
    xc = cs.solve(yc)
    y = yc.reshape(blk.nblocks, -1)
    r = y - coarse.coarse_apply(Dc, nbr, xc.reshape(blk.nblocks, -1))
    assert np.abs(r[cs.even]).max() < 1e-13 * np.abs(y).max()
    assert np.linalg.norm(r) <= 0.05 * np.linalg.norm(y) * (1 + 1e-12)
    assert cs.last_its >= 1
    # the Schur residual of the returned x_o is exactly the odd residual
    xo = xc.reshape(blk.nblocks, -1)[cs.odd]
    bo = y[cs.odd] - cs.D_oe(cs.Dee_solve(y[cs.even]))
    assert relerr(bo - cs.schur(xo), r[cs.odd]) < 1e-12


def test_coarse_gmres_textbook():
    """The GMRES routine on a dense random system: fixed iterations equal the
    minimal-residual solution over the Krylov space (numpy lstsq)."""
    rng = np.random.default_rng(7)
    n = 40
    M = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    k = 7
    x, its = coarse.gmres(lambda v: M @ v, b, np.zeros(n, complex), 0.0, 30, 100, fixed_its=k)
    K = np.array([np.linalg.matrix_power(M, j) @ b for j in range(k)]).T
    c, *_ = np.linalg.lstsq(M @ K, b, rcond=None)
    assert its == k
    assert relerr(x, K @ c) < 1e-10
    # restarted: 2 cycles of 4 equal two sequential minimal-residual steps
    x1, _ = coarse.gmres(lambda v: M @ v, b, np.zeros(n, complex), 0.0, 4, 8, fixed_its=8)
    xa, _ = coarse.gmres(lambda v: M @ v, b, np.zeros(n, complex), 0.0, 4, 4, fixed_its=4)
    r = b - M @ xa
    K2 = np.array([np.linalg.matrix_power(M, j) @ r for j in range(4)]).T
    c2, *_ = np.linalg.lstsq(M @ K2, r, rcond=None)
    assert relerr(x1, xa + K2 @ c2) < 1e-10


def test_cgc_projection(c1):
    """With an exact coarse solve the CGC is a Galerkin projection:
    R (y - D P D_c^{-1} R y) = 0 and T = I - P D_c^{-1} R D is idempotent."""
    U, A, blk, V, W, Dc = c1
    cs = coarse.CoarseSolver(blk, Dc, tol=1e-14, restart=60, maxit=1000)
    y = synth.gaussian_spinors(L, 1, 131)[0]
    def cgc(v):
        return coarse.prolong(blk, W, cs.solve(coarse.restrict(blk, W, v)))
    x = cgc(y)
    r = y - dirac.apply_D(U, A, x)
    assert np.linalg.norm(coarse.restrict(blk, W, r)) < 1e-11 * np.linalg.norm(y)
    e = synth.gaussian_spinors(L, 1, 132)[0]
    T = lambda v: v - cgc(dirac.apply_D(U, A, v))
    Te = T(e)
    assert relerr(T(Te), Te) < 1e-10
