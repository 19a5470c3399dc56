"""Pins of the oracle's block MR solver and SAP smoother (no GPU)."""
import numpy as np

import synth
from oracle import dirac, sap
from helpers import dense_from_apply, relerr

L = (4, 4, 4, 4)
BLK = (2, 2, 2, 2)


def _setup(eps=0.5, seed=51):
    U = synth.su3_field(L, eps, seed)
    A = dirac.clover_term(U, -0.2, 1.0)
    return U, A, sap.Blocking(L, BLK)


def test_blocking_roundtrip_and_colours():
    blk = sap.Blocking((4, 8, 4, 4), (2, 4, 2, 2))
    f = synth.gaussian_spinors(blk.L, 2, 1)
    assert np.array_equal(blk.field_view(blk.block_view(f)), f)
    # the block view groups exactly the sites of each block
    x, y, z, t = dirac.coords(blk.L)
    bid = (x // 2) + 2 * ((y // 4) + 2 * ((z // 2) + 2 * (t // 2)))
    g = np.zeros(blk.L[::-1] + (4, 3))
    g[...] = bid[..., None, None]
    gv = blk.block_view(g)
    assert np.all(gv == np.arange(blk.nblocks)[:, None, None, None])
    # colours alternate between face neighbours
    col = blk.block_colour().reshape(blk.NB[::-1])
    for ax in range(4):
        assert np.all(col != np.roll(col, 1, axis=ax))


def test_block_operator_is_block_diagonal_part_of_D():
    U, A, blk = _setup()
    shape = (L[3], L[2], L[1], L[0], 4, 3)
    Ls = (4, 4, 2, 2)
    Us = synth.su3_field(Ls, 0.5, 52)
    As = dirac.clover_term(Us, -0.2, 1.0)
    shp = (Ls[3], Ls[2], Ls[1], Ls[0], 4, 3)
    D = dense_from_apply(lambda p: dirac.apply_D(Us, As, p), shp)
    B = dense_from_apply(lambda p: dirac.apply_B(Us, As, p, Ls, (2, 2, 1, 1)), shp)
    x, y, z, t = dirac.coords(Ls)
    bid = ((x // 2) + 2 * ((y // 2) + 2 * (z + 2 * t))).reshape(-1)
    same = (bid[:, None] == bid[None, :])
    same12 = np.kron(same, np.ones((12, 12))).astype(bool)
    assert np.abs(B - np.where(same12, D, 0)).max() < 1e-15
    del shape, U, A, blk


def test_mr_orthogonality_and_monotone():
    U, A, blk = _setup()
    r = synth.gaussian_spinors(L, 1, 53)[0]
    rho = r.copy()
    prev = sap.block_dot(blk, rho, rho).real
    for _ in range(5):
        q = dirac.apply_B(U, A, rho, L, BLK)
        _, rho_new = sap.mr_blocks(U, A, blk, rho, 1)
        # MR step: the new residual is orthogonal to B rho, block by block
        assert np.abs(sap.block_dot(blk, q, rho_new)).max() < 1e-12 * np.sqrt(prev.max())
        cur = sap.block_dot(blk, rho_new, rho_new).real
        assert np.all(cur <= prev * (1 + 1e-14))
        prev, rho = cur, rho_new


def test_mr_residual_consistent():
    U, A, blk = _setup()
    r = synth.gaussian_spinors(L, 1, 54)[0]
    e, rho = sap.mr_blocks(U, A, blk, r, 4)
    assert relerr(r - dirac.apply_B(U, A, e, L, BLK), rho) < 1e-13


def _cut_links(U):
    """Zero the links that cross a block face, so that D = B."""
    Uc = U.copy()
    c = dirac.coords(L)
    for mu in range(4):
        face = (c[mu] % BLK[mu]) == BLK[mu] - 1
        Uc[..., mu, :, :][face] = 0.0
    return Uc


def test_sap_exact_when_blocks_decouple():
    """With the inter-block links cut, D = B; many MR steps solve each block,
    so one SAP cycle returns D^{-1} y (checked by the residual)."""
    U, _, blk = _setup()
    Uc = _cut_links(U)
    A = dirac.clover_term(U, -0.2, 1.0)       # clover of the uncut field
    y = synth.gaussian_spinors(L, 1, 55)[0]
    x = sap.sap(Uc, A, blk, y, np.zeros_like(y), 1, 80)
    r = y - dirac.apply_D(Uc, A, x)
    assert np.linalg.norm(r) / np.linalg.norm(y) < 1e-10


def test_sap_matches_schwarz_formula():
    """With exact block solves, one SAP cycle is
    x1 = x0 + K0 (y - D x0),  x2 = x1 + K1 (y - D x1),
    K_c = (restriction to colour c of B)^{-1}, computed with dense algebra."""
    Ls = (4, 4, 2, 2)
    bs = (2, 2, 1, 1)
    U = synth.su3_field(Ls, 0.5, 56)
    A = dirac.clover_term(U, -0.2, 1.0)
    blk = sap.Blocking(Ls, bs)
    shp = (Ls[3], Ls[2], Ls[1], Ls[0], 4, 3)
    D = dense_from_apply(lambda p: dirac.apply_D(U, A, p), shp)
    B = dense_from_apply(lambda p: dirac.apply_B(U, A, p, Ls, bs), shp)
    y = synth.gaussian_spinors(Ls, 1, 57)[0].reshape(-1)
    x0 = synth.gaussian_spinors(Ls, 1, 58)[0].reshape(-1)
    x = x0.copy()
    for c in (0, 1):
        m = blk.colour_mask_field(c).reshape(-1).astype(bool)
        r = y - D @ x
        e = np.zeros_like(x)
        e[m] = np.linalg.solve(B[np.ix_(m, m)], r[m])
        x = x + e
    got = sap.sap(U, A, blk, y.reshape(shp), x0.reshape(shp), 1, 60).reshape(-1)
    assert relerr(got, x) < 1e-10


def test_sap_homogeneous_and_reduces_error():
    U, A, blk = _setup()
    y = synth.gaussian_spinors(L, 1, 59)[0]
    x = sap.sap(U, A, blk, y, np.zeros_like(y), 3, 4)
    x2 = sap.sap(U, A, blk, (2.5 - 1j) * y, np.zeros_like(y), 3, 4)
    assert relerr(x2, (2.5 - 1j) * x) < 1e-13
    r = y - dirac.apply_D(U, A, x)
    assert np.linalg.norm(r) < 0.5 * np.linalg.norm(y)
