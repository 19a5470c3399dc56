"""Pins of the oracle's Wilson-clover operator against closed forms and
invariants (no GPU).  The paper fixes the operator only through its hopping
structure (Alg. 7) and the chirality-diagonal clover blocks; these tests pin
the reading (normalisation, signs, gamma basis, boundary conditions)."""
import numpy as np
import pytest

import synth
from oracle import dirac
from helpers import dense_from_apply, relerr


def test_gamma_basis():
    G = dirac.GAMMA
    for m in range(4):
        assert np.allclose(G[m], G[m].conj().T)
        for n in range(4):
            assert np.allclose(G[m] @ G[n] + G[n] @ G[m], 2.0 * (m == n) * np.eye(4))
    # chiral basis: g5 = diag(-1, -1, +1, +1) (left-handed = spins 0, 1)
    assert np.allclose(dirac.G5, np.diag([-1.0, -1.0, 1.0, 1.0]))


def _free_spectrum(L, m0):
    lam = []
    for nx in range(L[0]):
        for ny in range(L[1]):
            for nz in range(L[2]):
                for nt in range(L[3]):
                    p = [2 * np.pi * nx / L[0], 2 * np.pi * ny / L[1], 2 * np.pi * nz / L[2],
                         np.pi * (2 * nt + 1) / L[3]]
                    a = m0 + sum(1 - np.cos(q) for q in p)
                    b = np.sqrt(sum(np.sin(q) ** 2 for q in p))
                    lam += [a + 1j * b] * 6 + [a - 1j * b] * 6
    return np.array(lam)


@pytest.mark.parametrize("L", [(2, 2, 2, 4), (4, 2, 2, 2), (2, 4, 2, 4)])
def test_free_field_spectrum(L):
    m0 = -0.1
    U = synth.unit_field(L)
    A = dirac.clover_term(U, m0, 1.0)
    shape = (L[3], L[2], L[1], L[0], 4, 3)
    D = dense_from_apply(lambda p: dirac.apply_D(U, A, p), shape)
    ev = np.linalg.eigvals(D)
    lam = _free_spectrum(L, m0)
    used = np.zeros(len(lam), bool)
    dev = 0.0
    for e in ev:
        d = np.abs(lam - e)
        d[used] = np.inf
        k = int(np.argmin(d))
        used[k] = True
        dev = max(dev, d[k])
    assert dev < 1e-12


def test_free_field_plane_wave():
    """A plane wave with antiperiodic-allowed momentum is mapped to D(p) psi
    with D(p) = m0 + sum(1 - cos p) + i sum gamma sin p."""
    L = (4, 4, 4, 4)
    m0 = -0.2
    U = synth.unit_field(L)
    A = dirac.clover_term(U, m0, 1.0)
    n = (1, 3, 2, 0)
    p = [2 * np.pi * n[0] / 4, 2 * np.pi * n[1] / 4, 2 * np.pi * n[2] / 4, np.pi * (2 * n[3] + 1) / 4]
    x, y, z, t = dirac.coords(L)
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(5)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[..., None, None] * chi
    Dp = (m0 + sum(1 - np.cos(q) for q in p)) * np.eye(4)
    for mu in range(4):
        Dp = Dp + 1j * np.sin(p[mu]) * dirac.GAMMA[mu]
    expect = phase[..., None, None] * (Dp @ chi)
    assert relerr(dirac.apply_D(U, A, psi), expect) < 1e-13


def test_gamma5_hermiticity_dense():
    L = (2, 2, 2, 4)
    U = synth.su3_field(L, 0.5, 11)
    A = dirac.clover_term(U, -0.2, 1.0)
    shape = (L[3], L[2], L[1], L[0], 4, 3)
    D = dense_from_apply(lambda p: dirac.apply_D(U, A, p), shape)
    G5 = np.kron(np.eye(np.prod(L)), np.kron(dirac.G5, np.eye(3)))
    assert np.abs(G5 @ D @ G5 - D.conj().T).max() < 1e-13


def test_gamma5_hermiticity_inner_products():
    L = (4, 4, 4, 4)
    U = synth.su3_field(L, 0.5, 12)
    A = dirac.clover_term(U, -0.2, 1.0)
    x, y = synth.gaussian_spinors(L, 2, 13)
    lhs = np.vdot(x, dirac.apply_g5(dirac.apply_D(U, A, dirac.apply_g5(y))))
    rhs = np.vdot(dirac.apply_D(U, A, x), y)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13


def test_gauge_covariance():
    L = (4, 4, 2, 4)
    U = synth.su3_field(L, 0.5, 21)
    g = synth.random_su3_gauge_transform(L, 22)
    Ug = np.empty_like(U)
    for mu in range(4):
        gf = dirac.link_fwd(g, mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gf, -1, -2))
    A = dirac.clover_term(U, -0.2, 1.0)
    Ag = dirac.clover_term(Ug, -0.2, 1.0)
    psi = synth.gaussian_spinors(L, 1, 23)[0]
    gpsi = np.einsum('...ab,...sb->...sa', g, psi)
    lhs = dirac.apply_D(Ug, Ag, gpsi)
    rhs = np.einsum('...ab,...sb->...sa', g, dirac.apply_D(U, A, psi))
    assert relerr(lhs, rhs) < 1e-13


def test_clover_structure():
    L = (4, 4, 4, 4)
    U = synth.su3_field(L, 0.5, 31)
    m0 = -0.2
    A = dirac.clover_term(U, m0, 1.0).reshape(-1, 12, 12)
    assert np.abs(A - A.conj().transpose(0, 2, 1)).max() < 1e-14
    assert np.abs(A[:, :6, 6:]).max() == 0.0 and np.abs(A[:, 6:, :6]).max() == 0.0
    # linear in c_sw, (4 + m0) at c_sw = 0, no clover for the free field
    A2 = dirac.clover_term(U, m0, 2.0).reshape(-1, 12, 12)
    A0 = dirac.clover_term(U, m0, 0.0).reshape(-1, 12, 12)
    assert np.allclose(A0, (4 + m0) * np.eye(12), atol=0, rtol=0)
    assert np.abs((A2 - A0) - 2 * (A - A0)).max() < 1e-14
    Af = dirac.clover_term(synth.unit_field(L), m0, 1.0).reshape(-1, 12, 12)
    assert np.abs(Af - (4 + m0) * np.eye(12)).max() < 1e-15
    # flipping the sign of all time links on one time slice changes no plaquette
    Uf = U.copy()
    Uf[-1, :, :, :, 3] *= -1.0
    Afl = dirac.clover_term(Uf, m0, 1.0).reshape(-1, 12, 12)
    assert np.abs(Afl - A).max() < 1e-14


@pytest.mark.parametrize("plane", [(0, 1), (1, 3), (2, 3)])
def test_clover_constant_abelian_field(plane):
    """Constant field strength theta in one plane, embedded in the colour
    diagonal as diag(q) with charges q = (1, -1, 0): every plaquette leaf is
    diag(exp(i q theta)), so F = i sin(q theta) and the clover term is
    (4 + m0) - (c_sw/2) sin(q theta) sigma_{mu nu} exactly.  In the chiral
    basis sigma_{k4} = diag(-s_k, s_k) and sigma_{12} = -diag(s_3, s_3) with
    Pauli matrices s_k; those values are written out by hand below."""
    mu, nu = plane
    L = (4, 4, 4, 4)
    theta = 2 * np.pi / L[mu]
    U = synth.unit_field(L)
    c = dirac.coords(L)
    q = np.array([1.0, -1.0, 0.0])
    ph = np.exp(1j * theta * c[mu][..., None] * q)       # U_nu(x) = diag(e^{i q theta x_mu})
    U[..., nu, :, :] = ph[..., :, None] * np.eye(3)
    m0, csw = -0.2, 1.3
    A = dirac.clover_term(U, m0, csw)
    # closed form for sigma_{mu nu} in the chiral basis, written out by hand
    sig_hand = {
        (0, 1): -np.diag([1, -1, 1, -1]).astype(complex),
        (1, 3): np.array([[0, 1j, 0, 0], [-1j, 0, 0, 0], [0, 0, 0, -1j], [0, 0, 1j, 0]]),
        (2, 3): np.diag([-1, 1, 1, -1]).astype(complex),
    }[plane]
    expect = (4 + m0) * np.eye(12, dtype=complex) - 0.5 * csw * np.kron(sig_hand, np.diag(np.sin(q * theta)))
    got = A.reshape(-1, 12, 12)
    assert np.abs(got - expect).max() < 1e-13


def test_generator_su3():
    U = synth.su3_field((4, 4, 2, 2), 0.5, 41).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # mean plaquette trace decreases with disorder
    def plaq(eps):
        Uf = synth.su3_field((4, 4, 4, 4), eps, 42)
        Q = dirac.clover_leaves(Uf, 0, 1)
        return np.mean(np.trace(Q, axis1=-2, axis2=-1).real) / 12
    assert plaq(0.1) > plaq(0.3) > plaq(0.5)


def test_site_local_operator_matches_full_operator():
    """apply_D_sites (site by site from the definition) equals apply_D at
    every site of a lattice with an odd-sized t extent (boundary signs and
    clover leaves across every wrap)."""
    L = (4, 2, 2, 6)
    U = synth.su3_field(L, 0.7, 41)
    psi = synth.gaussian_spinors(L, 1, 42)[0]
    A = dirac.clover_term(U, -0.3, 1.3)
    ref = dirac.apply_D(U, A, psi)
    sites = np.array([(x, y, z, t) for t in range(L[3]) for z in range(L[2]) for y in range(L[1])
                      for x in range(L[0])])
    out = dirac.apply_D_sites(U, -0.3, 1.3, psi, sites)
    full = np.array([ref[t, z, y, x] for x, y, z, t in sites])
    assert np.abs(out - full).max() <= 1e-13 * np.abs(full).max()
