"""Wilson-clover Dirac operator in FP64 (oracle; test infrastructure only).

The paper solves D u = f for the Wilson-clover operator (Sec. 1) and writes
its structure in Alg. 7: nearest-neighbour hops (1 +- gamma_mu) U and a
clover term C^{hh}(x) that is diagonal in chirality h.  It fixes neither the
normalisation nor the gamma basis; the reading used here (also used by the
GPU library, each written separately) is

  (D psi)(x) = A(x) psi(x)
             - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
                          + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
  A(x) = (4 + m0) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x)
  sigma_{mu nu} = (i/2) [g_mu, g_nu],  F = (Q - Q^dag)/8,
  Q_{mu nu}(x) = sum of the four plaquette leaves at x (same orientation).

Space is periodic, time antiperiodic: a fermion hop across the t boundary
picks up a factor -1 (links are periodic).  Gamma matrices: Euclidean,
Hermitian, chiral basis with g5 = g1 g2 g3 g4 = diag(-1, -1, +1, +1), so the
left-handed aggregate holds spins {0, 1} and the right-handed one {2, 3}.

Spinor fields have shape (..., Lt, Lz, Ly, Lx, 4, 3); links (Lt, Lz, Ly, Lx,
4, 3, 3).
"""
import numpy as np

_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def _gammas():
    Z = np.zeros((2, 2), dtype=np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    g = [np.block([[Z, -1j * s], [1j * s, Z]]) for s in _SIGMA]
    g.append(np.block([[Z, -I2], [-I2, Z]]))
    return tuple(g)


GAMMA = _gammas()
G5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

# lattice axis of direction mu, counted from the end of a spinor field
# (..., t, z, y, x, spin, colour) or a single-direction link field (..., 3, 3)
_AX = (-3, -4, -5, -6)


def shift_fwd(f, mu, antiperiodic=True):
    """f(x + mu) with the fermion boundary condition (sign on the t wrap)."""
    g = np.roll(f, -1, axis=_AX[mu])
    if mu == 3 and antiperiodic:
        g[..., -1, :, :, :, :, :] *= -1.0
    return g


def shift_bwd(f, mu, antiperiodic=True):
    """f(x - mu) with the fermion boundary condition (sign on the t wrap)."""
    g = np.roll(f, 1, axis=_AX[mu])
    if mu == 3 and antiperiodic:
        g[..., 0, :, :, :, :, :] *= -1.0
    return g


def link_fwd(Umu, mu):
    """U_mu(x + mu) for one direction's links (periodic)."""
    return np.roll(Umu, -1, axis=_AX[mu])


def link_bwd(Umu, mu):
    """U_mu(x - mu) for one direction's links (periodic)."""
    return np.roll(Umu, 1, axis=_AX[mu])


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _colour(U, psi):
    """U acting on the colour index of psi (site by site)."""
    return np.einsum('...ab,...sb->...sa', U, psi)


def _spin(G, psi):
    return np.einsum('st,...tc->...sc', G, psi)


def clover_leaves(U, mu, nu):
    """Q_{mu nu}(x): sum of the four plaquettes in the (mu, nu) plane at x."""
    Um, Un = U[..., mu, :, :], U[..., nu, :, :]
    Um_pn = link_fwd(Um, nu)                 # U_mu(x+nu)
    Un_pm = link_fwd(Un, mu)                 # U_nu(x+mu)
    Um_mm = link_bwd(Um, mu)                 # U_mu(x-mu)
    Un_mm = link_bwd(Un, mu)                 # U_nu(x-mu)
    Um_mn = link_bwd(Um, nu)                 # U_mu(x-nu)
    Un_mn = link_bwd(Un, nu)                 # U_nu(x-nu)
    Um_mm_pn = link_fwd(Um_mm, nu)           # U_mu(x-mu+nu)
    Um_mm_mn = link_bwd(Um_mm, nu)           # U_mu(x-mu-nu)
    Un_mm_mn = link_bwd(Un_mm, nu)           # U_nu(x-mu-nu)
    Un_mn_pm = link_fwd(Un_mn, mu)           # U_nu(x-nu+mu)
    q = Um @ Un_pm @ _dag(Um_pn) @ _dag(Un)
    q = q + Un @ _dag(Um_mm_pn) @ _dag(Un_mm) @ Um_mm
    q = q + _dag(Um_mm) @ _dag(Un_mm_mn) @ Um_mm_mn @ Un_mn
    q = q + _dag(Un_mn) @ Um_mn @ Un_mn_pm @ _dag(Um)
    return q


def clover_term(U, m0, csw):
    """A(x) as a full 12x12 matrix per site: shape (Lt, Lz, Ly, Lx, 4, 3, 4, 3)."""
    shp = U.shape[:4]
    A = np.zeros(shp + (4, 3, 4, 3), dtype=np.complex128)
    eye3 = np.eye(3, dtype=np.complex128)
    A += (4.0 + m0) * np.einsum('st,ab->satb', np.eye(4), eye3)
    if csw != 0.0:
        for mu in range(4):
            for nu in range(4):
                if mu == nu:
                    continue
                Q = clover_leaves(U, mu, nu)
                F = (Q - _dag(Q)) / 8.0
                sig = 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
                A += csw * 0.25j * np.einsum('st,...ab->...satb', sig, F)
    return A


def apply_clover(A, psi):
    return np.einsum('...satb,...tb->...sa', A, psi)


def hopping(U, psi, fwd_mask=None, bwd_mask=None):
    """sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)].

    Optional 0/1 masks per direction (arrays over (Lt, Lz, Ly, Lx)) keep only
    selected hops; they weight the hop by the mask at the target site x.
    """
    out = np.zeros(np.broadcast_shapes(psi.shape), dtype=np.complex128)
    for mu in range(4):
        Umu = U[..., mu, :, :]
        a = _colour(Umu, shift_fwd(psi, mu))
        a = a - _spin(GAMMA[mu], a)
        if fwd_mask is not None:
            a = a * fwd_mask[mu][..., None, None]
        b = _colour(_dag(link_bwd(Umu, mu)), shift_bwd(psi, mu))
        b = b + _spin(GAMMA[mu], b)
        if bwd_mask is not None:
            b = b * bwd_mask[mu][..., None, None]
        out += a + b
    return out


def apply_D(U, A, psi):
    """D psi for the Wilson-clover operator (Sec. 1; hop structure of Alg. 7)."""
    return apply_clover(A, psi) - 0.5 * hopping(U, psi)


def apply_g5(psi):
    return _spin(G5, psi)


def coords(L):
    """Integer coordinate arrays x, y, z, t of shape (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly),
                             np.arange(Lx), indexing='ij')
    return (x, y, z, t)


def block_hop_masks(L, block):
    """Masks selecting hops that stay inside a block (the operator B of Alg. 3)
    and hops that cross a block face (the operator Z), per direction.

    Returns (in_fwd, in_bwd, cross_fwd, cross_bwd), each a list of 4 float
    arrays over (Lt, Lz, Ly, Lx); the mask is evaluated at the site x that
    receives the hop.
    """
    c = coords(L)
    in_fwd, in_bwd, cr_fwd, cr_bwd = [], [], [], []
    for mu in range(4):
        r = c[mu] % block[mu]
        f = (r != block[mu] - 1).astype(np.float64)
        b = (r != 0).astype(np.float64)
        in_fwd.append(f)
        in_bwd.append(b)
        cr_fwd.append(1.0 - f)
        cr_bwd.append(1.0 - b)
    return in_fwd, in_bwd, cr_fwd, cr_bwd


def apply_B(U, A, psi, L, block):
    """Block operator B: D with every hop that leaves its block dropped
    (Dirichlet truncation), i.e. the couplings within blocks of Alg. 3."""
    in_fwd, in_bwd, _, _ = block_hop_masks(L, block)
    return apply_clover(A, psi) - 0.5 * hopping(U, psi, in_fwd, in_bwd)


def _wrap(c, L):
    return tuple(int(c[i]) % L[i] for i in range(4))


def apply_D_sites(U, m0, csw, psi, sites):
    """(D psi)(x) at the listed sites only (the same operator as apply_D,
    computed site by site from its definition: clover term from the four
    leaves at x, then the eight hops with the sign on the t wrap).  For
    sampled checks on lattices too large for the full-field routines.

    sites: integer array (n, 4) of (x, y, z, t); returns (n, 4, 3)."""
    Lt, Lz, Ly, Lx = U.shape[:4]
    L = (Lx, Ly, Lz, Lt)

    def link(mu, c):
        x, y, z, t = _wrap(c, L)
        return U[t, z, y, x, mu]

    def field(c):
        x, y, z, t = c
        sign = -1.0 if (t < 0 or t >= Lt) else 1.0
        x, y, z, t = _wrap(c, L)
        return sign * psi[t, z, y, x]

    def step(c, mu, d):
        e = list(c)
        e[mu] += d
        return e

    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for n, c0 in enumerate(np.asarray(sites)):
        c = [int(v) for v in c0]
        A = (4.0 + m0) * np.eye(12, dtype=np.complex128)
        if csw != 0.0:
            for mu in range(4):
                for nu in range(4):
                    if mu == nu:
                        continue
                    pm, pn, mm, mn = step(c, mu, 1), step(c, nu, 1), step(c, mu, -1), step(c, nu, -1)
                    q = link(mu, c) @ link(nu, pm) @ _dag(link(mu, pn)) @ _dag(link(nu, c))
                    q = q + link(nu, c) @ _dag(link(mu, step(pn, mu, -1))) @ _dag(link(nu, mm)) @ link(mu, mm)
                    q = q + (_dag(link(mu, mm)) @ _dag(link(nu, step(mm, nu, -1))) @ link(mu, step(mm, nu, -1))
                             @ link(nu, mn))
                    q = q + _dag(link(nu, mn)) @ link(mu, mn) @ link(nu, step(mn, mu, 1)) @ _dag(link(mu, c))
                    F = (q - _dag(q)) / 8.0
                    sig = 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
                    A += csw * 0.25j * np.kron(sig, F)
        v = A @ psi[c[3] % Lt, c[2] % Lz, c[1] % Ly, c[0] % Lx].reshape(12)
        hop = np.zeros((4, 3), dtype=np.complex128)
        for mu in range(4):
            f = field(step(c, mu, 1))
            a = f @ link(mu, c).T                 # U_mu(x) psi(x+mu), colour index last
            hop += a - GAMMA[mu] @ a
            b = field(step(c, mu, -1)) @ np.conj(link(mu, step(c, mu, -1)))  # U_mu(x-mu)^dag psi(x-mu)
            hop += b + GAMMA[mu] @ b
        out[n] = v.reshape(4, 3) - 0.5 * hop
    return out
