"""Block minimal-residual solver and the SAP smoother (oracle; test only).

Alg. 3 of the paper writes the smoother as x <- x + B^{-1}(y - D x) with
D = B + Z (B: couplings inside blocks, Z: couplings between blocks) and notes
that in practice the Schwarz alternating procedure is used.  The reading
taken here is multiplicative red/black SAP: blocks are coloured by the parity
of the sum of their block coordinates, colour 0 ("red") first; in each colour
phase the residual y - D x is formed with the current x and every block of
that colour is corrected by an approximate block solve.  The block solve is
n_mr steps of minimal residual (MR) from a zero initial guess, with no
even/odd splitting inside the block.
"""
import numpy as np

from .dirac import apply_D, apply_B


class Blocking:
    """Block geometry: lattice L = (Lx, Ly, Lz, Lt), block extents b."""

    def __init__(self, L, block):
        self.L = tuple(int(v) for v in L)
        self.block = tuple(int(v) for v in block)
        for m in range(4):
            if self.L[m] % self.block[m]:
                raise ValueError('block extent must divide the lattice extent')
        self.NB = tuple(self.L[m] // self.block[m] for m in range(4))
        self.nblocks = int(np.prod(self.NB))
        self.vblock = int(np.prod(self.block))

    def block_view(self, f):
        """(..., Lt, Lz, Ly, Lx, 4, 3) -> (..., Nb, Vblock, 4, 3), block index
        bx + NBx (by + NBy (bz + NBz bt)), site-in-block in the same order."""
        Lx, Ly, Lz, Lt = self.L
        bx, by, bz, bt = self.block
        NBx, NBy, NBz, NBt = self.NB
        lead = f.shape[:-6]
        g = f.reshape(lead + (NBt, bt, NBz, bz, NBy, by, NBx, bx, 4, 3))
        k = len(lead)
        perm = list(range(k)) + [k + 0, k + 2, k + 4, k + 6, k + 1, k + 3, k + 5, k + 7, k + 8, k + 9]
        g = g.transpose(perm)
        return g.reshape(lead + (self.nblocks, self.vblock, 4, 3))

    def field_view(self, g):
        """Inverse of block_view."""
        Lx, Ly, Lz, Lt = self.L
        bx, by, bz, bt = self.block
        NBx, NBy, NBz, NBt = self.NB
        lead = g.shape[:-4]
        k = len(lead)
        h = g.reshape(lead + (NBt, NBz, NBy, NBx, bt, bz, by, bx, 4, 3))
        perm = list(range(k)) + [k + 0, k + 4, k + 1, k + 5, k + 2, k + 6, k + 3, k + 7, k + 8, k + 9]
        h = h.transpose(perm)
        return h.reshape(lead + (Lt, Lz, Ly, Lx, 4, 3))

    def block_coords(self):
        """Block coordinates (Bx, By, Bz, Bt), each an array over blocks."""
        NBx, NBy, NBz, NBt = self.NB
        bt, bz, by, bx = np.meshgrid(np.arange(NBt), np.arange(NBz), np.arange(NBy),
                                     np.arange(NBx), indexing='ij')
        return tuple(a.reshape(-1) for a in (bx, by, bz, bt))

    def block_colour(self):
        """Colour (sum of block coordinates) mod 2 of every block."""
        return np.sum(np.stack(self.block_coords()), axis=0) % 2

    def colour_mask_field(self, colour):
        """0/1 field over sites: 1 on blocks of the given colour."""
        m = (self.block_colour() == colour).astype(np.float64)
        g = np.broadcast_to(m[:, None, None, None], (self.nblocks, self.vblock, 4, 3))
        return self.field_view(np.ascontiguousarray(g))


def block_dot(blk, a, b):
    """Per-block inner products <a, b>_block = sum conj(a) b, shape (..., Nb)."""
    return np.sum(np.conj(blk.block_view(a)) * blk.block_view(b), axis=(-1, -2, -3))


def _per_block(blk, s):
    """Broadcast per-block scalars (..., Nb) back to a field."""
    g = np.broadcast_to(s[..., None, None, None], s.shape + (blk.vblock, 4, 3))
    return blk.field_view(np.ascontiguousarray(g))


def mr_blocks(U, A, blk, r, n_mr):
    """n_mr minimal-residual steps on B e = r, every block independently,
    zero initial guess: q = B rho, alpha = (q^H rho)/(q^H q), e += alpha rho,
    rho -= alpha q.  Blocks where q = 0 take alpha = 0.  Returns (e, rho)."""
    e = np.zeros_like(r)
    rho = r.copy()
    for _ in range(n_mr):
        q = apply_B(U, A, rho, blk.L, blk.block)
        qq = block_dot(blk, q, q).real
        qr = block_dot(blk, q, rho)
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1.0), 0.0)
        af = _per_block(blk, alpha)
        e = e + af * rho
        rho = rho - af * q
    return e, rho


def sap(U, A, blk, y, x0, nu, n_mr):
    """nu cycles of multiplicative red/black SAP on D x = y starting from x0
    (Alg. 3, SAP reading).  Works on one field or a stack of fields."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    masks = [blk.colour_mask_field(c) for c in (0, 1)]
    for _ in range(nu):
        for c in (0, 1):
            r = (y - apply_D(U, A, x)) * masks[c]
            e, _ = mr_blocks(U, A, blk, r, n_mr)
            x = x + e
    return x
