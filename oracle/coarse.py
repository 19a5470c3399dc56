"""Aggregates, restriction/prolongation, coarse operator and coarse solve
(oracle; test infrastructure only).

Aggregates (Sec. 2): each block holds two aggregates, the left-handed
(spins 0, 1) and the right-handed (spins 2, 3) components, 6 V_block degrees
of freedom each.  Coarse vectors have layout [block][h][a] with h = 0 (left),
1 (right) and a = 0..Ntv-1; the coarse component index is h * Ntv + a.

Coarse operator storage: D_c[i, slot] is a dense 2Ntv x 2Ntv block with slot
0 = self, 1 + 2 mu = forward neighbour i + mu, 2 + 2 mu = backward neighbour
i - mu (periodic block lattice), so that (D_c x)_i = sum_slot
D_c[i, slot] x_{nbr(i, slot)}.  Forward and backward couplings live in
separate slots even when they reach the same block (block-lattice extent 2).
"""
import numpy as np

from .dirac import apply_clover, hopping, block_hop_masks


def chirality_split(blk, f):
    """(..., Lt, Lz, Ly, Lx, 4, 3) -> (..., Nb, 2, Vblock*6): aggregate vectors.
    Row n enumerates (site in block, spin within the chirality, colour)."""
    g = blk.block_view(f)                         # (..., Nb, Vb, 4, 3)
    lead = g.shape[:-3]
    g = g.reshape(lead + (blk.vblock, 2, 2, 3))   # spin = 2 h + s
    k = len(lead)
    perm = list(range(k)) + [k + 1, k + 0, k + 2, k + 3]
    g = g.transpose(perm)                         # (..., Nb, 2, Vb, 2, 3)
    return g.reshape(lead + (2, blk.vblock * 6))


def chirality_merge(blk, g):
    """Inverse of chirality_split."""
    lead = g.shape[:-2]
    k = len(lead)
    h = g.reshape(lead + (2, blk.vblock, 2, 3))
    perm = list(range(k)) + [k + 1, k + 0, k + 2, k + 3]
    h = h.transpose(perm).reshape(lead + (blk.vblock, 4, 3))
    return blk.field_view(h)


def orthonormalise(blk, V):
    """Gram-Schmidt on every aggregate (Alg. 5): V is the stack of Ntv test
    vectors (Ntv, Lt, Lz, Ly, Lx, 4, 3).  For each aggregate the Ntv
    restricted vectors are the columns of X; the result W holds the columns
    of Q in the thin QR X = Q T with real positive diag(T) (the unique
    orthonormal basis produced by Gram-Schmidt), computed by modified
    Gram-Schmidt.  Returned as fields of the same shape as V."""
    X = chirality_split(blk, V)          # (Ntv, Nb, 2, n)
    X = np.moveaxis(X, 0, -1).copy()     # (Nb, 2, n, Ntv)
    ntv = X.shape[-1]
    Q = np.zeros_like(X)
    for a in range(ntv):
        v = X[..., a].copy()
        for b in range(a):
            c = np.sum(np.conj(Q[..., b]) * v, axis=-1)
            v = v - c[..., None] * Q[..., b]
        nrm = np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))
        if np.any(nrm == 0.0):
            raise FloatingPointError('rank-deficient aggregate')
        Q[..., a] = v / nrm[..., None]
    return chirality_merge(blk, np.moveaxis(Q, -1, 0))


def restrict(blk, W, y):
    """y_c = R y (Eq. R): y_c[b, h, a] = sum_{n in A_b^h} conj(W_a[n]) y[n].
    y may carry leading batch axes; result (..., Nb, 2, Ntv)."""
    Wa = chirality_split(blk, W)         # (Ntv, Nb, 2, n)
    ya = chirality_split(blk, y)         # (..., Nb, 2, n)
    return np.einsum('abhn,...bhn->...bha', np.conj(Wa), ya)


def prolong(blk, W, xc):
    """x = P x_c with P = R^dagger: x[n] = sum_a W_a[n] x_c[b, h, a]."""
    Wa = chirality_split(blk, W)
    xa = np.einsum('abhn,...bha->...bhn', Wa, xc)
    return chirality_merge(blk, xa)


def neighbour_table(blk):
    """nbr[i, slot] for the 9 slots (self, +x, -x, +y, -y, +z, -z, +t, -t)."""
    B = blk.block_coords()
    NB = blk.NB
    idx = lambda c: c[0] + NB[0] * (c[1] + NB[1] * (c[2] + NB[2] * c[3]))
    nbr = np.zeros((blk.nblocks, 9), dtype=np.int64)
    nbr[:, 0] = idx(B)
    for mu in range(4):
        for s, d in ((1, 1), (2, -1)):
            c = list(B)
            c[mu] = (c[mu] + d) % NB[mu]
            nbr[:, 2 * mu + s] = idx(c)
    return nbr


def coarse_operator(U, A, blk, W):
    """D_c = R D P (Eq. cgo), every slot computed directly.

    For each basis column (h', a) the prolongated field P e_{h',a} (test
    vector a on chirality h' of every block) is hit by one piece of D at a
    time: the block-internal part (clover plus hops inside blocks) for slot
    0, and for each mu the forward (backward) hops that cross a block face
    for slot 1 + 2 mu (2 + 2 mu).  Restricting each piece gives the couplings
    R_i D_ij P_j of that slot.  No symmetry (Eq. dagger) is used.
    """
    ntv = W.shape[0]
    n = 2 * ntv
    Dc = np.zeros((blk.nblocks, 9, n, n), dtype=np.complex128)
    in_f, in_b, cr_f, cr_b = block_hop_masks(blk.L, blk.block)
    zero = [np.zeros_like(m) for m in in_f]
    spin_h = np.zeros((2, 4))
    spin_h[0, :2] = 1.0
    spin_h[1, 2:] = 1.0
    for hp in range(2):
        Ph = W * spin_h[hp][:, None]            # (Ntv, ..., 4, 3)
        pieces = [apply_clover(A, Ph) - 0.5 * hopping(U, Ph, in_f, in_b)]
        for mu in range(4):
            fm = [cr_f[m] if m == mu else zero[m] for m in range(4)]
            bm = [cr_b[m] if m == mu else zero[m] for m in range(4)]
            pieces.append(-0.5 * hopping(U, Ph, fm, zero))
            pieces.append(-0.5 * hopping(U, Ph, zero, bm))
        for slot, T in enumerate(pieces):
            Tc = restrict(blk, W, T)            # (Ntv_col, Nb, 2, Ntv_row)
            Tc = Tc.reshape(ntv, blk.nblocks, n)
            Dc[:, slot, :, hp * ntv:(hp + 1) * ntv] = np.transpose(Tc, (1, 2, 0))
    return Dc


def coarse_apply(Dc, nbr, x):
    """(D_c x)_i = sum_slot D_c[i, slot] x_{nbr(i, slot)}; x (..., Nb, 2Ntv)."""
    xs = x[..., nbr, :]                         # (..., Nb, 9, n)
    return np.einsum('isrc,...isc->...ir', Dc, xs)


def coarse_parity(blk):
    return np.sum(np.stack(blk.block_coords()), axis=0) % 2


class CoarseSolver:
    """Even/odd preconditioned GMRES on the coarse grid (Alg. 2).

    Even coarse sites are eliminated: b_o = y_o - D_oe D_ee^{-1} y_e; GMRES
    with restart m_c, modified Gram-Schmidt and Givens rotations solves
    S x_o = b_o, S = D_oo - D_oe D_ee^{-1} D_eo, from x_o = 0 until the
    residual estimate is <= tol * ||y_c|| (with this x_e the full coarse
    residual is (0, b_o - S x_o), so the estimate measures the full system);
    then x_e = D_ee^{-1} (y_e - D_eo x_o).  With fixed_its set, exactly that
    many iterations run and the tolerance is not tested.
    """

    def __init__(self, blk, Dc, tol=0.05, restart=30, maxit=300, fixed_its=None):
        self.blk, self.Dc = blk, Dc
        self.nbr = neighbour_table(blk)
        p = coarse_parity(blk)
        self.even = np.nonzero(p == 0)[0]
        self.odd = np.nonzero(p == 1)[0]
        self.Dee_inv = np.linalg.inv(Dc[self.even, 0])
        self.tol, self.restart, self.maxit, self.fixed_its = tol, restart, maxit, fixed_its
        self.last_its = 0

    def _full(self, xe=None, xo=None):
        n = self.Dc.shape[-1]
        x = np.zeros((self.blk.nblocks, n), dtype=np.complex128)
        if xe is not None:
            x[self.even] = xe
        if xo is not None:
            x[self.odd] = xo
        return x

    def D_eo(self, xo):
        return coarse_apply(self.Dc, self.nbr, self._full(xo=xo))[self.even]

    def D_oe(self, xe):
        return coarse_apply(self.Dc, self.nbr, self._full(xe=xe))[self.odd]

    def D_oo(self, xo):
        return np.einsum('irc,ic->ir', self.Dc[self.odd, 0], xo)

    def Dee_solve(self, ve):
        return np.einsum('irc,ic->ir', self.Dee_inv, ve)

    def schur(self, xo):
        return self.D_oo(xo) - self.D_oe(self.Dee_solve(self.D_eo(xo)))

    def solve(self, yc):
        """yc: (Nb, 2, Ntv) -> x_c of the same shape."""
        shp = yc.shape
        y = yc.reshape(self.blk.nblocks, -1)
        ye, yo = y[self.even], y[self.odd]
        ynorm = np.linalg.norm(y)
        bo = yo - self.D_oe(self.Dee_solve(ye))
        xo = np.zeros_like(bo)
        self.last_its = 0
        if ynorm > 0.0:
            xo, self.last_its = gmres(self.schur, bo, xo, self.tol * ynorm, self.restart,
                                      self.maxit, self.fixed_its)
        xe = self.Dee_solve(ye - self.D_eo(xo))
        return self._full(xe, xo).reshape(shp)


def gmres(op, b, x, abstol, restart, maxit, fixed_its=None):
    """Restarted GMRES(restart) with modified Gram-Schmidt and Givens
    rotations on op x = b.  Stops when the residual estimate |g_{k+1}| <=
    abstol (not tested when fixed_its is given, which runs exactly that many
    iterations), after maxit iterations, or on exact breakdown.
    Returns (x, iterations)."""
    total = fixed_its if fixed_its is not None else maxit
    its = 0
    while its < total:
        r = b - op(x)
        beta = np.linalg.norm(r)
        if beta == 0.0 or (fixed_its is None and beta <= abstol):
            break
        m = min(restart, total - its)
        Vb = [r / beta]
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k_done = 0
        stop = False
        for k in range(m):
            w = op(Vb[k])
            for j in range(k + 1):
                H[j, k] = np.vdot(Vb[j], w)
                w = w - H[j, k] * Vb[j]
            H[k + 1, k] = np.linalg.norm(w)
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -np.conj(sn[j]) * H[j, k] + np.conj(cs[j]) * H[j + 1, k]
                H[j, k] = t
            cs[k], sn[k], H[k, k] = _givens(H[k, k], H[k + 1, k])
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_done = k + 1
            breakdown = False
            hn = np.linalg.norm(w)
            if hn == 0.0:
                breakdown = True
            else:
                Vb.append(w / hn)
            if breakdown or (fixed_its is None and abs(g[k + 1]) <= abstol):
                stop = True
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        for j in range(k_done):
            x = x + y[j] * Vb[j]
        if stop:
            break
    return x, its


def _givens(a, b):
    """Rotation [c s; -conj(s) conj(c)] with real c >= 0 mapping (a, b) to
    (r, 0) where |r| = sqrt(|a|^2 + |b|^2)."""
    if b == 0.0:
        return 1.0, 0.0, a
    if a == 0.0:
        return 0.0, 1.0 * np.conj(b) / abs(b), abs(b)
    na = abs(a)
    nrm = np.sqrt(na ** 2 + abs(b) ** 2)
    c = na / nrm
    s = (a / na) * np.conj(b) / nrm
    r = (a / na) * nrm
    return c, s, r
