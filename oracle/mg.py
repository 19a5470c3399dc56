"""Two-level V-cycle, adaptive setup and outer FGMRES (oracle; test only).

  vcycle  -- Alg. 1: coarse-grid correction (Alg. 2) of y, then the SAP
             smoother (Alg. 3) on y started from the prolongated coarse
             solution.
  setup   -- Alg. 4 with Alg. 5: random test vectors (passed in), three
             smoother passes with N_smoother = 1, 2, 3 from a zero guess,
             aggregate Gram-Schmidt and D_c, one normalisation of the test
             vectors, then N_setup passes that replace every test vector by
             the V-cycle applied to it (R and D_c frozen during a pass) and
             rebuild R and D_c (the algorithm normalises only once, after
             the initial setup).
  fgmres  -- right-preconditioned flexible GMRES(m) for D u = f (Sec. 1:
             solve D M^{-1} v = f, u = M^{-1} v), modified Gram-Schmidt,
             Givens rotations, stopped on |g_{j+1}| <= tol ||f||, with the
             true residual f - D u recomputed in FP64 at every restart and
             at the end.

Parity status: vcycle, fgmres and the pieces of setup are pinned by the
tests; the composition of setup (the number and order of its passes) is
pinned on a gauge field with the links across block faces cut, where every
smoother pass and V-cycle is an exact D^{-1} and Alg. 4 has the closed form
V ~ D^{-(3 + N_setup)} V_0 (dense solves).
"""
import numpy as np

from .dirac import clover_term, apply_D
from .sap import Blocking, sap
from .coarse import orthonormalise, coarse_operator, CoarseSolver, restrict, prolong, _givens


class Params:
    """Solver parameters; defaults follow the readings listed in the design
    notes (nu = 3 SAP cycles, 4 MR steps, coarse tolerance 0.05, coarse
    GMRES(30) with at most 300 iterations, FGMRES(20), tol 1e-10)."""

    def __init__(self, L, block, m0, csw, ntv, n_setup=3, nu=3, n_mr=4,
                 coarse_tol=0.05, coarse_restart=30, coarse_maxit=300,
                 coarse_fixed_its=None, outer_restart=20, outer_maxit=2000):
        self.L, self.block = tuple(L), tuple(block)
        self.m0, self.csw, self.ntv = m0, csw, ntv
        self.n_setup, self.nu, self.n_mr = n_setup, nu, n_mr
        self.coarse_tol, self.coarse_restart = coarse_tol, coarse_restart
        self.coarse_maxit, self.coarse_fixed_its = coarse_maxit, coarse_fixed_its
        self.outer_restart, self.outer_maxit = outer_restart, outer_maxit


class MG:
    """Two-level DD-alpha-AMG state: links, clover, test vectors, R, D_c."""

    def __init__(self, params, U):
        self.p = params
        self.U = U
        self.A = clover_term(U, params.m0, params.csw)
        self.blk = Blocking(params.L, params.block)
        self.W = None
        self.Dc = None
        self.coarse = None
        self.V = None
        self.coarse_its = []

    # -- operators -------------------------------------------------------
    def D(self, psi):
        return apply_D(self.U, self.A, psi)

    def smoother(self, y, x0, nu=None):
        return sap(self.U, self.A, self.blk, y, x0, self.p.nu if nu is None else nu, self.p.n_mr)

    def build_coarse(self, V):
        """Alg. 5: Gram-Schmidt on the aggregates, then D_c = R D P."""
        self.W = orthonormalise(self.blk, V)
        self.Dc = coarse_operator(self.U, self.A, self.blk, self.W)
        p = self.p
        self.coarse = CoarseSolver(self.blk, self.Dc, p.coarse_tol, p.coarse_restart,
                                   p.coarse_maxit, p.coarse_fixed_its)

    def set_basis(self, W):
        """Use a given orthonormal aggregate basis W (no Gram-Schmidt)."""
        self.W = W
        self.Dc = coarse_operator(self.U, self.A, self.blk, W)
        p = self.p
        self.coarse = CoarseSolver(self.blk, self.Dc, p.coarse_tol, p.coarse_restart,
                                   p.coarse_maxit, p.coarse_fixed_its)

    def cgc(self, y):
        """Alg. 2: x = P D_c^{-1} R y with the approximate coarse solve."""
        yc = restrict(self.blk, self.W, y)
        xc = self.coarse.solve(yc)
        self.coarse_its.append(self.coarse.last_its)
        return prolong(self.blk, self.W, xc)

    def vcycle(self, y):
        """Alg. 1 on one field y."""
        x0 = self.cgc(y)
        return self.smoother(y, x0)

    # -- setup -----------------------------------------------------------
    def setup(self, tv_init):
        """Alg. 4.  tv_init: (Ntv, Lt, Lz, Ly, Lx, 4, 3) random start vectors."""
        V = np.array(tv_init, dtype=np.complex128, copy=True)
        for k in (1, 2, 3):
            V = np.stack([self.smoother(V[j], np.zeros_like(V[j]), nu=k) for j in range(len(V))])
        self.build_coarse(V)
        V = _normalise(V)
        for _ in range(self.p.n_setup):
            V = np.stack([self.vcycle(V[j]) for j in range(len(V))])
            self.build_coarse(V)
        self.V = V
        return V

    # -- outer solve -----------------------------------------------------
    def solve(self, f, u0=None, tol=1e-10, fixed_its=None):
        """FGMRES(m) right-preconditioned by the V-cycle on one field f.
        Returns (u, stats dict)."""
        return fgmres(self.D, self.vcycle, f, u0, tol, self.p.outer_restart,
                      self.p.outer_maxit, fixed_its)


def _normalise(V):
    n = np.sqrt(np.sum(np.abs(V) ** 2, axis=tuple(range(1, V.ndim))))
    return V / n.reshape((-1,) + (1,) * (V.ndim - 1))


def fgmres(D, M, f, u0=None, tol=1e-10, restart=20, maxit=2000, fixed_its=None):
    """Flexible GMRES(restart) with right preconditioner M (a function).
    Stops when the FP64 true residual ||f - D u|| <= tol ||f||, checked when
    the Givens estimate reaches it and at every restart; with fixed_its,
    runs exactly that many iterations."""
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.complex128, copy=True)
    fnorm = np.sqrt(np.sum(np.abs(f) ** 2))
    stats = {'iterations': 0, 'restarts': 0, 'history': []}
    if fnorm == 0.0:
        stats['relres'] = 0.0
        return np.zeros_like(f), stats
    target = tol * fnorm
    total = fixed_its if fixed_its is not None else maxit
    its = 0
    while True:
        r = f - D(u)
        beta = np.sqrt(np.sum(np.abs(r) ** 2))
        stats['history'].append(beta / fnorm)
        if its >= total or (fixed_its is None and beta <= target) or beta == 0.0:
            break
        m = min(restart, total - its)
        Vb = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k_done = 0
        for k in range(m):
            z = M(Vb[k])
            Z.append(z)
            w = D(z)
            for j in range(k + 1):
                H[j, k] = np.vdot(Vb[j], w)
                w = w - H[j, k] * Vb[j]
            hn = np.sqrt(np.sum(np.abs(w) ** 2))
            H[k + 1, k] = hn
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
            if hn == 0.0:
                break
            Vb.append(w / hn)
            if fixed_its is None and abs(g[k + 1]) <= target:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        for j in range(k_done):
            u = u + y[j] * Z[j]
        stats['restarts'] += 1
    stats['iterations'] = its
    stats['relres'] = beta / fnorm
    return u, stats


def true_relres(D, u, f):
    """||f - D u|| / ||f|| in FP64 with the oracle's own D."""
    fn = np.sqrt(np.sum(np.abs(f) ** 2))
    r = f - D(u)
    return np.sqrt(np.sum(np.abs(r) ** 2)) / fn if fn > 0 else 0.0
