"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module holds no arithmetic of the solver: it only draws gauge fields,
right-hand sides and random starting test vectors.  Both the CPU oracle and
the GPU library receive the arrays it returns as plain inputs.

Canonical layouts (numpy, complex128, C order):
  gauge field  U[t, z, y, x, mu, a, b]      mu = 0..3 <-> x, y, z, t
  spinor field psi[..., t, z, y, x, spin, colour]

Gauge links follow U = exp(i eps H) with H a Gaussian Hermitian traceless
3x3 matrix (off-diagonal E|H_ij|^2 = 1), drawn site by site in the order
t, z, y, x, mu from numpy's PCG64 generator, then re-unitarised (Gram-Schmidt
on rows 1-2, row 3 = conj(row1 x row2)) so that det U = 1 to rounding.
"""
import numpy as np


def su3_field(L, eps, seed, chunk=1 << 20):
    """Random SU(3) links of disorder `eps` on lattice L = (Lx, Ly, Lz, Lt)."""
    Lx, Ly, Lz, Lt = L
    n = Lt * Lz * Ly * Lx * 4
    rng = np.random.default_rng(seed)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        g = rng.standard_normal((m, 3, 3, 2))
        M = g[..., 0] + 1j * g[..., 1]
        H = 0.5 * (M + np.conj(np.swapaxes(M, -1, -2)))
        tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
        H[:, 0, 0] -= tr
        H[:, 1, 1] -= tr
        H[:, 2, 2] -= tr
        w, Wv = np.linalg.eigh(H)
        U = (Wv * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(Wv, -1, -2))
        out[s:s + m] = _reunitarise(U)
    return out.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


def _reunitarise(U):
    r0 = U[:, 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[:, 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=1)


def unit_field(L):
    """Free field U = 1 on every link."""
    Lx, Ly, Lz, Lt = L
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    for a in range(3):
        U[..., a, a] = 1.0
    return U


def gaussian_spinors(L, n, seed):
    """n complex Gaussian spinor fields (re, im ~ N(0, 1))."""
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, Lt, Lz, Ly, Lx, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def point_sources(L, site=(0, 0, 0, 0)):
    """The 12 unit vectors e_{site, spin, colour}, ordered comp = 3*spin + colour."""
    Lx, Ly, Lz, Lt = L
    x, y, z, t = site
    f = np.zeros((12, Lt, Lz, Ly, Lx, 4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            f[3 * s + c, t, z, y, x, s, c] = 1.0
    return f


def gaussian_coarse(nblocks, ntv, n, seed):
    """n complex Gaussian coarse vectors, layout [n][block][2][ntv]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, nblocks, 2, ntv, 2))
    return g[..., 0] + 1j * g[..., 1]


def random_su3_gauge_transform(L, seed):
    """One random SU(3) matrix per site, g[t, z, y, x, a, b]."""
    Lx, Ly, Lz, Lt = L
    U = su3_field((Lx, Ly, Lz, Lt), 1.0, seed)
    return U[..., 0, :, :].copy()
