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


# --------------------------------------------------------------------------
# Counter-based draws for the seeded start of the setup.  The library draws
# its random starting test vectors on the device when the caller passes
# none; this is an independent host implementation of the same published
# generator, so that both sides can start from identical vectors:
#   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
#   easy as 1, 2, 3", SC 2011): 10 rounds of two 32x32 -> 64-bit products
#   with multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by the Weyl
#   constants 0x9E3779B9 and 0xBB67AE85 between rounds;
#   two 53-bit uniforms per call, u = (a >> 5) 2^-27 + (b >> 6) 2^-53 in
#   [0, 1) from the word pairs (x0, x1) and (x2, x3);
#   one Box-Muller pair per call: re = rho cos(2 pi u2), im = rho sin(2 pi u2),
#   rho = sqrt(-2 log(1 - u1)).
# Complex element i of the canonical array [n][t][z][y][x][spin][colour]
# uses the counter (i mod 2^32, i >> 32, 0, 0) and the key (seed mod 2^32,
# seed >> 32).
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays: ctr (4, N) and key (2, N) of uint32-valued
    integers; returns (4, N) uint64 arrays holding 32-bit words."""
    m32 = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & m32 for x in ctr]
    k = [np.asarray(x, dtype=np.uint64) & m32 for x in key]
    for rnd in range(10):
        if rnd:
            k = [(k[0] + np.uint64(_PHILOX_W[0])) & m32, (k[1] + np.uint64(_PHILOX_W[1])) & m32]
        p0 = np.uint64(_PHILOX_M[0]) * c[0]
        p1 = np.uint64(_PHILOX_M[1]) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c


def philox_gaussian_spinors(L, n, seed):
    """n complex Gaussian spinor fields drawn as the library draws them for a
    setup started without test vectors (see above)."""
    Lx, Ly, Lz, Lt = L
    N = n * Lt * Lz * Ly * Lx * 12
    out = np.empty(N, dtype=np.complex128)
    seed = int(seed) & ((1 << 64) - 1)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    step = 1 << 20
    for s in range(0, N, step):
        i = np.arange(s, min(N, s + step), dtype=np.uint64)
        z = np.zeros_like(i)
        x = philox4x32_10((i & np.uint64(0xFFFFFFFF), i >> np.uint64(32), z, z),
                          (np.full_like(i, key[0]), np.full_like(i, key[1])))
        u1 = (x[0] >> np.uint64(5)).astype(np.float64) * 2.0 ** -27 + (x[1] >> np.uint64(6)).astype(np.float64) * 2.0 ** -53
        u2 = (x[2] >> np.uint64(5)).astype(np.float64) * 2.0 ** -27 + (x[3] >> np.uint64(6)).astype(np.float64) * 2.0 ** -53
        rho = np.sqrt(-2.0 * np.log(1.0 - u1))
        out[s:s + len(i)] = rho * np.cos(2.0 * np.pi * u2) + 1j * rho * np.sin(2.0 * np.pi * u2)
    return out.reshape(n, Lt, Lz, Ly, Lx, 4, 3)


def network_weights(channels, seed):
    """Random starting weights of the test-vector network: one complex array
    (C_out, C_in, 18) per layer for the channel counts channels = (C_0, C_1,
    ..., C_L), entries complex Gaussian with variance 1 / (18 C_in)."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        g = rng.standard_normal((cout, cin, 18, 2)) / np.sqrt(2.0 * 18 * cin)
        out.append(g[..., 0] + 1j * g[..., 1])
    return out


# Batched serving of uneven instances: lattice shapes (Lx, Ly, Lz, Lt) and
# the block shape each one takes (12^4 splits into an even number of blocks
# only with 2^4 blocks).
UNEVEN_SHAPES = ((8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 12), (16, 16, 16, 16))


def uneven_instances(n, seed):
    """n independent instances for batched serving: shape uniform over
    UNEVEN_SHAPES, link disorder eps uniform in [0.3, 0.5], m0 uniform in
    [-0.2, -0.05], blocks 2^4 for 12^4 and 4^4 otherwise, N_tv = 16, c_sw = 1.
    Each instance also gets its own seeds for the gauge field, the setup's
    starting vectors and one Gaussian right-hand side.  Returns a list of
    dicts; nothing here draws the fields themselves."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = UNEVEN_SHAPES[int(rng.integers(len(UNEVEN_SHAPES)))]
        eps = float(rng.uniform(0.3, 0.5))
        m0 = float(rng.uniform(-0.2, -0.05))
        block = (2, 2, 2, 2) if L[0] == 12 else (4, 4, 4, 4)
        base = 1000 * seed + 3 * i
        out.append(dict(index=i, L=L, block=block, eps=eps, m0=m0, csw=1.0, ntv=16,
                        gauge_seed=base, setup_seed=base + 1, rhs_seed=base + 2))
    return out
