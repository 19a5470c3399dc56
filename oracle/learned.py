"""Learned proposal of test vectors for the adaptive setup (oracle; test
infrastructure only: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it).

The paper's setup (Alg. 4) starts from random vectors and smooths them
before the first aggregate Gram-Schmidt (Alg. 5).  This module defines a
small gauge-covariant network that maps random fields to proposed test
vectors instead, the span loss that compares a proposal with the aggregate
basis of a plain setup, and the gradients of that loss, in plain FP64
numpy.  None of it is in the paper; the choices are listed here.

Network.  A layer maps C_in channel fields phi_j (spinor fields, shape
(..., Lt, Lz, Ly, Lx, 4, 3)) to C_out channel fields

  psi_i(x) = sum_j [ (a_ij + b_ij g5) phi_j(x)
                     + sum_mu sum_s (c_ij,mu,s + d_ij,mu,s g_mu) (T_mu,s phi_j)(x) ]

with the parallel transports (T_mu,+ phi)(x) = U_mu(x) phi(x + mu) and
(T_mu,- phi)(x) = U_mu(x - mu)^dag phi(x - mu), under the fermion boundary
conditions of D (time antiperiodic).  The weights of a layer form a complex
array w[i, j, k] of shape (C_out, C_in, 18): k = 0 is a, k = 1 is b, and hop
h = 2 mu + s (s = 0 forward, 1 backward) has k = 2 + 2h (c) and k = 3 + 2h
(d).  With a = 4 + m0, b = 0 and c = -1/2, d = +1/2 (forward) or -1/2
(backward) a single-channel layer is the Wilson operator without clover.
Between layers every channel passes the gauge-invariant gate
sigma(psi)(x) = psi(x) / sqrt(1 + |psi(x)|^2 / 12), |.| over spin and
colour at the site.  The last layer has no gate; its C_out = N_tv channels
are the proposed test vectors.  A gauge transformation g(x) of the links
(U_mu(x) -> g(x) U_mu(x) g(x + mu)^dag) and of the inputs (phi -> g phi)
transforms every layer's output as psi -> g psi.

Span loss.  For aggregate A (Sec. 2: a block and a chirality) let X_A
(n_A x N_tv) hold the proposal restricted to A and T_A (n_A x N_tv) an
orthonormal basis of the target span (the aggregate basis of a plain setup,
the rows of its R).  With P_A = X_A (X_A^H X_A)^-1 X_A^H,

  loss = (1 / (N_A N_tv)) sum_A || (1 - P_A) T_A ||_F^2
       = 1 - (1 / (N_A N_tv)) sum_A tr(C_A^H G_A^-1 C_A),
  G_A = X_A^H X_A,  C_A = X_A^H T_A,

which is 0 when every aggregate's proposal spans its target and 1 when it
is orthogonal to it, and does not change if the proposal or the target is
replaced by another basis of the same span on an aggregate (the aggregate
basis of Alg. 5 is defined only up to such a change).

Gradients.  For the real loss and a complex variable w the gradient is
reported as dL/dRe w + i dL/dIm w.  In terms of Gamma = dL/d conj(w) (the
Wirtinger derivative, dL = 2 Re sum conj(Gamma) dw) it is 2 Gamma.  With
Z_A = G_A^-1 C_A the loss gives Gamma_X = -(T_A - X_A Z_A) Z_A^H / (N_A N_tv)
on every aggregate; a layer psi_i = sum_jk w_ijk F_jk(phi) (F_jk the 18
feature maps) passes back Gamma_w[i, j, k] = sum_x <F_jk(phi)(x), Gamma_i(x)>
and Gamma_phi_j = sum_ik conj(w_ijk) F_jk^dag Gamma_i, where T_mu,s^dag =
T_mu,-s and g5, g_mu are Hermitian and commute with the transports; the gate
passes back Gamma_psi = g Gamma_sigma + (rho g'(n) / 6) psi with n =
|psi|^2 / 12, g(n) = (1 + n)^(-1/2), rho = Re <psi, Gamma_sigma> at the site.

Training.  Adam (Kingma and Ba, 2015) on the real and imaginary parts of
every weight, as the GPU trainer runs it.
"""
import numpy as np

from .dirac import GAMMA, G5, shift_fwd, shift_bwd, link_bwd, _colour, _spin, _dag
from .coarse import chirality_split

NFEAT = 18


def transport(U, phi, mu, s):
    """T_mu,s phi: forward (s = 0) U_mu(x) phi(x + mu), backward (s = 1)
    U_mu(x - mu)^dag phi(x - mu), t antiperiodic."""
    Umu = U[..., mu, :, :]
    if s == 0:
        return _colour(Umu, shift_fwd(phi, mu))
    return _colour(_dag(link_bwd(Umu, mu)), shift_bwd(phi, mu))


def features(U, phi):
    """The 18 feature fields of phi (..., site, 4, 3): phi, g5 phi, and per
    hop h = 2 mu + s the transport T_h phi and g_mu T_h phi.  Returns a list."""
    out = [phi, _spin(G5, phi)]
    for mu in range(4):
        for s in range(2):
            t = transport(U, phi, mu, s)
            out.append(t)
            out.append(_spin(GAMMA[mu], t))
    return out


def features_adjoint(U, gam):
    """The adjoints F_k^dag applied to gam, one field per feature k."""
    out = [gam, _spin(G5, gam)]
    for mu in range(4):
        for s in range(2):
            t = transport(U, gam, mu, 1 - s)   # T_mu,s^dag = T_mu,-s
            out.append(t)
            out.append(_spin(GAMMA[mu], t))    # g_mu commutes with the transport
    return out


def layer(U, w, phi):
    """psi_i = sum_jk w[i, j, k] F_k(phi_j); phi (C_in, site..., 4, 3)."""
    cout, cin, nf = w.shape
    assert nf == NFEAT and phi.shape[0] == cin
    psi = np.zeros((cout,) + phi.shape[1:], dtype=np.complex128)
    for j in range(cin):
        F = features(U, phi[j])
        for k in range(NFEAT):
            psi += w[:, j, k].reshape((cout,) + (1,) * (phi.ndim - 1)) * F[k][None]
    return psi


def gate(psi):
    """sigma(psi) = psi / sqrt(1 + |psi(x)|^2 / 12) per channel and site."""
    n = np.sum(np.abs(psi) ** 2, axis=(-1, -2), keepdims=True) / 12.0
    return psi / np.sqrt(1.0 + n)


def forward(U, weights, noise):
    """Network output (the proposed test vectors, (N_tv, site..., 4, 3)) for
    the input fields noise (C_0, site..., 4, 3); weights: list of layer
    weight arrays.  Also returns the pre-gate activations of every layer."""
    act = []
    x = noise
    for l, w in enumerate(weights):
        psi = layer(U, w, x)
        act.append((x, psi))
        x = gate(psi) if l + 1 < len(weights) else psi
    return x, act


def span_loss(blk, X, T):
    """Span loss and its Wirtinger gradient Gamma_X = dL/d conj(X) for the
    proposal X and the orthonormal target basis T (both (N_tv, site..., 4, 3)),
    summed over the aggregates of the blocking blk."""
    Xa = np.moveaxis(chirality_split(blk, X), 0, -1)   # (Nb, 2, n, Ntv)
    Ta = np.moveaxis(chirality_split(blk, T), 0, -1)
    nagg = Xa.shape[0] * Xa.shape[1]
    ntv = Ta.shape[-1]
    XH = np.conj(np.swapaxes(Xa, -1, -2))
    G = XH @ Xa
    C = XH @ Ta
    Z = np.linalg.solve(G, C)
    explained = np.real(np.trace(np.conj(np.swapaxes(C, -1, -2)) @ Z, axis1=-2, axis2=-1))
    scale = 1.0 / (nagg * ntv)
    loss = 1.0 - scale * np.sum(explained)
    gam = -scale * (Ta - Xa @ Z) @ np.conj(np.swapaxes(Z, -1, -2))
    from .coarse import chirality_merge
    return loss, chirality_merge(blk, np.moveaxis(gam, -1, 0))


def loss_and_grad(U, weights, noise, blk, T):
    """Span loss of the network's proposal against the target basis T and the
    gradient dL/dRe w + i dL/dIm w of every layer's weights (a list)."""
    X, act = forward(U, weights, noise)
    loss, gam = span_loss(blk, X, T)
    grads = [None] * len(weights)
    for l in range(len(weights) - 1, -1, -1):
        phi, psi = act[l]
        w = weights[l]
        if l + 1 < len(weights):
            # gam is dL/d conj(sigma(psi)): back through the gate
            n = np.sum(np.abs(psi) ** 2, axis=(-1, -2), keepdims=True) / 12.0
            g = 1.0 / np.sqrt(1.0 + n)
            dg = -0.5 * g ** 3
            rho = np.real(np.sum(np.conj(psi) * gam, axis=(-1, -2), keepdims=True))
            gam = g * gam + (rho * dg / 6.0) * psi
        cout, cin, _ = w.shape
        gw = np.zeros_like(w)
        gphi = np.zeros_like(phi)
        for j in range(cin):
            F = features(U, phi[j])
            for k in range(NFEAT):
                gw[:, j, k] = np.sum(np.conj(F[k])[None] * gam, axis=tuple(range(1, gam.ndim)))
        for i in range(cout):
            Fa = features_adjoint(U, gam[i])
            for j in range(cin):
                for k in range(NFEAT):
                    gphi[j] += np.conj(w[i, j, k]) * Fa[k]
        grads[l] = 2.0 * gw
        gam = gphi
    return loss, grads


def adam_step(weights, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) on the real and imaginary parts
    of every weight; m, v: first and second moments (complex arrays holding
    the real and imaginary parts' moments), t: step number from 1.  Returns
    the new (weights, m, v)."""
    out_w, out_m, out_v = [], [], []
    for w, g, mm, vv in zip(weights, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * (g.real ** 2 + 1j * g.imag ** 2)
        mh = mm / (1 - beta1 ** t)
        vh = vv / (1 - beta2 ** t)
        step = mh.real / (np.sqrt(vh.real) + eps) + 1j * mh.imag / (np.sqrt(vh.imag) + eps)
        out_w.append(w - lr * step)
        out_m.append(mm)
        out_v.append(vv)
    return out_w, out_m, out_v
