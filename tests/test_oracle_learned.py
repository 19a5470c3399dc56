"""Pins of the oracle's test-vector network, span loss and gradients (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import dirac, sap, coarse, learned
from helpers import relerr

L = (4, 4, 2, 2)
BLK = (2, 2, 1, 1)


def _field(seed, eps=0.5):
    return synth.su3_field(L, eps, seed)


def test_wilson_weights_give_the_dirac_operator_without_clover():
    """One channel with a = 4 + m0, c = -1/2 and d = +1/2 (forward hops),
    -1/2 (backward hops) is D at c_sw = 0; b alone is g5."""
    U = _field(71)
    m0 = -0.2
    w = np.zeros((1, 1, 18), dtype=complex)
    w[0, 0, 0] = 4 + m0
    for mu in range(4):
        for s in range(2):
            h = 2 * mu + s
            w[0, 0, 2 + 2 * h] = -0.5
            w[0, 0, 3 + 2 * h] = 0.5 if s == 0 else -0.5
    phi = synth.gaussian_spinors(L, 1, 72)
    ref = dirac.apply_D(U, dirac.clover_term(U, m0, 0.0), phi[0])
    assert relerr(learned.layer(U, w, phi)[0], ref) < 1e-14
    w5 = np.zeros((1, 1, 18), dtype=complex)
    w5[0, 0, 1] = 1.0
    assert relerr(learned.layer(U, w5, phi)[0], dirac.apply_g5(phi[0])) < 1e-15


def test_layer_is_linear_in_channels():
    U = _field(73)
    w = synth.network_weights((3, 2), 74)[0]
    phi = synth.gaussian_spinors(L, 3, 75)
    out = learned.layer(U, w, phi)
    for i in range(2):
        acc = sum(learned.layer(U, w[i:i + 1, j:j + 1], phi[j:j + 1])[0] for j in range(3))
        assert relerr(out[i], acc) < 1e-14


def test_gauge_covariance():
    """U_mu(x) -> g(x) U_mu(x) g(x + mu)^dag and noise -> g noise transform
    the proposal as X -> g X; the span loss against g T is unchanged."""
    U = _field(76)
    g = synth.random_su3_gauge_transform(L, 77)
    Ug = np.empty_like(U)
    for mu in range(4):
        gf = np.roll(g, -1, axis=3 - mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gf, -1, -2))
    ws = synth.network_weights((2, 3, 3, 4), 78)
    noise = synth.gaussian_spinors(L, 2, 79)
    gx = lambda f: np.einsum('...ab,...sb->...sa', g, f)
    X, _ = learned.forward(U, ws, noise)
    Xg, _ = learned.forward(Ug, ws, gx(noise))
    assert relerr(Xg, gx(X)) < 1e-13
    blk = sap.Blocking(L, BLK)
    T = coarse.orthonormalise(blk, synth.gaussian_spinors(L, 4, 80))
    l1, _ = learned.loss_and_grad(U, ws, noise, blk, T)
    l2, _ = learned.loss_and_grad(Ug, ws, gx(noise), blk, gx(T))
    assert abs(l1 - l2) < 1e-13


def test_span_loss_closed_forms_and_invariances():
    blk = sap.Blocking(L, BLK)
    ntv = 4
    T = coarse.orthonormalise(blk, synth.gaussian_spinors(L, ntv, 81))
    M = (np.random.default_rng(82).standard_normal((ntv, ntv)) +
         1j * np.random.default_rng(83).standard_normal((ntv, ntv)))
    mix = lambda F: np.einsum('ia,a...->i...', M, F)
    # the same span on every aggregate: loss 0
    assert abs(learned.span_loss(blk, mix(T), T)[0]) < 1e-13
    # orthogonal to the target on every aggregate: loss 1
    R = synth.gaussian_spinors(L, ntv, 84)
    Ra = coarse.chirality_split(blk, R)
    Ta = coarse.chirality_split(blk, T)
    c = np.einsum('abhn,cbhn->cabh', np.conj(Ta), Ra)   # (ntv_R, ntv_T, Nb, 2)
    Rp = Ra - np.einsum('cabh,abhn->cbhn', c, Ta)
    Xo = coarse.chirality_merge(blk, Rp)
    assert abs(learned.span_loss(blk, Xo, T)[0] - 1.0) < 1e-13
    # independent of the basis chosen for either span
    X = synth.gaussian_spinors(L, ntv, 85)
    l0 = learned.span_loss(blk, X, T)[0]
    assert abs(learned.span_loss(blk, mix(X), T)[0] - l0) < 1e-13
    T2 = coarse.orthonormalise(blk, mix(T))
    assert abs(learned.span_loss(blk, X, T2)[0] - l0) < 1e-13
    # one test vector: the mean over aggregates of sin^2 of the angle
    x1, t1 = X[:1], T[:1]
    xa, ta = coarse.chirality_split(blk, x1)[0], coarse.chirality_split(blk, t1)[0]
    cos2 = np.abs(np.sum(np.conj(xa) * ta, axis=-1)) ** 2 / np.sum(np.abs(xa) ** 2, axis=-1)
    assert abs(learned.span_loss(blk, x1, t1)[0] - np.mean(1 - cos2)) < 1e-14


def _fd(fn, w, dw, h=1e-6):
    return (fn(w + h * dw) - fn(w - h * dw)) / (2 * h)


def test_span_loss_gradient_by_finite_differences():
    blk = sap.Blocking(L, BLK)
    T = coarse.orthonormalise(blk, synth.gaussian_spinors(L, 3, 86))
    X = synth.gaussian_spinors(L, 3, 87)
    loss, gam = learned.span_loss(blk, X, T)
    grad = 2 * gam
    rng = np.random.default_rng(88)
    for _ in range(3):
        D = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
        fd = _fd(lambda Y: learned.span_loss(blk, Y, T)[0], X, D)
        assert abs(fd - np.real(np.sum(np.conj(grad) * D))) < 1e-8 * max(1.0, abs(fd))


def test_weight_gradients_by_finite_differences():
    """Every layer's gradient (three layers, two gates) against central
    differences along random directions and in single real and imaginary
    parts of sampled weights."""
    U = _field(89)
    blk = sap.Blocking(L, BLK)
    ws = synth.network_weights((2, 3, 3, 4), 90)
    noise = synth.gaussian_spinors(L, 2, 91)
    T = coarse.orthonormalise(blk, synth.gaussian_spinors(L, 4, 92))
    loss, grads = learned.loss_and_grad(U, ws, noise, blk, T)
    assert 0.0 < loss < 1.0
    rng = np.random.default_rng(93)

    def L_at(l, wl):
        w2 = list(ws)
        w2[l] = wl
        return learned.forward(U, w2, noise)[0]

    for l in range(3):
        f = lambda wl: learned.span_loss(blk, L_at(l, wl), T)[0]
        D = rng.standard_normal(ws[l].shape) + 1j * rng.standard_normal(ws[l].shape)
        fd = _fd(f, ws[l], D)
        an = np.real(np.sum(np.conj(grads[l]) * D))
        assert abs(fd - an) < 1e-7 * max(1e-2, abs(fd)), (l, fd, an)
        for idx in [(0, 0, 0), (1, 1, 5), (2, 0, 17)]:
            E = np.zeros_like(ws[l])
            E[idx] = 1.0
            assert abs(_fd(f, ws[l], E) - grads[l][idx].real) < 1e-7
            assert abs(_fd(f, ws[l], 1j * E) - grads[l][idx].imag) < 1e-7


def test_adam_first_steps():
    """First Adam step moves every real and imaginary part by lr against the
    sign of its gradient (bias-corrected moments m = g, v = g^2); a gradient
    that stays the same keeps that step."""
    g = [np.array([[[0.3 - 2j, -1e-3 + 5j]]])]
    w = [np.zeros_like(g[0])]
    m = [np.zeros_like(g[0])]
    v = [np.zeros_like(g[0])]
    eps = 1e-8
    w1, m1, v1 = learned.adam_step(w, g, m, v, 1, 0.01, eps=eps)
    gr, gi = g[0].real, g[0].imag
    first = -0.01 * (gr / (np.abs(gr) + eps) + 1j * gi / (np.abs(gi) + eps))
    assert np.abs(w1[0] - first).max() < 1e-15
    assert np.abs(first.real - (-0.01 * np.sign(gr))).max() < 1e-6
    w2, _, _ = learned.adam_step(w1, g, m1, v1, 2, 0.01, eps=eps)
    assert np.abs(w2[0] - 2 * first).max() < 1e-15
