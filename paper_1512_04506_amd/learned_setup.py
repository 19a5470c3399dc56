"""Training and use of the learned test-vector proposal (ddamg_net).

Host-side orchestration only: every step -- the plain setups that produce
the targets, the network's forward and backward passes, the span loss and
Adam -- runs in the library's kernels through the C ABI.

  training_samples  plain setups (Alg. 4, Alg. 5) on generated gauge fields;
                    their aggregate bases become the network's targets
  train             Adam over the samples with fresh random inputs per step
  propose_setup     mg_setup started from the network's proposal, skipping
                    the initial smoother passes of Alg. 4
"""
import time

import numpy as np

import paper_1512_04506_amd as dd

CHANNELS = (12, 16, 16, 16)  # input fields and hidden layers; the output layer has ntv channels


def channels_for(ntv):
    return CHANNELS + (int(ntv),)


def smoother_init(channels, kappa, noise, seed):
    """Starting weights (complex64, the layer layout of the C ABI): every
    layer starts as phi_i + kappa H phi_i on the channels it shares with
    its input, H = sum_mu [(1 - g_mu) T_mu,+ + (1 + g_mu) T_mu,-] the Wilson
    hopping term, so the untrained network already damps the high modes of D
    (a polynomial in H that grows towards H's largest real eigenvalues,
    where D's low modes are); plus complex Gaussian noise of the given scale
    on every weight to break the symmetry between channels."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        g = rng.standard_normal((cout, cin, 18, 2)) * (noise / np.sqrt(2.0))
        w = g[..., 0] + 1j * g[..., 1]
        for i in range(min(cin, cout)):
            w[i, i, 0] += 1.0
            for mu in range(4):
                w[i, i, 2 + 4 * mu] += kappa          # forward: (1 - g_mu) T_mu,+
                w[i, i, 3 + 4 * mu] -= kappa
                w[i, i, 4 + 4 * mu] += kappa          # backward: (1 + g_mu) T_mu,-
                w[i, i, 5 + 4 * mu] += kappa
        out.append(w.reshape(-1))
    return np.concatenate(out).astype(np.complex64)


def training_samples(net, fields, params, seed0=0, log=None):
    """For every gauge field (device complex128 tensors, canonical layout):
    a plain setup with the given parameters started from the seeded random
    vectors of mg_setup, its aggregate basis added to the network as a
    training target.  Returns the sample indices and the setup times."""
    import torch
    idx, times = [], []
    for k, U in enumerate(fields):
        params.seed = seed0 + k
        ctx = dd.Context(params, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mg_setup()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        idx.append(net.add_sample(ctx))
        ctx.close()
        if log:
            log("  sample %d: plain setup %.1f ms" % (k, times[-1] * 1e3))
    return idx, times


def train(net, samples, epochs, lr, seed0=1 << 20, decay=0.5, decay_every=None, log=None):
    """Adam over the samples, one step per sample and epoch, each with fresh
    random input fields; the learning rate is multiplied by decay every
    decay_every epochs.  Returns the mean loss of every epoch."""
    hist = []
    step = 0
    for e in range(epochs):
        cur = lr * (decay ** (e // decay_every) if decay_every else 1.0)
        losses = []
        for s in samples:
            losses.append(net.train_step(s, seed0 + step, cur))
            step += 1
        hist.append(float(np.mean(losses)))
        if log:
            log("  epoch %d: lr %.2e mean span loss %.4f" % (e, cur, hist[-1]))
    return hist


def propose_setup(net, ctx, seed):
    """mg_setup from the network's proposal on ctx's lattice (the context
    must have been created with init_passes = 0 to use it as it is).
    Returns (proposal ms, setup ms)."""
    import torch
    shape = (ctx.ntv,) + tuple(reversed(ctx.L)) + (4, 3)
    tv = torch.empty(shape, dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.propose(ctx, tv, seed=seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.mg_setup(tv)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del tv
    return (t1 - t0) * 1e3, (t2 - t1) * 1e3
