"""What the trained network gains over the method without it, on the GPU
through the C ABI: a network trained on plain setups of a few generated
8^4 fields (N_tv 8, 4^4 blocks), evaluated on a held-out field against the
same short setup started from random vectors (Alg. 4 without its initial
smoother passes) and against the untrained network.

* span loss against the held-out plain setup's aggregate basis, computed by
  the oracle from the exported proposals: trained < untrained < random;
* the outer solve (FP32 preconditioner, FP64 FGMRES to 1e-10) after a setup
  of no smoother and one V-cycle pass: the trained proposal needs no more
  outer iterations than the random start (or the random start diverges)."""
import sys

import numpy as np
import pytest

import synth
from oracle import sap, learned

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L = (8, 8, 8, 8)
BLOCK = (4, 4, 4, 4)
NTV = 8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_04506_amd as dd
    return dd


def _params(dd, **kw):
    return dd.default_params(L=L, block=BLOCK, m0=-0.2, csw=1.0, ntv=NTV, prec=dd.FP32, max_rhs=NTV, **kw)


def _proposal(dd, net, ctx, seed):
    out = torch.empty((NTV,) + tuple(reversed(L)) + (4, 3), dtype=torch.complex128, device="cuda")
    net.propose(ctx, out, seed=seed)
    torch.cuda.synchronize()
    return out


def test_trained_network_beats_random_start():
    dd = _gpu()
    from paper_1512_04506_amd import learned_setup as ls
    ch = ls.channels_for(NTV)
    net = dd.Net(ch)
    net.set_weights(torch.from_numpy(ls.smoother_init(ch, 0.1, 0.01, 7)).cuda())
    fields = [torch.from_numpy(synth.su3_field(L, 0.5, 900 + k)).cuda() for k in range(5)]
    samples, _ = ls.training_samples(net, fields[:4], _params(dd), seed0=910)
    held_U = fields[4]
    held = dd.Context(_params(dd, seed=920), held_U)
    held.mg_setup()
    T = torch.zeros((NTV,) + tuple(reversed(L)) + (4, 3), dtype=torch.complex128, device="cuda")
    held.export_basis(T)
    Tn = T.cpu().numpy()
    blk = sap.Blocking(L, BLOCK)
    untrained = _proposal(dd, net, held, 930).cpu().numpy()
    hist = ls.train(net, samples, 30, 3e-3)
    trained = _proposal(dd, net, held, 930).cpu().numpy()
    rand = synth.philox_gaussian_spinors(L, NTV, 931)
    l_tr, _ = learned.span_loss(blk, trained, Tn)
    l_un, _ = learned.span_loss(blk, untrained, Tn)
    l_rd, _ = learned.span_loss(blk, rand, Tn)
    say("held-out span loss: trained %.4f, untrained %.4f, random %.4f (training loss %.4f -> %.4f)" %
        (l_tr, l_un, l_rd, hist[0], hist[-1]))
    assert l_tr < l_un < l_rd
    # the short setup from each start, then the solve
    f = torch.from_numpy(synth.gaussian_spinors(L, 1, 932)).cuda()
    its = {}
    for name in ("trained", "random"):
        ctx = dd.Context(_params(dd, init_passes=0, n_setup=1, seed=931), held_U)
        if name == "trained":
            ctx.mg_setup(_proposal(dd, net, ctx, 930))
        else:
            ctx.mg_setup()  # the seeded random start: the same vectors as rand
        u = torch.zeros_like(f)
        try:
            rc, st = ctx.solve(u, f, 1, 1e-10)
            its[name] = st["outer_iterations"] if rc == 0 else None
        except dd.DDAMGError:
            its[name] = None
        ctx.close()
    say("outer iterations after no smoother and one V-cycle pass: trained %s, random %s" %
        (its["trained"], its["random"]))
    assert its["trained"] is not None
    assert its["random"] is None or its["trained"] <= its["random"]
    held.close()
    net.close()
