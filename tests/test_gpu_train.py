"""Training loop (paper_2004_11658_amd.train): Adam on the energy + force loss through
the library's batched forces, parameter gradient and Adam kernel, against the same
loop on the oracle side (PyTorch-CPU FP64 double back propagation for the gradient,
the oracle's Adam step, pinned by hand-worked steps in test_oracle_pins.py).

Bar: the losses along the trajectory agree to 1e-8 relative, and the final parameters
to 1e-2 of the learning rate.  Both gradients are exact FP64 derivatives that differ by
summation order (~1e-12 relative); Adam's update g / (sqrt(v) + eps) is continuous in g,
so that difference reaches theta scaled by at most lr / eps times itself on components
with |g| below eps, where the loss is flat.  A wrong sign, a missing bias correction or
a skipped step moves theta by about lr.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle, set_threads
from oracle import torch_ref as TR
from test_gpu_grad import _frames, _targets

pytestmark = pytest.mark.gpu
set_threads(8)


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    return D


def test_train_matches_oracle_loop(dp, tiny_model):
    from paper_2004_11658_amd import train as T
    frames = _frames("tiny")
    print("train case tiny", [len(f[1]) for f in frames], flush=True)
    o = Oracle(tiny_model)
    tg = _targets(o, frames, 9)
    lam, lr, steps = 0.5, 1e-3, 4
    arch = TR.Arch(tiny_model)
    ofr = []
    for (c, t, b), (Et, Ft) in zip(frames, tg):
        nl, img, _, _ = o.nlist(c, t, b)
        ofr.append((c, t, b, nl, img, Et, Ft))
    th = arch.params.copy()
    m, v = np.zeros_like(th), np.zeros_like(th)
    ref_losses = []
    for step in range(1, steps + 1):
        L, g = TR.loss_and_grad(arch, th, ofr, lam)
        ref_losses.append(L)
        th, m, v = TR.adam_step(th, m, v, g, step, lr)
    model = dp.DPModel(tiny_model)
    coords = np.concatenate([f[0] for f in frames])
    types = np.concatenate([f[1] for f in frames])
    boxes = np.stack([f[2] for f in frames])
    off = np.concatenate([[0], np.cumsum([len(f[1]) for f in frames])])
    losses = T.train(model, coords, types, off, boxes, [x[0] for x in tg], np.concatenate([x[1] for x in tg]),
                     steps, lr=lr, lam=lam)
    print("losses gpu", losses, "ref", ref_losses, flush=True)
    for a, b in zip(losses, ref_losses):
        assert abs(a - b) <= 1e-8 * abs(b)
    assert ref_losses[-1] < ref_losses[0]
    d = np.abs(model.get_params().cpu().numpy() - th).max()
    print("theta max diff", d, flush=True)
    assert d <= 1e-2 * lr
