"""Training loop of a DP model on energy and force labels.

The paper trains its models elsewhere and notes that training is cheap next to MD
(Sec. 1); it needs the forces' parameter gradient, which Remark 2's double back
propagation gives.  This loop fits the flat parameter vector theta of a loaded model to
labelled frames by Adam on the usual energy + force least-squares loss

    L(theta) = sum_f (E_f - E*_f)^2 / N_f + lam * sum_i |F_i - F*_i|^2,

one full batch per step.  Each step runs three library calls on the device: the batched
energies and forces (dp_compute_batch), the parameter gradient for the loss's seeds
gE_f = 2 (E_f - E*_f) / N_f and gF_i = 2 lam (F_i - F*_i) (dp_param_grad), and the Adam
update (dp_adam), after which the model takes the new theta (dp_set_params).
"""
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

from . import dp as D


def train(model: "D.DPModel", coords, types, offsets: Sequence[int], boxes, E_ref, F_ref, steps: int,
          lr: float = 1e-3, lam: float = 1.0, betas=(0.9, 0.999), eps: float = 1e-8,
          callback: Optional[Callable[[int, float], None]] = None) -> List[float]:
    """Run `steps` Adam steps from the model's current parameters; returns the loss
    before each step (the loss at theta_0, ..., theta_{steps-1}).  The model holds the
    final parameters on return."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nf = len(off) - 1
    dev = torch.device("cuda")
    nat = torch.as_tensor(np.diff(off), dtype=torch.float64, device=dev)
    Et = torch.as_tensor(np.asarray(E_ref, dtype=np.float64).reshape(nf), device=dev)
    Ft = torch.as_tensor(np.asarray(F_ref, dtype=np.float64).reshape(-1, 3), device=dev)
    x = torch.as_tensor(np.asarray(coords, dtype=np.float64).reshape(-1, 3), device=dev)
    t = torch.as_tensor(np.asarray(types, dtype=np.int32), device=dev)
    theta = model.get_params()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    losses = []
    for step in range(1, steps + 1):
        E, F, _ = model.compute_batch(x, t, off, boxes)
        dE = E.reshape(nf) - Et
        dF = F.reshape(-1, 3) - Ft
        L = float(((dE * dE) / nat).sum() + lam * (dF * dF).sum())
        losses.append(L)
        if callback is not None:
            callback(step - 1, L)
        g = model.param_grad(x, t, off, boxes, 2.0 * dE / nat, (2.0 * lam) * dF)
        D.adam_step(theta, m, v, g, step, lr, betas[0], betas[1], eps)
        model.set_params(theta)
    return losses
