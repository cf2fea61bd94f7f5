"""Training driver of the student embedding nets (all arithmetic in libdp kernels).

For every species pair (alpha, beta) a student G_s(s) = tanh(s W1 + b1) W2 + b2
(1 -> hidden -> M) is fitted to the full embedding net on s values that the full model
visits along its own MD trajectory:
  1. run FP64 velocity-Verlet MD with the full model and keep frames,
  2. gather s of the real (alpha, beta) neighbours of those frames (dp_student_samples),
  3. evaluate the full net at those s (dp_embed_eval, FP64),
  4. fit: hidden units tanh(s W1 + b1) spread evenly over the sample range and the output
     layer by least squares (dp_student_lsq: design matrix, normal equations by GEMM,
     Cholesky on the device); then the hidden layer is trained by Adam with the loss
     gradient kernel (dp_student_loss_grad, dp_adam), the output layer re-solved by least
     squares after every step (variable projection).
The trained range [s_lo, s_hi] is the [1e-4, 1 - 1e-4] quantile range of the samples
(rarer, more extreme s values go to the full net), extended upward to twice its top value
with extra uniform points (closer approaches than the sampled frames hold); dp_set_student
installs the result.
The installed lower end is 0 when the trained one is tiny (below 1e-6 s_hi, the
neighbours just inside the cutoff): extrapolating the smooth student from s_lo down to
0 changes G by at most s_lo max|dG/ds|, and those neighbours enter T through
R~ = s (1, x/r, y/r, z/r) anyway, so they need no fallback.
Random numbers (neighbour subsampling) are drawn here with numpy PCG64 and passed to
the kernels.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np
import torch

from . import dp as D


def spread_hidden(hidden: int, s_lo: float, s_hi: float, kappa: float = 0.25):
    """Hidden layer tanh(s W1 + b1) with centres c_j spread evenly over [s_lo, s_hi] and
    slope kappa / spacing: a smooth, well-covering basis of the trained range."""
    cen = np.linspace(s_lo, s_hi, hidden)
    spacing = max((s_hi - s_lo) / max(hidden - 1, 1), 1e-12)
    W1 = np.full(hidden, kappa / spacing)
    return W1, -W1 * cen


def gather_samples(model: D.DPModel, frames, n_samples: int, seed: int, q: float = 1e-4):
    """s samples per species pair from frames [(coords device, types, box)], restricted to
    the [q, 1 - q] quantile range of what the frames contain."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out: Dict[Tuple[int, int], torch.Tensor] = {}
    nt = model.ntypes
    for a in range(nt):
        for b in range(nt):
            # counting pass (keep all), then keep with the probability giving ~n_samples
            total = 0
            for (x, t, box) in frames:
                u = torch.zeros(x.shape[0] * model.nm, dtype=torch.float32)
                _, c = model.student_samples(a, b, x, t, box, u, 1.0, 0)
                total += c
            keep = min(1.0, 1.05 * n_samples / max(total, 1))
            chunks = []
            got = 0
            for (x, t, box) in frames:
                u = torch.as_tensor(rng.random(x.shape[0] * model.nm, dtype=np.float32))
                s, c = model.student_samples(a, b, x, t, box, u, keep, n_samples - got)
                chunks.append(s)
                got += s.numel()
                if got >= n_samples:
                    break
            s = torch.cat(chunks)[:n_samples]
            sh = np.sort(s.cpu().numpy())
            lo = sh[int(q * (len(sh) - 1))]
            hi = sh[int((1.0 - q) * (len(sh) - 1))]
            out[(a, b)] = s[(s >= lo) & (s <= hi)].contiguous()
    return out


def train_pair(model: D.DPModel, alpha: int, beta: int, s: torch.Tensor, hidden: int,
               steps: int = 300, lr_rel: float = 2e-3, kappa: float = 0.25):
    """Fit one species pair.  Start: hidden units spread over the sample range and the
    output layer by least squares (GPU).  Then train the hidden layer by Adam on the loss
    gradient (dp_student_loss_grad), re-solving the output layer by least squares after
    every step, so the loss minimised is the variable-projection one, L(W1, b1) =
    min over (W2, b2) of the MSE; its gradient in (W1, b1) is the partial gradient at the
    least-squares output layer.  The step size is lr_rel times the initial slope |W1|
    (Adam moves every parameter by about lr per step).  Returns the best parameters, their
    loss, the loss of the least-squares start, the RMS of G and the sample range."""
    M = model.M
    G = model.embed_eval(alpha, beta, s)
    lo, hi = float(s.min()), float(s.max())
    W1, b1 = spread_hidden(hidden, lo, hi, kappa)
    th = torch.as_tensor(np.concatenate([W1, b1, np.zeros(hidden * M + M)]), device=s.device)
    D.student_lsq(hidden, M, s, G, th)
    loss, g, scratch = D.student_loss_grad(hidden, M, s, G, th)
    loss_lsq = float(loss.item())
    best, best_loss = th.clone(), loss_lsq
    mask = torch.zeros_like(th)
    mask[:2 * hidden] = 1.0
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    lr = lr_rel * float(np.abs(W1).mean())
    for step in range(1, steps + 1):
        D.adam_step(th, m, v, g * mask, step, lr)
        D.student_lsq(hidden, M, s, G, th)
        loss, g, scratch = D.student_loss_grad(hidden, M, s, G, th, scratch)
        lv = float(loss.item())
        if lv < best_loss:
            best, best_loss = th.clone(), lv
    return best, best_loss, loss_lsq, float(torch.sqrt((G * G).mean()).item()), lo, hi


def extend_upward(s: torch.Tensor, margin: float, frac: float, seed: int) -> torch.Tensor:
    """The samples plus frac * len(s) points spread uniformly over (s_max, s_max (1 + margin)]:
    s grows as neighbours approach, and MD runs longer than the sampled frames reach closer
    approaches; the full net is evaluated there like anywhere else."""
    if margin <= 0 or frac <= 0 or s.numel() == 0:
        return s
    hi = float(s.max())
    rng = np.random.Generator(np.random.PCG64(seed))
    extra = hi * (1.0 + margin * (1.0 - rng.random(max(1, int(frac * s.numel())))))
    return torch.cat([s, torch.as_tensor(extra, dtype=s.dtype, device=s.device)])


def train_students(model: D.DPModel, frames, hidden: int = 32, n_samples: int = 1_000_000,
                   seed_sample: int = 405, steps: int = 300, margin: float = 1.0,
                   margin_frac: float = 0.05):
    """Train one student per species pair; returns (theta_all, s_lo, s_hi, report).  The
    trained range reaches margin * s_max above the largest sampled s (margin_frac more
    samples there)."""
    samples = gather_samples(model, frames, n_samples, seed_sample)
    nt = model.ntypes
    thetas, los, his, report = [], [], [], {}
    for a in range(nt):
        for b in range(nt):
            s = extend_upward(samples[(a, b)], margin, margin_frac, seed_sample + 1 + a * nt + b)
            th, loss, loss_lsq, rms, lo, hi = train_pair(model, a, b, s, hidden, steps)
            thetas.append(th)
            los.append(0.0 if lo < 1e-6 * hi else lo)
            his.append(hi)
            report["%d-%d" % (a, b)] = dict(samples=int(s.numel()), s_lo=lo, s_hi=hi,
                                            rmse_rel=math.sqrt(loss) / rms,
                                            rmse_rel_lsq_start=math.sqrt(loss_lsq) / rms)
    return torch.cat(thetas), np.array(los), np.array(his), report
