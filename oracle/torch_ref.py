"""FP64 PyTorch-CPU reference of the DP-SE energy, differentiated by autograd.

TEST INFRASTRUCTURE ONLY (the oracle side; never imported by the product path).

It evaluates the same definitions as dp_oracle.c (Section 2, Eq. 1-9 of the paper) with
plain tensor operations, on a formatted neighbour list taken from the C oracle, and
lets autograd do what the paper's Remark 2 (Eq. 10) does by back propagation:
  * forces F = -dE/dr (an independent check of the C oracle's hand-written adjoint),
  * parameter gradients of the energy + force loss
        L = sum_f (E_f - E*_f)^2 / N_f + lam * sum_f sum_i |F_i - F*_i|^2
    by double back propagation,
  * the student embedding net (1 -> 32 tanh -> M affine) and its MSE loss gradient.
"""
from __future__ import annotations

import math
import struct

import numpy as np
import torch

torch.set_default_dtype(torch.float64)


class Arch:
    """Architecture read from a DPSEMDL1 model file (own parser)."""

    def __init__(self, path: str):
        with open(path, "rb") as f:
            buf = f.read()
        assert buf[:8] == b"DPSEMDL1"
        _ver, hb, npar = struct.unpack_from("<iiq", buf, 8)
        (self.ntypes, n_emb, n_fit, self.m2, self.switch_kind,
         self.desc_norm) = struct.unpack_from("<6i", buf, 24)
        self.rc, self.rcs = struct.unpack_from("<dd", buf, 48)
        ints = struct.unpack_from("<%di" % (n_emb + n_fit + self.ntypes), buf, 64)
        self.emb_w = list(ints[:n_emb])
        self.fit_w = list(ints[n_emb:n_emb + n_fit])
        self.sel = list(ints[n_emb + n_fit:])
        self.M = self.emb_w[-1]
        self.nm = sum(self.sel)
        self.params = np.frombuffer(buf, dtype="<f8", offset=hb, count=npar).copy()
        # (W offset, W shape, b offset) per layer
        off = 0
        self.emb = {}
        for a in range(self.ntypes):
            for b in range(self.ntypes):
                layers, nin = [], 1
                for w in self.emb_w:
                    layers.append((off, (nin, w), off + nin * w))
                    off += nin * w + w
                    nin = w
                self.emb[(a, b)] = layers
        self.fit = {}
        for a in range(self.ntypes):
            layers, nin = [], self.M * self.m2
            for w in self.fit_w + [1]:
                layers.append((off, (nin, w), off + nin * w))
                off += nin * w + w
                nin = w
            self.fit[a] = layers
        assert off == npar
        self.nparams = npar


def _layer(theta, spec):
    off, (ni, no), boff = spec
    return theta[off:off + ni * no].view(ni, no), theta[boff:boff + no]


def smooth(arch: Arch, r: torch.Tensor) -> torch.Tensor:
    """s(r) = w(r)/r with the switch of Section 2 (Eq. 5), C2 quintic or cosine."""
    u = ((r - arch.rcs) / (arch.rc - arch.rcs)).clamp(0.0, 1.0)
    if arch.switch_kind == 1:
        w = 0.5 * torch.cos(math.pi * u) + 0.5
    else:
        w = u ** 3 * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0
    w = torch.where(r < arch.rc, w, torch.zeros_like(w))
    return w / r


def embed(arch: Arch, theta, a: int, b: int, s: torch.Tensor) -> torch.Tensor:
    """Embedding net G^{a,b}(s) (Eq. 7-9): plain tanh first layer, then (x,x)+tanh."""
    h = None
    for k, spec in enumerate(arch.emb[(a, b)]):
        W, bias = _layer(theta, spec)
        if k == 0:
            h = torch.tanh(s[:, None] * W[0][None, :] + bias)
            continue
        t = torch.tanh(h @ W + bias)
        ni, no = W.shape
        if no == 2 * ni:
            h = torch.cat([h, h], dim=1) + t
        elif no == ni:
            h = h + t
        else:
            h = t
    return h


def fitting(arch: Arch, theta, a: int, x: torch.Tensor) -> torch.Tensor:
    """Fitting net of species a (Eq. 2-3) with an affine output layer."""
    layers = arch.fit[a]
    for spec in layers[:-1]:
        W, bias = _layer(theta, spec)
        t = torch.tanh(x @ W + bias)
        x = x + t if W.shape[0] == W.shape[1] else t
    W, bias = _layer(theta, layers[-1])
    return (x @ W + bias)[:, 0]


def box_K(arch: Arch, box: np.ndarray):
    Bi = np.linalg.inv(box)
    width = 1.0 / np.sqrt((Bi * Bi).sum(0))
    return [int(math.ceil(arch.rc / w)) for w in width]


def decode_img(img: np.ndarray, K):
    n2 = img % (2 * K[2] + 1) - K[2]
    q = img // (2 * K[2] + 1)
    n1 = q % (2 * K[1] + 1) - K[1]
    n0 = q // (2 * K[1] + 1) - K[0]
    return np.stack([n0, n1, n2], -1)


def energy(arch: Arch, theta: torch.Tensor, x: torch.Tensor, types: np.ndarray,
           box: np.ndarray, nlist: np.ndarray, img: np.ndarray, student=None, out=None):
    """E and E_i of one frame (Eq. 1) for a formatted neighbour list (Alg. 1).

    student: optional {(a, b): (theta_s, H, s_lo, s_hi)}: for those species pairs G(s)
    is the student net 1 -> H tanh -> M affine where s_lo <= s <= s_hi and the full
    net elsewhere.  out: optional dict that receives T [n][M][4] (Eq. 4)."""
    n = len(types)
    B = torch.as_tensor(box)
    K = box_K(arch, box)
    wrap = np.floor(x.detach().numpy() @ np.linalg.inv(box))     # integer image of each atom
    ii, kk = np.nonzero(nlist >= 0)
    jj = nlist[ii, kk].astype(np.int64)
    nimg = decode_img(img[ii, kk], K)
    shift = (nimg - wrap[jj] + wrap[ii]) @ box                    # integer lattice shift
    d = x[jj] - x[ii] + torch.as_tensor(shift)
    r = torch.sqrt((d * d).sum(1))
    s = smooth(arch, r)
    R = torch.cat([s[:, None], (s / r)[:, None] * d], dim=1)       # Eq. 5
    slot_type = np.zeros(arch.nm, np.int64)
    o = 0
    for t, c in enumerate(arch.sel):
        slot_type[o:o + c] = t
        o += c
    st = slot_type[kk]
    G = torch.zeros(len(ii), arch.M)
    ti = types[ii]
    for a in range(arch.ntypes):
        for b in range(arch.ntypes):
            m = np.nonzero((ti == a) & (st == b))[0]
            if m.size:
                g = embed(arch, theta, a, b, s[m])
                if student is not None and (a, b) in student:
                    ths, H, lo, hi = student[(a, b)]
                    gs = student_forward(torch.as_tensor(ths), H, arch.M, s[m])
                    inr = ((s[m] >= lo) & (s[m] <= hi))[:, None]
                    g = torch.where(inr, gs, g)
                G = G.index_copy(0, torch.as_tensor(m), g)
    norm = float(arch.nm) if arch.desc_norm == 0 else 1.0
    T = torch.zeros(n, arch.M, 4).index_add(0, torch.as_tensor(ii),
                                            G[:, :, None] * R[:, None, :]) / norm
    if out is not None:
        out["T"] = T
    D = torch.einsum("nac,nbc->nab", T, T[:, :arch.m2, :]).reshape(n, -1)   # Eq. 4
    Ei = torch.zeros(n)
    for a in range(arch.ntypes):
        m = np.nonzero(types == a)[0]
        if m.size:
            Ei = Ei.index_copy(0, torch.as_tensor(m), fitting(arch, theta, a, D[m]))
    return Ei.sum(), Ei


def energy_forces(arch: Arch, theta, coords, types, box, nlist, img, create_graph=False, student=None):
    x = torch.as_tensor(np.asarray(coords, np.float64)).clone().requires_grad_(True)
    E, Ei = energy(arch, theta, x, np.asarray(types), np.asarray(box), nlist, img, student)
    (gx,) = torch.autograd.grad(E, x, create_graph=create_graph)
    return E, -gx, Ei


def loss_and_grad(arch: Arch, theta_np: np.ndarray, frames, lam: float):
    """Energy + force loss over frames [(coords, types, box, nlist, img, E*, F*)] and
    its gradient with respect to the flat parameter vector (double back propagation)."""
    theta = torch.as_tensor(theta_np).clone().requires_grad_(True)
    L = torch.zeros(())
    for (coords, types, box, nlist, img, Et, Ft) in frames:
        E, F, _ = energy_forces(arch, theta, coords, types, box, nlist, img, create_graph=True)
        nat = len(types)
        L = L + (E - float(Et)) ** 2 / nat + lam * ((F - torch.as_tensor(Ft)) ** 2).sum()
    (g,) = torch.autograd.grad(L, theta)
    return float(L.detach()), g.numpy()


# ---------------------------------------------------------------------------------------
# student embedding net: 1 -> H (tanh) -> M (affine)
# ---------------------------------------------------------------------------------------

def student_layout(H: int, M: int):
    """Flat parameter layout of one student net: W1[1][H], b1[H], W2[H][M], b2[M]."""
    return dict(W1=(0, (1, H)), b1=(H, (H,)), W2=(2 * H, (H, M)), b2=(2 * H + H * M, (M,)),
                size=2 * H + H * M + M)


def student_forward(theta_s: torch.Tensor, H: int, M: int, s: torch.Tensor):
    lay = student_layout(H, M)
    W1 = theta_s[0:H]
    b1 = theta_s[H:2 * H]
    W2 = theta_s[2 * H:2 * H + H * M].view(H, M)
    b2 = theta_s[2 * H + H * M:2 * H + H * M + M]
    assert theta_s.numel() == lay["size"]
    h = torch.tanh(s[:, None] * W1[None, :] + b1)
    return h @ W2 + b2


def student_loss_grad(theta_np, H, M, s_np, target_np):
    """MSE over samples and outputs, L = mean (G_s(s) - G(s))^2, and dL/dtheta_s."""
    th = torch.as_tensor(theta_np).clone().requires_grad_(True)
    out = student_forward(th, H, M, torch.as_tensor(s_np))
    L = ((out - torch.as_tensor(target_np)) ** 2).mean()
    (g,) = torch.autograd.grad(L, th)
    return float(L.detach()), g.numpy()


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), bias-corrected, step t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
