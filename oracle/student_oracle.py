"""FP64 CPU oracle of the distilled student's training step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP path.

The student is the same PWC-shaped light flow network as the per-frame path
(Sec. 3.2), narrower and shallower, trained to reproduce the flows of the
full network (the teacher).  This module restates that network's forward
pass with batched torch float64 CPU ops so that torch's reverse-mode
autograd (a library primitive) supplies exact gradients, and writes out:

* the multi-scale training loss of the supplementary material: one term per
  flow estimator, each the robust loss of Eq. S2, mean over pixels of
  (|du| + |dv| + eps)^q, against the teacher flow downscaled to that level
  (mean over each 2^l x 2^l block, divided by 2^l so that it is in level-l
  pixels), the terms weighted equally (Sec. 3.2, "Training");
* one AdamW step (decoupled weight decay; Sec. 3.2 names AdamW).

Pins (tests/test_oracle_student.py): the forward pass equals the numpy
oracle's network; gradients equal central finite differences of the loss;
the loss of a constructed constant-flow network has a closed form; the AdamW
step equals torch.optim.AdamW; block means of constant and ramp fields have
closed forms.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fnn

from oracle import tcflow_oracle as O

DT = torch.float64
TRAIN_DEFAULTS = dict(lr=1e-4, beta1=0.9, beta2=0.99, eps=1e-8, weight_decay=4e-4,
                      loss_eps=0.01, loss_q=0.4)


def lrelu(z, s):
    return torch.where(z >= 0, z, s * z)


def pad_frames(x, levels):
    """Edge-replicate the bottom and right borders up to a multiple of 2^L
    (x: (N, C, H, W))."""
    m = 2 ** levels
    H, W = x.shape[-2:]
    Hp, Wp = -(-H // m) * m, -(-W // m) * m
    if Hp == H and Wp == W:
        return x
    return Fnn.pad(x, (0, Wp - W, 0, Hp - H), mode="replicate")


def up2(f):
    """Bilinear 2x upsampling, half-pixel centres, source index clamped."""
    def taps(n):
        src = torch.clamp((torch.arange(2 * n, dtype=DT) + 0.5) / 2.0 - 0.5, 0.0, n - 1)
        i0 = torch.floor(src).long()
        i1 = torch.clamp(i0 + 1, max=n - 1)
        return i0, i1, src - i0
    h, w = f.shape[-2:]
    r0, r1, ry = taps(h)
    c0, c1, rx = taps(w)
    rows = f[:, :, r0, :] * (1 - ry)[:, None] + f[:, :, r1, :] * ry[:, None]
    return rows[:, :, :, c0] * (1 - rx) + rows[:, :, :, c1] * rx


def warp_zero(F, flow):
    """out(x) = F(x + flow(x)), bilinear, taps outside the image give zero.
    F: (N, C, h, w); flow: (N, 2, h, w).  Differentiable in F and flow."""
    N, C, h, w = F.shape
    yy, xx = torch.meshgrid(torch.arange(h, dtype=DT), torch.arange(w, dtype=DT), indexing="ij")
    sx = xx + flow[:, 0]
    sy = yy + flow[:, 1]
    x0 = torch.floor(sx).detach()
    y0 = torch.floor(sy).detach()
    ax, ay = sx - x0, sy - y0
    Fl = F.reshape(N, C, h * w)
    out = torch.zeros_like(F)
    for dy, wy in ((0, 1 - ay), (1, ay)):
        for dx, wx in ((0, 1 - ax), (1, ax)):
            xi, yi = (x0 + dx).long(), (y0 + dy).long()
            ok = (xi >= 0) & (xi <= w - 1) & (yi >= 0) & (yi <= h - 1)
            idx = (yi.clamp(0, h - 1) * w + xi.clamp(0, w - 1)).reshape(N, 1, h * w)
            v = torch.gather(Fl, 2, idx.expand(N, C, h * w)).reshape(N, C, h, w)
            out = out + torch.where(ok, wx * wy, torch.zeros_like(wx))[:, None] * v
    return out


def cost_volume(F1, F2w, r, slope):
    """lrelu((1/C) sum_c F1(x) F2w(x + d)), d row-major with dy outer, zero
    outside the image."""
    N, C, h, w = F1.shape
    P = Fnn.pad(F2w, (r, r, r, r))
    out = []
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            sh = P[:, :, r + dy:r + dy + h, r + dx:r + dx + w]
            out.append((F1 * sh).sum(1) / C)
    return lrelu(torch.stack(out, 1), slope)


def conv(x, wb, stride=1):
    w, b = wb
    return Fnn.conv2d(x, w, b, stride=stride, padding=1)


def student_flows(A, B, wts, desc):
    """Per-level flows [flow_1, ..., flow_L] (level-l pixels) of the network
    from frames A to frames B (N, 3, H, W), on the padded grid."""
    L, s = desc["levels"], desc["leaky"]
    x = pad_frames(torch.cat([A, B], 0), L)
    N = A.shape[0]
    feats = []
    for l in range(1, L + 1):
        x = lrelu(conv(x, wts[f"pyr{l}a"], 2), s)
        x = lrelu(conv(x, wts[f"pyr{l}b"]), s)
        feats.append(x)
    flows = [None] * L
    flow = None
    for l in range(L, 0, -1):
        F1, F2 = feats[l - 1][:N], feats[l - 1][N:]
        U = torch.zeros((N, 2) + F1.shape[-2:], dtype=DT) if flow is None else 2.0 * up2(flow)
        cv = cost_volume(F1, warp_zero(F2, U), desc["radius"], s)
        z = torch.cat([cv, F1, U], 1)
        h1 = lrelu(conv(z, wts[f"dec{l}c1"]), s)
        h2 = lrelu(conv(h1, wts[f"dec{l}c2"]), s)
        h3 = lrelu(conv(h2, wts[f"dec{l}c3"]), s)
        flow = U + conv(torch.cat([h2, h3], 1), wts[f"dec{l}head"])
        flows[l - 1] = flow
    return flows


def level_targets(T, levels):
    """Teacher flow (N, 2, H, W) in input pixels -> per-level targets: the
    flow edge-padded to the network's grid, averaged over 2^l x 2^l blocks and
    divided by 2^l."""
    Tp = pad_frames(T, levels)
    return [Fnn.avg_pool2d(Tp, 2 ** l) / 2 ** l for l in range(1, levels + 1)]


def robust_loss(flows, targets, eps, q):
    """Equally weighted sum over levels of mean_x (|du| + |dv| + eps)^q."""
    tot = 0.0
    for f, t in zip(flows, targets):
        tot = tot + ((f - t).abs().sum(1) + eps).pow(q).mean()
    return tot


def _params(blob, desc):
    wts = O.unpack_weights(blob, desc)
    tw = {k: (torch.tensor(w, dtype=DT, requires_grad=True),
              torch.tensor(b, dtype=DT, requires_grad=True)) for k, (w, b) in wts.items()}
    return tw


def _flatten(tw, attr):
    parts = []
    for w, b in tw.values():
        for t in (w, b):
            v = getattr(t, attr) if attr else t
            parts.append(v.detach().reshape(-1))
    return torch.cat(parts).numpy()


def loss_and_grad(blob, A, B, T, desc, prm=None):
    """Loss and its gradient (blob layout) for frames A, B (N, 3, H, W) and
    teacher flows T (N, 2, H, W), all float64."""
    prm = dict(TRAIN_DEFAULTS, **(prm or {}))
    tw = _params(blob, desc)
    A, B, T = (torch.as_tensor(np.asarray(x), dtype=DT) for x in (A, B, T))
    flows = student_flows(A, B, tw, desc)
    loss = robust_loss(flows, level_targets(T, desc["levels"]), prm["loss_eps"], prm["loss_q"])
    loss.backward()
    return float(loss.detach()), _flatten(tw, "grad")


def loss_only(blob, A, B, T, desc, prm=None):
    prm = dict(TRAIN_DEFAULTS, **(prm or {}))
    with torch.no_grad():
        tw = _params(blob, desc)
        A, B, T = (torch.as_tensor(np.asarray(x), dtype=DT) for x in (A, B, T))
        flows = student_flows(A, B, tw, desc)
        return float(robust_loss(flows, level_targets(T, desc["levels"]), prm["loss_eps"],
                                 prm["loss_q"]))


def adamw_step(p, g, m, v, t, prm=None):
    """One AdamW step (t = 1, 2, ...): decoupled decay p <- p (1 - lr wd),
    then the bias-corrected Adam update.  Returns new (p, m, v)."""
    prm = dict(TRAIN_DEFAULTS, **(prm or {}))
    lr, b1, b2, eps, wd = prm["lr"], prm["beta1"], prm["beta2"], prm["eps"], prm["weight_decay"]
    p = np.asarray(p, np.float64) * (1 - lr * wd)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
