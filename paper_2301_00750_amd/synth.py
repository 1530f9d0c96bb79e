"""Seeded synthetic inputs: network weights, frames, ground truth, fake stylizer.

This module only draws and renders inputs.  It holds none of the method's
arithmetic (no convolution, warp, cost volume or blend); both the FP64 oracle
and the HIP path receive the very same arrays from it.

Contents
  * ``load_desc(name)``       network/workload descriptor (JSON under configs/).
  * ``layer_shapes(desc)``    (name, cout, cin, taps) of every conv in blob order.
  * ``he_weights(desc)``      one flat float32 blob of He-normal weights.
  * ``tiny_pair()``           periodic value-noise frame and its copy rolled by
                              an integer flow (the 128x96 workload).
  * ``LayeredScene``          opaque textured layers under per-layer affine
                              motion, with analytic ground-truth flow and
                              occlusion (the 1920x1080 workload).
  * ``stylize(I, t)``         per-frame random colour map standing in for a
                              stylization network (it flickers from frame to
                              frame, which is what the method removes).

Weight blob layout (float32, little endian), layer after layer:
  W[cout][cin][taps] followed by b[cout]  (taps = 9 for a 3x3 kernel, 1 for a
  pointwise one; a depthwise layer has cin = 1).
Layer order: for level l = 1..L the two pyramid convs (stride 2: C_{l-1}->C_l,
then stride 1: C_l->C_l, with C_0 = 3); then for each level l = f..L that has
an estimator (f = ``finest``, 1 unless the finest estimator is dropped) the
decoder c1 (81+C_l+2 -> d1), c2 (d1 -> d2), c3 (d2 -> d3), head (d2+d3 -> 2);
then for each refinement layer j = 1..R its depthwise 3x3 (c_{j-1} channels,
c_0 = d2+d3+2) and its pointwise 1x1 (c_{j-1} -> c_j).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

_CFG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def load_desc(name: str) -> dict:
    """Read a network/workload descriptor (``tiny``, ``fullhd``, ...)."""
    path = name if name.endswith(".json") else os.path.join(_CFG_DIR, name + ".json")
    with open(path) as f:
        return json.load(f)


def finest(desc: dict) -> int:
    """Finest level with a flow estimator (2 when the finest one is dropped)."""
    return int(desc.get("finest", 1))


def refine_layers(desc: dict) -> list:
    """[(width, dilation)] of the separable refinement network (may be empty)."""
    r = desc.get("refine") or {}
    return list(zip(r.get("ch", []), r.get("dil", [])))


def layer_shapes(desc: dict) -> list:
    """(name, cout, cin, taps) of every conv in blob order."""
    L, ch, dec = desc["levels"], desc["ch"], desc["dec"]
    ncv = (2 * desc["radius"] + 1) ** 2
    out = []
    for l in range(1, L + 1):
        cin = 3 if l == 1 else ch[l - 2]
        out.append((f"pyr{l}a", ch[l - 1], cin, 9))
        out.append((f"pyr{l}b", ch[l - 1], ch[l - 1], 9))
    for l in range(finest(desc), L + 1):
        din = ncv + ch[l - 1] + 2
        out.append((f"dec{l}c1", dec[0], din, 9))
        out.append((f"dec{l}c2", dec[1], dec[0], 9))
        out.append((f"dec{l}c3", dec[2], dec[1], 9))
        out.append((f"dec{l}head", 2, dec[1] + dec[2], 9))
    cin = dec[1] + dec[2] + 2
    for j, (co, _) in enumerate(refine_layers(desc), start=1):
        out.append((f"ref{j}dw", cin, 1, 9))
        out.append((f"ref{j}pw", co, cin, 1))
        cin = co
    return out


def blob_floats(desc: dict) -> int:
    return sum(co * ci * k + co for _, co, ci, k in layer_shapes(desc))


def he_weights(desc: dict, seed: int | None = None) -> np.ndarray:
    """He-normal weights, std = sqrt(2 / fan_in) with fan_in = taps * cin, zero
    biases.

    Drawn with ``numpy.random.default_rng(seed)`` layer by layer in blob order.
    The layers that output a flow (the estimator heads and the last
    refinement layer) are additionally scaled by ``desc['head_gain']``.
    """
    rng = np.random.default_rng(desc.get("weight_seed", 0) if seed is None else seed)
    shapes = layer_shapes(desc)
    parts = []
    for i, (name, co, ci, k) in enumerate(shapes):
        w = rng.standard_normal((co, ci, k)) * math.sqrt(2.0 / (k * ci))
        if name.endswith("head") or (name.startswith("ref") and i == len(shapes) - 1):
            w = w * desc.get("head_gain", 1.0)
        parts.append(w.astype(np.float32).ravel())
        parts.append(np.zeros(co, np.float32))
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# value noise


def _smooth(f):
    return f * f * (3.0 - 2.0 * f)


class ValueNoise:
    """Periodic multi-octave value noise, evaluated at continuous coordinates.

    Octave k has a lattice of cell size ``cells[k]`` px with i.i.d. uniform
    [0,1) values per RGB channel, periodic with period ``period`` px; values
    between lattice points use smoothstep weights.  Octave amplitudes are
    1/2^k, normalised so the sum stays in [0, 1].
    """

    def __init__(self, period_x, period_y, cells, rng):
        self.cells = list(cells)
        self.lat = []
        for s in self.cells:
            assert period_x % s == 0 and period_y % s == 0
            self.lat.append(rng.random((3, period_y // s, period_x // s)))
        amp = np.array([0.5 ** k for k in range(len(self.cells))])
        self.amp = amp / amp.sum()

    def eval(self, u: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
        """u, v: (...) float tensors (x and y).  Returns (3, ...) in [0, 1]."""
        out = None
        for s, lat, a in zip(self.cells, self.lat, self.amp):
            lt = torch.as_tensor(lat, dtype=u.dtype, device=u.device)
            hy, wx = lt.shape[1], lt.shape[2]
            gx, gy = u / s, v / s
            x0, y0 = torch.floor(gx), torch.floor(gy)
            fx, fy = _smooth(gx - x0), _smooth(gy - y0)
            ix0 = torch.remainder(x0.long(), wx)
            iy0 = torch.remainder(y0.long(), hy)
            ix1 = torch.remainder(ix0 + 1, wx)
            iy1 = torch.remainder(iy0 + 1, hy)
            v00 = lt[:, iy0, ix0]
            v01 = lt[:, iy0, ix1]
            v10 = lt[:, iy1, ix0]
            v11 = lt[:, iy1, ix1]
            top = v00 + (v01 - v00) * fx
            bot = v10 + (v11 - v10) * fx
            val = (top + (bot - top) * fy) * a
            out = val if out is None else out + val
        return out


def tiny_pair(width=128, height=96, shift=(3, -2), seed=0):
    """(prev, cur, gt_fw, gt_bw) of the 128x96 workload.

    ``prev`` is periodic value noise (cells 32/16/8/4 px), ``cur`` is ``prev``
    rolled by ``shift`` = (dx, dy), so the exact forward flow is ``shift`` and
    the backward flow is ``-shift`` at every pixel (circularly).  Frames are
    (3, H, W) float32 in [0, 1]; flows are (2, H, W) float32.
    """
    rng = np.random.default_rng(seed)
    noise = ValueNoise(width, height, (32, 16, 8, 4), rng)
    yy, xx = torch.meshgrid(torch.arange(height, dtype=torch.float64),
                            torch.arange(width, dtype=torch.float64), indexing="ij")
    prev = noise.eval(xx, yy).float()
    cur = torch.roll(prev, shifts=(shift[1], shift[0]), dims=(1, 2))
    fw = torch.empty(2, height, width)
    fw[0], fw[1] = float(shift[0]), float(shift[1])
    return prev.contiguous(), cur.contiguous(), fw, -fw


# --------------------------------------------------------------------------
# layered affine scene


class LayeredScene:
    """Opaque textured layers under constant-velocity affine motion.

    Layer 0 is a full-frame background; layers 1..n-1 are ellipses drawn on
    top in order.  Layer k maps its own coordinates u (origin at the layer's
    centroid) to the screen as x = R(theta_k + t*omega_k) u + c_k + t*v_k.
    Velocities: translation uniform in a disc of radius ``max_shift`` px per
    frame, rotation uniform in [-max_rot_deg, max_rot_deg] degrees per frame.

    Ground truth: the forward flow of pixel x at frame t is the motion of the
    point of the topmost layer under x from frame t to t+1; it is occluded
    when that point leaves the frame or a higher layer covers it at t+1.
    """

    def __init__(self, width=1920, height=1080, n_layers=3, seed=0,
                 max_shift=8.0, max_rot_deg=1.0, cells=(64, 32, 16, 8)):
        rng = np.random.default_rng(seed)
        self.W, self.H = width, height
        self.layers = []
        for k in range(n_layers):
            noise = ValueNoise(2048, 2048, cells, rng)
            r = max_shift * math.sqrt(rng.random())
            phi = 2 * math.pi * rng.random()
            vel = (r * math.cos(phi), r * math.sin(phi))
            omega = math.radians(max_rot_deg) * (2 * rng.random() - 1)
            if k == 0:
                c0 = ((width - 1) / 2.0, (height - 1) / 2.0)
                axes = None
            else:
                c0 = (width * (0.25 + 0.5 * rng.random()), height * (0.25 + 0.5 * rng.random()))
                axes = (height * (0.15 + 0.2 * rng.random()), height * (0.15 + 0.2 * rng.random()))
            theta0 = 2 * math.pi * rng.random()
            self.layers.append(dict(noise=noise, vel=vel, omega=omega, c0=c0,
                                    axes=axes, theta0=theta0))

    def _pose(self, k, t):
        L = self.layers[k]
        th = L["theta0"] + t * L["omega"]
        cx = L["c0"][0] + t * L["vel"][0]
        cy = L["c0"][1] + t * L["vel"][1]
        return th, cx, cy

    def _to_layer(self, k, t, x, y):
        th, cx, cy = self._pose(k, t)
        c, s = math.cos(th), math.sin(th)
        dx, dy = x - cx, y - cy
        return c * dx + s * dy, -s * dx + c * dy

    def _to_screen(self, k, t, u, v):
        th, cx, cy = self._pose(k, t)
        c, s = math.cos(th), math.sin(th)
        return c * u - s * v + cx, s * u + c * v + cy

    def _inside(self, k, u, v):
        ax = self.layers[k]["axes"]
        if ax is None:
            return torch.ones_like(u, dtype=torch.bool)
        return (u / ax[0]) ** 2 + (v / ax[1]) ** 2 <= 1.0

    def _grid(self, device, dtype):
        yy, xx = torch.meshgrid(torch.arange(self.H, dtype=dtype, device=device),
                                torch.arange(self.W, dtype=dtype, device=device), indexing="ij")
        return xx, yy

    def top_layer(self, t, x, y):
        top = torch.zeros_like(x, dtype=torch.long)
        for k in range(1, len(self.layers)):
            u, v = self._to_layer(k, t, x, y)
            top = torch.where(self._inside(k, u, v), torch.full_like(top, k), top)
        return top

    def frame(self, t, device="cpu"):
        """I_t as (3, H, W) float32 in [0, 1]."""
        xx, yy = self._grid(device, torch.float64)
        img = None
        for k in range(len(self.layers)):
            u, v = self._to_layer(k, t, xx, yy)
            # textures live on a 2048-periodic lattice; shift u, v to positive
            col = self.layers[k]["noise"].eval(u + 4096.0, v + 4096.0)
            if img is None:
                img = col
            else:
                img = torch.where(self._inside(k, u, v)[None], col, img)
        return img.float().contiguous()

    def gt_flow(self, t, t2, device="cpu"):
        """Flow from frame t to frame t2 on frame t's grid and its occlusion.

        Returns (flow (2,H,W) float32, occluded (H,W) bool).
        """
        xx, yy = self._grid(device, torch.float64)
        top = self.top_layer(t, xx, yy)
        fx = torch.zeros_like(xx)
        fy = torch.zeros_like(yy)
        for k in range(len(self.layers)):
            u, v = self._to_layer(k, t, xx, yy)
            x2, y2 = self._to_screen(k, t2, u, v)
            sel = top == k
            fx = torch.where(sel, x2 - xx, fx)
            fy = torch.where(sel, y2 - yy, fy)
        x2, y2 = xx + fx, yy + fy
        occ = (x2 < 0) | (x2 > self.W - 1) | (y2 < 0) | (y2 > self.H - 1)
        top2 = self.top_layer(t2, x2, y2)
        occ = occ | (top2 > top)
        return torch.stack([fx, fy]).float().contiguous(), occ


# --------------------------------------------------------------------------
# stylizer stand-in

_STYLE_BASE = np.array([[0.393, 0.769, 0.189],
                        [0.349, 0.686, 0.168],
                        [0.272, 0.534, 0.131]])


def stylize(I: torch.Tensor, t: int, jitter=0.05) -> torch.Tensor:
    """P_t = clip(M_t I + b_t, 0, 1): a fixed colour matrix plus per-frame
    N(0, jitter) noise on the matrix and the offset, seed 1 + t."""
    rng = np.random.default_rng(1 + t)
    M = _STYLE_BASE + rng.normal(0.0, jitter, (3, 3))
    b = rng.normal(0.0, jitter, 3)
    Mt = torch.as_tensor(M, dtype=I.dtype, device=I.device)
    bt = torch.as_tensor(b, dtype=I.dtype, device=I.device)
    out = (Mt @ I.reshape(3, -1)).reshape(I.shape) + bt[:, None, None]
    return out.clamp_(0.0, 1.0).contiguous()
