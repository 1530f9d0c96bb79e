"""FP64 CPU oracle of the per-frame hot path: lite flow network + consistency step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code with
the HIP path (no kernels, headers, helpers or constants); the two meet only in
the seeded inputs they are both given.

Everything is plain numpy float64, written for a reader to check against the
paper by eye; convolutions are im2col in row bands followed by one BLAS matmul,
the only library primitive used.

What it follows (paper: "Interactive Control over Temporal Consistency while
Stylizing Video Streams"):

* Sec. 3.1, problem statement: given input frames I and per-frame stylized
  frames P, produce O with O_1 = P_1 and O_t computed from O_{t-1}.
* Sec. 3.1, Eq. 4: the global term G_t = Gamma(O_{t-1}), Gamma a backward warp
  by optical flow.
* Sec. 3.1, Eq. 5: the blend A_t = w_p G_t + (1 - w_p) L_t, whose upper clamp
  k_1 of w_p is the interactive share of global consistency ("Consistency
  Control Modes").  Here the strength alpha takes the role of k_1, w_p is
  alpha times a binary visibility mask and L_t = P_t; the output is A_t (the
  limit of Eq. 1 where the smoothness term dominates).  These readings are
  listed in the design notes.
* Sec. 5, Eq. 9: the non-occlusion mask is the forward-backward consistency
  check; its threshold is 0.01 (|f_b|^2 + |f~_f|^2) + 0.5.
* Sec. 3.2 and supplementary S1: the flow network is PWC-Net-shaped (feature
  pyramid, warping, correlation, CNN flow estimator per level, coarse to
  fine) with "light" estimators that keep a dense connection only into the
  last layer.
* Supplementary Eq. S1: the end-point error.
* Sec. 4.1, implementation details: the fast preset computes the flow on
  half-sized inputs (2 x 2 block means here) and upsamples it back; Sec. 4.2,
  parameter settings: the "objective" and final parameter sets.
* Sec. 3.2, "Optimized Network Architecture", and the supplementary ablation
  of the flow estimators and the refinement: the network variant without the
  estimator of the finest level (its flow, at the next level, is upsampled
  bilinearly to the input size) and the refinement network whose standard
  convolutions are replaced by depthwise separable ones ("-sepref").

Parity status: every op (pad, conv, LeakyReLU, up2, warp, cost volume, mask,
blend) is pinned by tests/test_oracle.py against closed forms, brute force,
library routines and exact invariants; the level recursion and the decoder's
channel order are pinned with constructed weights.  The composition of the
random-weight network as a whole has no published value to pin against.
The variants' ops (integer-factor upsampling, dilated depthwise and pointwise
convs) and their composition (input order, dilation per layer, dropped level,
output scale) are pinned by tests/test_oracle_variants.py.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# weights


def unpack_weights(blob, desc):
    """Split the flat float32 weight blob into {name: (W, b)} in float64.

    Blob layout, layer after layer: W[cout][cin][3][3] then b[cout].  Order:
    pyramid convs of level 1..L (stride 2 then stride 1), then the decoder of
    every level that has one, f..L with f = desc["finest"] (c1, c2, c3, head),
    then the separable refinement layers: a depthwise 3x3 W[c][3][3], b[c],
    then a pointwise W[cout][cin], b[cout].
    """
    L, ch, dec, r = desc["levels"], desc["ch"], desc["dec"], desc["radius"]
    ncv = (2 * r + 1) * (2 * r + 1)
    names = []
    for l in range(1, L + 1):
        names.append((f"pyr{l}a", (ch[l - 1], 3 if l == 1 else ch[l - 2], 3, 3)))
        names.append((f"pyr{l}b", (ch[l - 1], ch[l - 1], 3, 3)))
    for l in range(desc.get("finest", 1), L + 1):
        names.append((f"dec{l}c1", (dec[0], ncv + ch[l - 1] + 2, 3, 3)))
        names.append((f"dec{l}c2", (dec[1], dec[0], 3, 3)))
        names.append((f"dec{l}c3", (dec[2], dec[1], 3, 3)))
        names.append((f"dec{l}head", (2, dec[1] + dec[2], 3, 3)))
    width = dec[1] + dec[2] + 2
    for j, co in enumerate((desc.get("refine") or {}).get("ch", []), start=1):
        names.append((f"ref{j}dw", (width, 3, 3)))
        names.append((f"ref{j}pw", (co, width)))
        width = co
    blob = np.asarray(blob, dtype=np.float64).ravel()
    out, pos = {}, 0
    for name, shape in names:
        n = int(np.prod(shape))
        w = blob[pos:pos + n].reshape(shape)
        pos += n
        b = blob[pos:pos + shape[0]]
        pos += shape[0]
        out[name] = (w, b)
    if pos != blob.size:
        raise ValueError(f"weight blob has {blob.size} floats, layout needs {pos}")
    return out


# --------------------------------------------------------------------------
# elementary ops


def lrelu(z, slope=0.1):
    """LeakyReLU: z where z >= 0, slope * z elsewhere."""
    return np.where(z >= 0, z, slope * z)


def pad_frame(img, levels):
    """Edge-replicate the bottom and right borders up to a multiple of 2^L.

    img: (C, H, W).  The network halves the resolution L times, so every
    level must have integer size.
    """
    m = 2 ** levels
    C, H, W = img.shape
    Hp, Wp = -(-H // m) * m, -(-W // m) * m
    return np.pad(img, ((0, 0), (0, Hp - H), (0, Wp - W)), mode="edge")


def conv3x3(x, w, b, stride=1, band_bytes=96 << 20):
    """3x3 cross-correlation with zero padding 1 and the given stride.

    y[o, i, j] = b[o] + sum_{c,p,q} w[o, c, p, q] * x[c, s*i + p - 1, s*j + q - 1]

    x: (Cin, H, W); w: (Cout, Cin, 3, 3); b: (Cout,).  Output rows are
    produced in bands so the im2col matrix stays within ``band_bytes``.
    """
    x = np.asarray(x, np.float64)
    cin, H, W = x.shape
    cout = w.shape[0]
    s = stride
    Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    wm = np.asarray(w, np.float64).reshape(cout, cin * 9)
    out = np.empty((cout, Ho, Wo))
    band = max(1, int(band_bytes // (cin * 9 * Wo * 8)))
    for r0 in range(0, Ho, band):
        r1 = min(Ho, r0 + band)
        nr = r1 - r0
        cols = np.empty((cin, 3, 3, nr, Wo))
        for p in range(3):
            for q in range(3):
                cols[:, p, q] = xp[:, s * r0 + p: s * (r1 - 1) + p + 1: s,
                                   q: q + s * (Wo - 1) + 1: s]
        out[:, r0:r1] = (wm @ cols.reshape(cin * 9, nr * Wo)).reshape(cout, nr, Wo)
    out += np.asarray(b, np.float64)[:, None, None]
    return out


def up2(f):
    """Bilinear 2x upsampling, half-pixel centres (align_corners=False).

    Output index i samples the input at (i + 1/2)/2 - 1/2, clamped to
    [0, n-1]; separable over rows and columns.  f: (C, h, w) -> (C, 2h, 2w).
    """
    def axis_taps(n):
        src = np.clip((np.arange(2 * n) + 0.5) / 2.0 - 0.5, 0.0, n - 1)
        i0 = np.floor(src).astype(np.int64)
        i1 = np.minimum(i0 + 1, n - 1)
        return i0, i1, src - i0

    C, h, w = f.shape
    r0, r1, ry = axis_taps(h)
    c0, c1, rx = axis_taps(w)
    rows = f[:, r0, :] * (1 - ry)[None, :, None] + f[:, r1, :] * ry[None, :, None]
    return rows[:, :, c0] * (1 - rx)[None, None, :] + rows[:, :, c1] * rx[None, None, :]


def upsample(f, s):
    """Bilinear upsampling by an integer factor s, half-pixel centres
    (align_corners=False): output index i samples the input at
    (i + 1/2)/s - 1/2, clamped to [0, n-1].  (C, h, w) -> (C, s h, s w).
    For s = 2 this is up2."""
    def axis_taps(n):
        src = np.clip((np.arange(s * n) + 0.5) / s - 0.5, 0.0, n - 1)
        i0 = np.floor(src).astype(np.int64)
        i1 = np.minimum(i0 + 1, n - 1)
        return i0, i1, src - i0

    C, h, w = f.shape
    r0, r1, ry = axis_taps(h)
    c0, c1, rx = axis_taps(w)
    rows = f[:, r0, :] * (1 - ry)[None, :, None] + f[:, r1, :] * ry[None, :, None]
    return rows[:, :, c0] * (1 - rx)[None, None, :] + rows[:, :, c1] * rx[None, None, :]


def _bilinear_taps(flow):
    h, w = flow.shape[1:]
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    sx = xx + flow[0]
    sy = yy + flow[1]
    x0, y0 = np.floor(sx), np.floor(sy)
    return sx, sy, x0.astype(np.int64), y0.astype(np.int64), sx - x0, sy - y0


def warp_zero(F, flow):
    """Backward warp Gamma: out(x) = F(x + flow(x)), bilinear.

    Taps at floor and floor + 1 in each axis; a tap outside the image
    contributes zero.  F: (C, h, w); flow: (2, h, w), channel 0 = dx.
    """
    C, h, w = F.shape
    _, _, x0, y0, ax, ay = _bilinear_taps(flow)
    out = np.zeros_like(F, dtype=np.float64)
    for dy, wy in ((0, 1 - ay), (1, ay)):
        for dx, wx in ((0, 1 - ax), (1, ax)):
            xi, yi = x0 + dx, y0 + dy
            ok = (xi >= 0) & (xi <= w - 1) & (yi >= 0) & (yi <= h - 1)
            v = F[:, np.clip(yi, 0, h - 1), np.clip(xi, 0, w - 1)]
            out += np.where(ok, wx * wy, 0.0)[None] * v
    return out


def warp_clamp(F, flow):
    """Backward warp with tap indices clamped to the image (border value)."""
    C, h, w = F.shape
    _, _, x0, y0, ax, ay = _bilinear_taps(flow)
    out = np.zeros_like(F, dtype=np.float64)
    for dy, wy in ((0, 1 - ay), (1, ay)):
        for dx, wx in ((0, 1 - ax), (1, ax)):
            xi = np.clip(x0 + dx, 0, w - 1)
            yi = np.clip(y0 + dy, 0, h - 1)
            out += (wx * wy)[None] * F[:, yi, xi]
    return out


def cost_volume(F1, F2w, radius=4, slope=0.1):
    """Correlation layer: 81 channels for radius 4.

    CV[k, y, x] = lrelu( (1/C) sum_c F1[c, y, x] * F2w[c, y + dy, x + dx] ),
    k = (dy + r)(2r + 1) + (dx + r), dy, dx in [-r, r]; a displaced position
    outside the image gives a zero product.
    """
    C, h, w = F1.shape
    n = 2 * radius + 1
    cv = np.zeros((n * n, h, w))
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            k = (dy + radius) * n + (dx + radius)
            ys0, ys1 = max(0, -dy), min(h, h - dy)
            xs0, xs1 = max(0, -dx), min(w, w - dx)
            if ys0 >= ys1 or xs0 >= xs1:
                continue
            a = F1[:, ys0:ys1, xs0:xs1]
            bb = F2w[:, ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
            cv[k, ys0:ys1, xs0:xs1] = np.einsum("chw,chw->hw", a, bb) / C
    return lrelu(cv, slope)


# --------------------------------------------------------------------------
# network


def pyramid(img_padded, wts, desc):
    """Feature pyramid: per level a stride-2 conv then a stride-1 conv, each
    followed by LeakyReLU.  Returns [F^1, ..., F^L], F^l: (C_l, H/2^l, W/2^l).
    """
    slope = desc["leaky"]
    x = np.asarray(img_padded, np.float64)
    feats = []
    for l in range(1, desc["levels"] + 1):
        x = lrelu(conv3x3(x, *wts[f"pyr{l}a"], stride=2), slope)
        x = lrelu(conv3x3(x, *wts[f"pyr{l}b"], stride=1), slope)
        feats.append(x)
    return feats


def decode_level(l, F1, F2, U, wts, desc, features=False):
    """One light flow estimator at level l.

    Warp the second image's features by the upsampled flow U, correlate with
    the first image's features, and estimate a flow increment from
    [cost volume | F1 | U] with three conv layers; the head sees the last two
    layers' outputs [h2 | h3].  Returns flow_l = U + increment (and, with
    ``features``, also h2 and h3).
    """
    slope = desc["leaky"]
    F2w = warp_zero(F2, U)
    cv = cost_volume(F1, F2w, desc["radius"], slope)
    z = np.concatenate([cv, F1, U], axis=0)
    h1 = lrelu(conv3x3(z, *wts[f"dec{l}c1"]), slope)
    h2 = lrelu(conv3x3(h1, *wts[f"dec{l}c2"]), slope)
    h3 = lrelu(conv3x3(h2, *wts[f"dec{l}c3"]), slope)
    delta = conv3x3(np.concatenate([h2, h3], axis=0), *wts[f"dec{l}head"])
    if features:
        return U + delta, h2, h3
    return U + delta


def depthwise3x3(x, w, b, dilation):
    """Depthwise 3x3 cross-correlation with the given dilation, zero padding:
    y[c, i, j] = b[c] + sum_{p,q} w[c, p, q] x[c, i + (p-1) d, j + (q-1) d]."""
    C, H, W = x.shape
    d = dilation
    xp = np.zeros((C, H + 2 * d, W + 2 * d))
    xp[:, d:d + H, d:d + W] = x
    y = np.repeat(np.asarray(b, np.float64)[:, None, None], H, axis=1).repeat(W, axis=2)
    for p in range(3):
        for q in range(3):
            y = y + w[:, p, q][:, None, None] * xp[:, p * d:p * d + H, q * d:q * d + W]
    return y


def pointwise(x, w, b):
    """1x1 convolution: y[o] = b[o] + sum_c w[o, c] x[c]."""
    C, H, W = x.shape
    return (w @ x.reshape(C, H * W) + np.asarray(b)[:, None]).reshape(-1, H, W)


def refine(h2, h3, flow_f, wts, desc):
    """Separable refinement ("context") network on the finest estimator.

    Input [h2 | h3 | flow]; each layer is a depthwise 3x3 conv with its
    dilation, bias and LeakyReLU, then a pointwise conv with bias (LeakyReLU
    on all but the last layer, which outputs 2 channels); the result is added
    to the flow (Sec. 3.2, the "-sepref" design: the refinement's standard
    convolutions replaced by depthwise separable ones).
    """
    slope = desc["leaky"]
    dils = desc["refine"]["dil"]
    x = np.concatenate([h2, h3, flow_f], axis=0)
    for j, d in enumerate(dils, start=1):
        x = lrelu(depthwise3x3(x, *wts[f"ref{j}dw"], d), slope)
        x = pointwise(x, *wts[f"ref{j}pw"])
        if j < len(dils):
            x = lrelu(x, slope)
    return flow_f + x


def flow_from_pyramids(P1, P2, wts, desc, out_hw):
    """Coarse-to-fine flow from image 1 to image 2 given both pyramids.

    U_L = 0; U_l = 2 up2(flow_{l+1}) down to the finest estimator level f
    (1, or 2 with the finest estimator dropped); optionally refined; output
    crop(2^f upsample(flow_f, 2^f)) in pixels of the input resolution,
    cropped to ``out_hw``.
    """
    L = desc["levels"]
    f = desc.get("finest", 1)
    has_ref = bool((desc.get("refine") or {}).get("ch"))
    flow = None
    for l in range(L, f - 1, -1):
        F1, F2 = P1[l - 1], P2[l - 1]
        U = np.zeros((2,) + F1.shape[1:]) if flow is None else 2.0 * up2(flow)
        if l == f and has_ref:
            flow, h2, h3 = decode_level(l, F1, F2, U, wts, desc, features=True)
            flow = refine(h2, h3, flow, wts, desc)
        else:
            flow = decode_level(l, F1, F2, U, wts, desc)
    s = 2 ** f
    full = s * upsample(flow, s)
    H, W = out_hw
    return full[:, :H, :W]


def flow(A, B, wts, desc):
    """flow_estimate(prev=A, cur=B): flow from A to B on A's grid, (2, H, W)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    L = desc["levels"]
    PA = pyramid(pad_frame(A, L), wts, desc)
    PB = pyramid(pad_frame(B, L), wts, desc)
    return flow_from_pyramids(PA, PB, wts, desc, A.shape[1:])


def flow_pair(A, B, wts, desc):
    """(flow A->B, flow B->A) sharing the two pyramids."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    L = desc["levels"]
    PA = pyramid(pad_frame(A, L), wts, desc)
    PB = pyramid(pad_frame(B, L), wts, desc)
    hw = A.shape[1:]
    return (flow_from_pyramids(PA, PB, wts, desc, hw),
            flow_from_pyramids(PB, PA, wts, desc, hw))


# --------------------------------------------------------------------------
# the paper's fast preset: flow on half-sized inputs (Sec. 4.1)


def half_frame(img):
    """(C, h, w) -> (C, ceil(h/2), ceil(w/2)): the mean of each 2 x 2 pixel
    block; a block that runs past the last row or column repeats it (the
    image is extended by edge replication to even size first)."""
    img = np.asarray(img, np.float64)
    C, h, w = img.shape
    ext = np.pad(img, ((0, 0), (0, h % 2), (0, w % 2)), mode="edge")
    H2, W2 = ext.shape[1] // 2, ext.shape[2] // 2
    out = np.zeros((C, H2, W2))
    for dy in (0, 1):
        for dx in (0, 1):
            out += ext[:, dy::2, dx::2]
    return out / 4.0


def flow_pair_half(A, B, wts, desc):
    """Flow pair of the fast preset: both frames halved (half_frame), the
    pair estimated at that size, each flow upsampled by 2 (bilinear, half-pixel
    centres), cropped to the input size and multiplied by 2 (one half-size
    pixel spans two input pixels)."""
    A = np.asarray(A, np.float64)
    h, w = A.shape[1:]
    fa, fb = flow_pair(half_frame(A), half_frame(B), wts, desc)
    return tuple(2.0 * upsample(f, 2)[:, :h, :w] for f in (fa, fb))


# --------------------------------------------------------------------------
# consistency step


def consistency(P, Oprev, ffw, fbw, alpha):
    """One consistency step; returns (out, mask, margin, G).

    P = P_t, Oprev = O_{t-1}: (3, H, W); ffw = flow(I_{t-1} -> I_t) and
    fbw = flow(I_t -> I_{t-1}): (2, H, W); alpha in [0, 1].

    s = x + fbw(x) is where pixel x of frame t came from in frame t-1.
      G   = bilinear(O_{t-1}, s)      (Eq. 4, Gamma by backward warp)
      f~  = bilinear(ffw, s)
      m   = s inside the frame and |fbw + f~|^2 <= 0.01 (|fbw|^2 + |f~|^2) + 0.5
      w   = alpha * m                 (w_p with the clamp k_1 = alpha)
      out = (1 - w) P + w G           (Eq. 5 with L_t = P_t)
    ``margin`` is rhs - lhs of the test (m = inside and margin >= 0).
    """
    P = np.asarray(P, np.float64)
    Oprev = np.asarray(Oprev, np.float64)
    ffw = np.asarray(ffw, np.float64)
    fbw = np.asarray(fbw, np.float64)
    H, W = P.shape[1:]
    sx, sy, *_ = _bilinear_taps(fbw)
    inside = (sx >= 0) & (sx <= W - 1) & (sy >= 0) & (sy <= H - 1)
    G = warp_clamp(Oprev, fbw)
    ft = warp_clamp(ffw, fbw)
    lhs = (fbw[0] + ft[0]) ** 2 + (fbw[1] + ft[1]) ** 2
    rhs = 0.01 * (fbw[0] ** 2 + fbw[1] ** 2 + ft[0] ** 2 + ft[1] ** 2) + 0.5
    margin = rhs - lhs
    m = inside & (margin >= 0)
    w = alpha * m.astype(np.float64)
    out = (1.0 - w)[None] * P + w[None] * G
    return out, m, margin, G


def run_sequence(I, P, wts, desc, alpha):
    """O_1 = P_1; O_t = consistency(P_t, O_{t-1}, flow(I_{t-1}, I_t),
    flow(I_t, I_{t-1}), alpha).  Returns the list of O_t."""
    outs = [np.asarray(P[0], np.float64)]
    for t in range(1, len(I)):
        ffw, fbw = flow_pair(I[t - 1], I[t], wts, desc)
        outs.append(consistency(P[t], outs[-1], ffw, fbw, alpha)[0])
    return outs


# --------------------------------------------------------------------------
# metrics


def epe(a, b):
    """Mean end-point error over pixels (supplementary Eq. S1): mean |a - b|_2."""
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return float(np.mean(np.sqrt(d[0] ** 2 + d[1] ** 2)))


def warping_error(Vt, Vt1, flow_t_t1, mask):
    """Eq. 9: sum_i M_i |V_t - warp(V_{t+1})|_1 / sum_i M_i, with the warp a
    backward bilinear warp of V_{t+1} by the flow from t to t+1."""
    Vh = warp_clamp(np.asarray(Vt1, np.float64), np.asarray(flow_t_t1, np.float64))
    d = np.abs(np.asarray(Vt, np.float64) - Vh).sum(axis=0)
    M = np.asarray(mask, np.float64)
    return float((M * d).sum() / M.sum())


# --------------------------------------------------------------------------
# the paper's full consistency step (Sec. 3.1, Eq. 1-8)

PAPER_DEFAULTS = dict(k1=0.3, k2=0.5, a_ph=6.5e3, lam=2.0, eta=0.15, kappa=0.2, iters=150)

# Sec. 4.2, parameter settings: the final setting (= PAPER_DEFAULTS) and the
# one tuned for low warping error ("objective"); Sec. 4.1 and the caption of
# its runtime table: a fast preset with 50 iterations instead of 150, used
# with flow on half-sized inputs (flow_pair_half).
PAPER_PRESETS = {
    "final": dict(PAPER_DEFAULTS),
    "objective": dict(PAPER_DEFAULTS, k1=0.3, k2=0.3, a_ph=10e3, lam=0.7),
    "fast": dict(PAPER_DEFAULTS, iters=50),
}


def photometric_weight(I, Iw, a_ph):
    """Eq. 3: exp(-a_ph |I - Iw|^2), the squared norm over the RGB channels."""
    d = np.asarray(I, np.float64) - np.asarray(Iw, np.float64)
    return np.exp(-a_ph * (d ** 2).sum(axis=0))


def laplacian(X):
    """5-point Laplacian with Neumann borders: sum over the in-image
    4-neighbours of (neighbour - centre), per channel.  X: (C, H, W)."""
    X = np.asarray(X, np.float64)
    out = np.zeros_like(X)
    out[:, :, :-1] += X[:, :, 1:] - X[:, :, :-1]
    out[:, :, 1:] += X[:, :, :-1] - X[:, :, 1:]
    out[:, :-1, :] += X[:, 1:, :] - X[:, :-1, :]
    out[:, 1:, :] += X[:, :-1, :] - X[:, 1:, :]
    return out


def paper_reference(I_prev, I, I_next, P_prev, P, P_next, O_prev, f_tp, f_tn, prm):
    """A_t and w_c of the paper's consistency step.

    f_tp: flow from frame t to t-1 (on t's grid); f_tn: flow from t to t+1.
    Gamma is the backward bilinear warp with border clamping.
      w_p = min(exp(-a_ph |I_t - Gamma(I_{t-1})|^2), k1)      (Eq. 3 + clamp)
      w_n = min(exp(-a_ph |I_t - Gamma(I_{t+1})|^2), k2)
      L_t  = (1 - w_p - w_n) P_t + w_p Gamma(P_{t-1}) + w_n Gamma(P_{t+1})   (Eq. 2)
      G_t  = Gamma(O_{t-1})                                     (Eq. 4)
      A_t  = w_p G_t + (1 - w_p) L_t                            (Eq. 5)
      A^I_t = (1 - w_p - w_n) I_t + w_p Gamma(I_{t-1}) + w_n Gamma(I_{t+1})  (Eq. 6)
      w_c  = lambda exp(-a_ph |I_t - A^I_t|^2)                   (Eq. 7)
    Returns (A_t, w_c, w_p, w_n).
    """
    f_tp = np.asarray(f_tp, np.float64)
    f_tn = np.asarray(f_tn, np.float64)
    Ip_w = warp_clamp(np.asarray(I_prev, np.float64), f_tp)
    In_w = warp_clamp(np.asarray(I_next, np.float64), f_tn)
    Pp_w = warp_clamp(np.asarray(P_prev, np.float64), f_tp)
    Pn_w = warp_clamp(np.asarray(P_next, np.float64), f_tn)
    G = warp_clamp(np.asarray(O_prev, np.float64), f_tp)
    I = np.asarray(I, np.float64)
    P = np.asarray(P, np.float64)
    w_p = np.minimum(photometric_weight(I, Ip_w, prm["a_ph"]), prm["k1"])
    w_n = np.minimum(photometric_weight(I, In_w, prm["a_ph"]), prm["k2"])
    L = (1 - w_p - w_n)[None] * P + w_p[None] * Pp_w + w_n[None] * Pn_w
    A = w_p[None] * G + (1 - w_p)[None] * L
    AI = (1 - w_p - w_n)[None] * I + w_p[None] * Ip_w + w_n[None] * In_w
    w_c = prm["lam"] * photometric_weight(I, AI, prm["a_ph"])
    return A, w_c, w_p, w_n


def energy_gradient(O, P, A, w_c):
    """Gradient of the discrete Eq. 1, E = 1/2 sum |D(O - P)|^2 +
    1/2 sum w_c |O - A|^2 with forward differences D:
    -Laplacian(O - P) + w_c (O - A)."""
    return -laplacian(np.asarray(O) - P) + w_c[None] * (np.asarray(O) - A)


def poisson_solve(P, A, w_c, prm, O0=None):
    """Eq. 8, gradient descent with momentum on Eq. 1:
    O^{j+1} = O^j - eta grad E(O^j) + kappa (O^j - O^{j-1}),
    O^0 = O^{-1} = A_t (or O0), for prm['iters'] iterations."""
    P = np.asarray(P, np.float64)
    A = np.asarray(A, np.float64)
    O = np.array(A if O0 is None else O0, np.float64)
    O_old = O.copy()
    for _ in range(prm["iters"]):
        O_new = O - prm["eta"] * energy_gradient(O, P, A, w_c) + prm["kappa"] * (O - O_old)
        O_old, O = O, O_new
    return O


def paper_consistency(I_prev, I, I_next, P_prev, P, P_next, O_prev, f_tp, f_tn, prm=None):
    """O_t of the paper's step: reference A_t and weight w_c (Eq. 2-7), then
    the screened-Poisson solve (Eq. 1) by Eq. 8.  Returns (O_t, A_t, w_c)."""
    prm = dict(PAPER_DEFAULTS, **(prm or {}))
    A, w_c, _, _ = paper_reference(I_prev, I, I_next, P_prev, P, P_next, O_prev, f_tp, f_tn, prm)
    return poisson_solve(P, A, w_c, prm), A, w_c
