"""Pins of the oracle's network variants (paper Sec. 3.2, "Optimized Network
Architecture"): the finest flow estimator dropped, and the refinement network
built from depthwise separable convolutions ("-sepref").

Each op is tied to a library routine used only here, a brute-force loop or a
closed form; the composition is pinned with constructed weights whose result
is known exactly.  CPU only.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn

from oracle import tcflow_oracle as O
from paper_2301_00750_amd import synth

RNG = np.random.default_rng(2301)


def rand(*shape):
    return RNG.standard_normal(shape)


# ---------------------------------------------------------------- upsample


@pytest.mark.parametrize("s", [2, 4, 8])
def test_upsample_vs_interpolate(s):
    f = rand(2, 5, 7)
    ref = Fnn.interpolate(torch.from_numpy(f)[None], scale_factor=s, mode="bilinear",
                          align_corners=False)[0].numpy()
    assert np.allclose(O.upsample(f, s), ref, rtol=0, atol=1e-13)


def test_upsample_x4_closed_form_interior():
    """Output 4i + k samples the input at i + (k + 1/2)/4 - 1/2."""
    f = rand(1, 1, 9)
    u = O.upsample(f, 4)[0, 0]
    g = f[0, 0]
    for i in range(1, 8):
        assert np.isclose(u[4 * i + 0], 0.375 * g[i - 1] + 0.625 * g[i], rtol=0, atol=1e-15)
        assert np.isclose(u[4 * i + 1], 0.125 * g[i - 1] + 0.875 * g[i], rtol=0, atol=1e-15)
        assert np.isclose(u[4 * i + 2], 0.875 * g[i] + 0.125 * g[i + 1], rtol=0, atol=1e-15)
        assert np.isclose(u[4 * i + 3], 0.625 * g[i] + 0.375 * g[i + 1], rtol=0, atol=1e-15)
    assert np.all(u[:2] == g[0]) and np.all(u[-2:] == g[-1])


def test_upsample_x2_is_up2():
    f = rand(2, 6, 5)
    assert np.allclose(O.upsample(f, 2), O.up2(f), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- separable convs


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_depthwise_vs_torch_conv2d(d):
    C = 6
    x, w, b = rand(C, 11, 13), rand(C, 3, 3), rand(C)
    ref = Fnn.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w)[:, None],
                     torch.from_numpy(b), padding=d, dilation=d, groups=C)[0].numpy()
    assert np.allclose(O.depthwise3x3(x, w, b, d), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p,q,d", [(0, 0, 1), (0, 2, 2), (2, 1, 3), (1, 0, 4)])
def test_depthwise_single_tap_is_a_shift(p, q, d):
    """A one-hot tap (p, q) reads x at (i + (p-1) d, j + (q-1) d), zero outside."""
    C, H, W = 2, 7, 9
    x = rand(C, H, W)
    w = np.zeros((C, 3, 3))
    w[:, p, q] = 1.0
    y = O.depthwise3x3(x, w, np.zeros(C), d)
    for c in range(C):
        for i in range(H):
            for j in range(W):
                ii, jj = i + (p - 1) * d, j + (q - 1) * d
                exp = x[c, ii, jj] if 0 <= ii < H and 0 <= jj < W else 0.0
                assert y[c, i, j] == exp


def test_pointwise_vs_brute_force():
    x, w, b = rand(5, 3, 4), rand(7, 5), rand(7)
    y = O.pointwise(x, w, b)
    for o in range(7):
        for i in range(3):
            for j in range(4):
                assert np.isclose(y[o, i, j], b[o] + sum(w[o, c] * x[c, i, j] for c in range(5)),
                                  rtol=0, atol=1e-13)


# ---------------------------------------------------------------- weights layout


def test_unpack_weights_variant_layout():
    """Marker blob: every layer starts where the layer sizes before it end,
    with no estimator at level 1 and the refinement after the decoders."""
    d = synth.load_desc("tiny_sepref")
    n = synth.blob_floats(d)
    wts = O.unpack_weights(np.arange(n, dtype=np.float64), d)
    assert "dec1c1" not in wts and "dec2c1" in wts
    ch, dec, L = d["ch"], d["dec"], d["levels"]
    pos = 0
    for l in range(1, L + 1):
        cin = 3 if l == 1 else ch[l - 2]
        pos += (ch[l - 1] * cin * 9 + ch[l - 1]) + (ch[l - 1] * ch[l - 1] * 9 + ch[l - 1])
    for l in range(2, L + 1):
        assert wts[f"dec{l}c1"][0].ravel()[0] == pos
        din = 81 + ch[l - 1] + 2
        pos += dec[0] * din * 9 + dec[0] + dec[1] * dec[0] * 9 + dec[1] \
            + dec[2] * dec[1] * 9 + dec[2] + 2 * (dec[1] + dec[2]) * 9 + 2
    width = dec[1] + dec[2] + 2
    for j, co in enumerate(d["refine"]["ch"], start=1):
        w, b = wts[f"ref{j}dw"]
        assert w.shape == (width, 3, 3) and w[0, 0, 0] == pos and b[0] == pos + 9 * width
        pos += 10 * width
        w, b = wts[f"ref{j}pw"]
        assert w.shape == (co, width) and w[0, 0] == pos and w[1, 0] == pos + width
        assert b[0] == pos + co * width
        pos += co * width + co
        width = co
    assert pos == n and width == 2


# ---------------------------------------------------------------- refinement


def _zero_weights(desc):
    blob = synth.he_weights(desc)
    return {k: (np.zeros_like(w), np.zeros_like(b)) for k, (w, b) in O.unpack_weights(blob, desc).items()}


def test_refine_zero_weights_adds_last_bias():
    d = synth.load_desc("tiny_sepref")
    wts = _zero_weights(d)
    R = len(d["refine"]["ch"])
    c = np.array([0.75, -1.5])
    wts[f"ref{R}pw"] = (wts[f"ref{R}pw"][0], c)
    h2, h3, fl = rand(64, 5, 6), rand(32, 5, 6), rand(2, 5, 6)
    out = O.refine(h2, h3, fl, wts, d)
    assert np.array_equal(out, fl + c[:, None, None])


def test_refine_input_order_and_per_layer_dilation():
    """Copy network: layer 1 picks h3 channel 0 and the flow's v channel into
    channels 0, 1 (centre tap); layer 2 (dilation 2) reads one tap right and
    layer 3 (dilation 4) one tap down, the rest copy through the centre.  The
    increment is therefore [h3_0, v] read 2 px right and 4 px down, zero where
    that leaves the image, so the order [h2 | h3 | flow] and the layer-to-
    dilation pairing are both fixed."""
    d = synth.load_desc("tiny_sepref")
    assert d["refine"]["dil"][:3] == [1, 2, 4]
    wts = _zero_weights(d)
    dec1, dec2 = d["dec"][1], d["dec"][2]
    taps = {1: (1, 1), 2: (1, 2), 3: (2, 1)}
    for j, co in enumerate(d["refine"]["ch"], start=1):
        wd, bd = wts[f"ref{j}dw"]
        wd = np.zeros_like(wd)
        p, q = taps.get(j, (1, 1))
        wd[:, p, q] = 1.0
        wp = np.zeros_like(wts[f"ref{j}pw"][0])
        if j == 1:
            wp[0, dec1] = 1.0                 # h3 channel 0
            wp[1, dec1 + dec2 + 1] = 1.0      # flow v
        else:
            wp[0, 0] = wp[1, 1] = 1.0
        wts[f"ref{j}dw"] = (wd, bd)
        wts[f"ref{j}pw"] = (wp, np.zeros(co))
    H, W = 9, 11
    h2 = rand(dec1, H, W)
    h3 = np.abs(rand(dec2, H, W))             # positive: LeakyReLU keeps them
    fl = np.abs(rand(2, H, W))
    out = O.refine(h2, h3, fl, wts, d)
    exp = fl.copy()
    for i in range(H):
        for j in range(W):
            ii, jj = i + 4, j + 2
            if ii < H and jj < W:
                exp[0, i, j] += h3[0, ii, jj]
                exp[1, i, j] += fl[1, ii, jj]
    assert np.allclose(out, exp, rtol=0, atol=1e-15)


def test_drop_finest_recursion_closed_form():
    """Zero weights, head bias b at the estimator levels f..L and refinement
    bias c: flow_f = (2^(L-f+1) - 1) b + c, output 2^f flow_f everywhere."""
    d = synth.load_desc("tiny_sepref")
    wts = _zero_weights(d)
    L, f, R = d["levels"], d["finest"], len(d["refine"]["ch"])
    b, c = np.array([0.5, -0.25]), np.array([0.125, 2.0])
    for l in range(f, L + 1):
        wts[f"dec{l}head"] = (wts[f"dec{l}head"][0], b.copy())
    wts[f"ref{R}pw"] = (wts[f"ref{R}pw"][0], c.copy())
    A = RNG.random((3, 45, 70))
    out = O.flow(A, A, wts, d)
    assert out.shape == (2, 45, 70)
    exp = 2 ** f * ((2 ** (L - f + 1) - 1) * b + c)
    assert np.all(out[0] == exp[0]) and np.all(out[1] == exp[1])


def test_drop_finest_without_refinement():
    """No refinement: flow_2 = (2^(L-1) - 1) b and the output 4 flow_2."""
    d = dict(synth.load_desc("tiny_sepref"), refine=None)
    wts = _zero_weights(d)
    assert not any(k.startswith("ref") for k in wts)
    L = d["levels"]
    b = np.array([-0.5, 0.75])
    for l in range(2, L + 1):
        wts[f"dec{l}head"] = (wts[f"dec{l}head"][0], b.copy())
    A = RNG.random((3, 40, 52))
    out = O.flow(A, A, wts, d)
    assert np.all(out[0] == 4 * (2 ** (L - 1) - 1) * b[0])
    assert np.all(out[1] == 4 * (2 ** (L - 1) - 1) * b[1])
