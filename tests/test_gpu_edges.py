"""Edge cases through the C ABI against the FP64 oracle: degenerate image
sizes (1 x 1, 1 x n, sizes below one tile, odd sizes that pad by almost a
whole 2^L block), batches of many tiny images, and the distilled student at
the 3840 x 2160 size it is measured on (BF16 and FP32 against the numpy
oracle of the same network)."""
import sys

import numpy as np
import pytest
import torch

from oracle import tcflow_oracle as O
from paper_2301_00750_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    from paper_2301_00750_amd import tcflow
    assert torch.cuda.is_available()
    return tcflow


def f64(t):
    return t.detach().cpu().double().numpy()


def epe(a, b):
    e = np.sqrt(((f64(a) - b) ** 2).sum(0))
    return e.mean(), e.max()


@pytest.mark.parametrize("hw", [(1, 1), (1, 37), (29, 1), (5, 7), (17, 33)])
def test_degenerate_sizes_vs_oracle(tc, hw):
    d = synth.load_desc("tiny")
    blob = synth.he_weights(d)
    wts = O.unpack_weights(blob, d)
    net = tc.Net(d, blob)
    gen = torch.Generator().manual_seed(hw[0] * 100 + hw[1])
    A = torch.rand(1, 3, *hw, generator=gen)
    B = torch.rand(1, 3, *hw, generator=gen)
    say(f"[edge] flow pair {hw}")
    fw, bw = net.flow_estimate_pair(A.cuda(), B.cuda())
    torch.cuda.synchronize()
    assert fw.shape == (1, 2) + hw
    rfw, rbw = O.flow_pair(f64(A[0]), f64(B[0]), wts, d)
    for a, b in ((fw[0], rfw), (bw[0], rbw)):
        mean, mx = epe(a, b)
        assert mx <= 2e-3, (hw, mean, mx)
    # the consistency step on these sizes
    P = torch.rand(1, 3, *hw, generator=gen).cuda()
    Op = torch.rand(1, 3, *hw, generator=gen).cuda()
    out, m = tc.consistency_step(P, Op, fw, bw, 0.5, mask=True)
    ro, rm, margin, _ = O.consistency(f64(P[0]), f64(Op[0]), f64(fw[0]), f64(bw[0]), 0.5)
    sure = np.abs(margin) > 1e-4
    assert np.array_equal(m[0].cpu().numpy().astype(bool)[sure], rm[sure])


def test_many_tiny_images_batch(tc):
    """64 images of 8 x 12 in one call equal the images one by one."""
    d = synth.load_desc("tiny")
    net = tc.Net(d, synth.he_weights(d))
    gen = torch.Generator().manual_seed(5)
    A = torch.rand(64, 3, 8, 12, generator=gen).cuda()
    B = torch.rand(64, 3, 8, 12, generator=gen).cuda()
    say("[edge] batch of 64 tiny images")
    fw, bw = net.flow_estimate_pair(A, B)
    for i in (0, 31, 63):
        f1, b1 = net.flow_estimate_pair(A[i:i + 1].contiguous(), B[i:i + 1].contiguous())
        assert torch.equal(f1[0], fw[i]) and torch.equal(b1[0], bw[i])


_4K = {}


def student_4k_case():
    """Weights, frames and the oracle's flows of the 4K student case (once)."""
    if not _4K:
        from paper_2301_00750_amd import student as stu
        d = synth.load_desc("student")
        w = np.load(stu.DEFAULT_WEIGHTS, allow_pickle=False)
        sc = synth.LayeredScene(3840, 2160, seed=7)
        I0, I1 = sc.frame(0), sc.frame(1)
        say("   oracle: student flow pair at 3840x2160 (about a minute on the host)")
        _4K.update(d=d, w=w, I0=I0, I1=I1,
                   ref=O.flow_pair(f64(I0), f64(I1), O.unpack_weights(w, d), d))
    return _4K


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("level", [0.0, 0.5])
def test_precision_forms_flat_frames(tc, prec, level):
    """Flat frames through the precision forms: all-zero inputs give a zero
    per-image maximum (the FP8 input scale falls back to 1), a constant
    frame a single value everywhere; the flows stay finite and within the
    forms' bar of the oracle's."""
    p = {"bf16": tc.TC_BF16, "fp8": tc.TC_FP8_E4M3}[prec]
    d = synth.load_desc("tiny")
    blob = synth.he_weights(d)
    wts = O.unpack_weights(blob, d)
    net = tc.Net(d, blob, precision=p)
    h, w = 64, 96
    A = torch.full((1, 3, h, w), level)
    say(f"[edge] {prec} flat frames at {level}")
    fw, bw = net.flow_estimate_pair(A.cuda(), A.cuda())
    torch.cuda.synchronize()
    assert torch.isfinite(fw).all() and torch.isfinite(bw).all()
    rfw, rbw = O.flow_pair(f64(A[0]), f64(A[0]), wts, d)
    for a, b in ((fw[0], rfw), (bw[0], rbw)):
        mean, mx = epe(a, b)
        say(f"   EPE mean {mean:.3e} max {mx:.3e}")
        assert mean <= 0.25 and mx <= 1.0, (prec, level, mean, mx)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_student_4k_vs_oracle(tc, prec):
    """The trained student at 3840 x 2160 against the numpy oracle of the same
    weights (FP32 bar 0.05 px mean, BF16 0.25 px)."""
    say(f"[edge] student 3840x2160 {prec}")
    c = student_4k_case()
    p = tc.TC_FP32 if prec == "fp32" else tc.TC_BF16
    net = tc.Net(c["d"], c["w"], precision=p)
    fw, bw = net.flow_estimate_pair(c["I0"][None].cuda(), c["I1"][None].cuda())
    torch.cuda.synchronize()
    rfw, rbw = c["ref"]
    for a, b in ((fw[0], rfw), (bw[0], rbw)):
        mean, mx = epe(a, b)
        say(f"   EPE mean={mean:.3e} max={mx:.3e}")
        assert mean <= (0.05 if prec == "fp32" else 0.25)
