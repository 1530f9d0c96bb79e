"""GPU parity of the network variants (paper Sec. 3.2): the finest flow
estimator dropped (flow of level f upsampled by 2^f to the input) and the
depthwise separable refinement network, through the C ABI against the FP64
oracle on the same seeded inputs.

Bars: FP32 mean EPE <= 0.05 px with max |diff| <= 2e-3 px on the small
workloads (FP32 accumulation over at most 1908 terms per conv output, as for
the base network) and <= 0.05 px at 1920x1080; BF16 / FP8 forms mean EPE
<= 0.25 px.  Sizes span several pixel tiles of the refinement kernel with a
ragged last tile (80 x 112 pads to 80 x 112: level 2 has 20 x 28 = 560
pixels, 4.4 tiles of 128).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import tcflow_oracle as O
from paper_2301_00750_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    from paper_2301_00750_amd import tcflow
    assert torch.cuda.is_available()
    return tcflow


def g(t):
    return t.to(DEV).contiguous()


def f64(t):
    return t.detach().cpu().double().numpy()


def flow_err(a, b):
    d = f64(a) - b
    e = np.sqrt((d ** 2).sum(0))
    return e.mean(), e.max()


def variant(name, **kw):
    return dict(synth.load_desc(name), **kw)


def frames(h, w, seed):
    sc = synth.LayeredScene(w, h, seed=seed, max_shift=3.0)
    return sc.frame(0), sc.frame(1)


def run_pair(tc, d, prec, h, w, seed, label):
    blob = synth.he_weights(d)
    wts = O.unpack_weights(blob, d)
    net = tc.Net(d, blob, precision=prec)
    A, B = frames(h, w, seed)
    say(f"[variant] {label} prec={prec} {h}x{w} finest={d.get('finest', 1)} "
        f"refine={(d.get('refine') or {}).get('ch')}")
    fw, bw = net.flow_estimate_pair(g(A[None]), g(B[None]))
    torch.cuda.synchronize()
    rfw, rbw = O.flow_pair(f64(A), f64(B), wts, d)
    errs = []
    for name, a, b in (("fw", fw[0], rfw), ("bw", bw[0], rbw)):
        mean, mx = flow_err(a, b)
        say(f"   {name}: EPE mean={mean:.3e} max={mx:.3e} |flow| rms={np.sqrt((b ** 2).sum(0).mean()):.2f}")
        errs.append((mean, mx))
    return net, errs


@pytest.mark.parametrize("hw", [(96, 128), (80, 112)])
def test_sepref_fp32_tiny(tc, hw):
    _, errs = run_pair(tc, variant("tiny_sepref"), tc.TC_FP32, *hw, 3, "tiny_sepref")
    for mean, mx in errs:
        assert mean <= 0.05 and mx <= 2e-3


def test_drop_finest_without_refinement_fp32(tc):
    _, errs = run_pair(tc, variant("tiny_sepref", refine=None), tc.TC_FP32, 96, 128, 4, "4light")
    for mean, mx in errs:
        assert mean <= 0.05 and mx <= 2e-3


def test_drop_two_levels_with_refinement_fp32(tc):
    """finest = 3: output upsampled by 8; refinement on level 3."""
    _, errs = run_pair(tc, variant("tiny_sepref", finest=3), tc.TC_FP32, 80, 112, 5, "finest3")
    for mean, mx in errs:
        assert mean <= 0.05 and mx <= 2e-3


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_sepref_low_precision_tiny(tc, prec):
    p = tc.TC_BF16 if prec == "bf16" else tc.TC_FP8_E4M3
    _, errs = run_pair(tc, variant("tiny_sepref"), p, 96, 128, 6, "tiny_sepref")
    for mean, mx in errs:
        # stated bar, and the regression guards of the base network's forms
        assert mean <= 0.25
        assert mean <= 0.05 and mx <= 0.3


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_sepref_batch_invariance_and_determinism(tc, prec):
    d = variant("tiny_sepref")
    net = tc.Net(d, synth.he_weights(d), precision=tc.TC_FP32 if prec == "fp32" else tc.TC_BF16)
    gen = torch.Generator().manual_seed(8)
    A = torch.rand(3, 3, 80, 112, generator=gen)
    B = torch.rand(3, 3, 80, 112, generator=gen)
    say(f"[variant] batch 3 vs 1, {prec}")
    fw, bw = net.flow_estimate_pair(g(A), g(B))
    fw2, bw2 = net.flow_estimate_pair(g(A), g(B))
    s2 = net.flow_estimate_pair(g(A[2:]), g(B[2:]))
    torch.cuda.synchronize()
    assert torch.equal(fw, fw2) and torch.equal(bw, bw2)
    assert torch.equal(s2[0][0], fw[2]) and torch.equal(s2[1][0], bw[2])


def test_sepref_list_decoder_equals_pair(tc):
    """The per-stream (pointer table) decoder gives the batched pair's flows."""
    d = variant("tiny_sepref")
    net = tc.Net(d, synth.he_weights(d))
    A, B = frames(96, 128, 9)
    C, D = frames(96, 128, 10)
    say("[variant] list decoder vs pair")
    pa, pb, pc, pd = (net.pyramid(g(x[None])) for x in (A, B, C, D))
    fws = [torch.empty(1, 2, 96, 128, device=DEV) for _ in range(2)]
    bws = [torch.empty(1, 2, 96, 128, device=DEV) for _ in range(2)]
    ws = torch.empty(net.decoder_list_workspace_bytes(2, 96, 128), dtype=torch.uint8, device=DEV)
    net.flow_from_pyramid_list([pa, pc], [pb, pd], 96, 128, fws, bws, ws)
    r1 = net.flow_estimate_pair(g(A[None]), g(B[None]))
    r2 = net.flow_estimate_pair(g(C[None]), g(D[None]))
    torch.cuda.synchronize()
    assert torch.equal(fws[0], r1[0]) and torch.equal(bws[0], r1[1])
    assert torch.equal(fws[1], r2[0]) and torch.equal(bws[1], r2[1])


_FULLHD = {}


def fullhd_case():
    """Inputs, weights and oracle flows of the 1920x1080 variant, computed once."""
    if not _FULLHD:
        d = synth.load_desc("fullhd_sepref")
        blob = synth.he_weights(d)
        sc = synth.LayeredScene(1920, 1080, seed=0)
        I0, I1 = sc.frame(0), sc.frame(1)
        _FULLHD.update(d=d, blob=blob, I0=I0, I1=I1,
                       ref=O.flow_pair(f64(I0), f64(I1), O.unpack_weights(blob, d), d))
    return _FULLHD


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_sepref_fullhd_vs_oracle(tc, prec):
    c = fullhd_case()
    p = tc.TC_FP32 if prec == "fp32" else tc.TC_BF16
    net = tc.Net(c["d"], c["blob"], precision=p)
    say(f"[variant] fullhd_sepref 1920x1080 pair, {prec}")
    fw, bw = net.flow_estimate_pair(g(c["I0"][None]), g(c["I1"][None]))
    torch.cuda.synchronize()
    rfw, rbw = c["ref"]
    for name, a, b in (("fw", fw[0], rfw), ("bw", bw[0], rbw)):
        mean, mx = flow_err(a, b)
        say(f"   {name}: EPE mean={mean:.3e} max={mx:.3e}")
        if prec == "fp32":
            assert mean <= 0.05 and mx <= 0.05
        else:
            assert mean <= 0.25
            assert mean <= 0.05 and mx <= 0.3  # regression guards (base network's)
