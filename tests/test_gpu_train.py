"""GPU parity of student training (tc_trainer_*) against the FP64 oracle.

* loss and full gradient of one batch vs the oracle's float64 autograd
  gradient (which is itself pinned to finite differences): every layer's
  gradient within 1e-3 of that layer's largest entry, the whole gradient
  within 1e-4 relative L2 (FP32 sums over at most a few thousand pixels per
  weight);
* AdamW steps vs the oracle's AdamW fed with the GPU's gradients;
* a few steps on a fixed batch lower the loss.
Frames 21 x 30 pad to 24 x 32 (3 levels): the padding path is covered.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import student_oracle as S
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


def batch(n, h, w, seed):
    sc = [synth.LayeredScene(w, h, seed=seed + i, max_shift=2.0) for i in range(n)]
    A = torch.stack([s.frame(0) for s in sc])
    B = torch.stack([s.frame(1) for s in sc])
    T = torch.stack([s.gt_flow(0, 1)[0] for s in sc])
    return A, B, T


def layer_slices(d, blob):
    wts = O.unpack_weights(blob, d)
    pos, out = 0, []
    for name, (w, b) in wts.items():
        out.append((name, pos, pos + w.size + b.size))
        pos += w.size + b.size
    return out


def test_gradient_vs_oracle(tc):
    d = synth.load_desc("student")
    blob = synth.he_weights(d)
    A, B, T = batch(2, 21, 30, 5)
    say("[train] gradient 2 x 21x30")
    tr = tc.Trainer(d, blob, 2, 21, 30)
    loss = tr.grad(A.cuda().contiguous(), B.cuda().contiguous(), T.cuda().contiguous())
    g = tr.copy(1).cpu().double().numpy()
    lref, gref = S.loss_and_grad(blob.astype(np.float64), A.double(), B.double(), T.double(), d)
    say(f"   loss gpu={float(loss):.7f} oracle={lref:.7f}")
    assert abs(float(loss) - lref) <= 1e-5 * abs(lref)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"   gradient relative L2 error {rel:.2e}")
    worst = []
    for name, a, b in layer_slices(d, blob):
        err = np.abs(g[a:b] - gref[a:b]).max() / max(np.abs(gref[a:b]).max(), 1e-12)
        worst.append((err, name))
    worst.sort(reverse=True)
    say(f"   worst layers: {worst[:4]}")
    assert rel <= 1e-4
    assert worst[0][0] <= 1e-3


def test_gradient_vs_oracle_wide_flows(tc):
    """Head gain 50 makes the level-1 flows large and spatially varying: the
    warp backward then meets both its paths (16 x 16 tiles whose taps fit a
    40 x 40 window, added in LDS first, and wider tiles scattered straight to
    the gradient); the oracle's own level-1 flow shows that both occur."""
    d = dict(synth.load_desc("student"), head_gain=50.0)
    blob = synth.he_weights(d)
    A, B, T = batch(2, 96, 128, 11)
    wts = {k: (torch.from_numpy(w).double(), torch.from_numpy(b).double())
           for k, (w, b) in O.unpack_weights(blob, d).items()}
    U = (2.0 * S.up2(S.student_flows(A.double(), B.double(), wts, d)[1])).numpy()
    n, _, h, w = U.shape
    wide = fit = 0
    for i in range(n):
        for ty in range(0, h, 16):
            for tx in range(0, w, 16):
                ys, xs = np.mgrid[ty:min(ty + 16, h), tx:min(tx + 16, w)]
                x0 = np.floor(xs + U[i, 0, ty:ty + 16, tx:tx + 16]).astype(int)
                y0 = np.floor(ys + U[i, 1, ty:ty + 16, tx:tx + 16]).astype(int)
                ww = min(x0.max() + 1, w - 1) - max(x0.min(), 0) + 1
                wh = min(y0.max() + 1, h - 1) - max(y0.min(), 0) + 1
                if ww > 0 and wh > 0 and ww * wh <= 1600:
                    fit += 1
                else:
                    wide += 1
    say(f"[train] gradient 2 x 96x128, head gain 50: level-1 |U| <= {np.abs(U).max():.1f}, "
        f"tiles fitting the window {fit}, wider {wide}")
    assert fit > 0 and wide > 0
    tr = tc.Trainer(d, blob, 2, 96, 128)
    loss = tr.grad(A.cuda().contiguous(), B.cuda().contiguous(), T.cuda().contiguous())
    g = tr.copy(1).cpu().double().numpy()
    lref, gref = S.loss_and_grad(blob.astype(np.float64), A.double(), B.double(), T.double(), d)
    say(f"   loss gpu={float(loss):.7f} oracle={lref:.7f}")
    assert abs(float(loss) - lref) <= 1e-5 * abs(lref)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    worst = max(np.abs(g[a:b] - gref[a:b]).max() / max(np.abs(gref[a:b]).max(), 1e-12)
                for _, a, b in layer_slices(d, blob))
    say(f"   gradient relative L2 error {rel:.2e}, worst layer {worst:.2e}")
    assert rel <= 1e-4
    assert worst <= 1e-3


@pytest.mark.parametrize("hw", [(512, 1024), (520, 1000)])
def test_gradient_vs_oracle_winograd_level(hw):
    """At 512 x 1024 level 1 (256 x 512) has 256 regions of 16 x 32 pixels, so
    the trainer runs its c1 and c2 forward and its c1, c2 and c3 data
    gradients there through the F(4x4) Winograd conv (weights transformed on
    the device from the current blob every call); level 2 stays direct.
    520 x 1000: level 1 is 260 x 500, ragged against the 16 x 32 regions."""
    from paper_2301_00750_amd import tcflow as tc
    h, w = hw
    d = synth.load_desc("student")
    blob = synth.he_weights(d)
    A, B, T = batch(1, h, w, 21)
    say(f"[train] gradient 1 x {h}x{w} (Winograd on level 1)")
    tr = tc.Trainer(d, blob, 1, h, w)
    loss = tr.grad(A.cuda().contiguous(), B.cuda().contiguous(), T.cuda().contiguous())
    g = tr.copy(1).cpu().double().numpy()
    lref, gref = S.loss_and_grad(blob.astype(np.float64), A.double(), B.double(), T.double(), d)
    say(f"   loss gpu={float(loss):.7f} oracle={lref:.7f}")
    assert abs(float(loss) - lref) <= 1e-5 * abs(lref)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    worst = max(np.abs(g[a:b] - gref[a:b]).max() / max(np.abs(gref[a:b]).max(), 1e-12)
                for _, a, b in layer_slices(d, blob))
    say(f"   gradient relative L2 error {rel:.2e}, worst layer {worst:.2e}")
    assert rel <= 1e-4
    assert worst <= 1e-3


def test_gradient_vs_oracle_wide_decoder(tc):
    """A decoder of 96/64/32 channels: the weight gradient splits c1's and
    c2's output channels over two groups of 48 (the second group of c2 holds
    one block of 16), which the student's 48/32/16 never does."""
    d = dict(synth.load_desc("student"), ch=[16, 24, 32], dec=[96, 64, 32])
    blob = synth.he_weights(d)
    A, B, T = batch(2, 40, 56, 13)
    say("[train] gradient 2 x 40x56, decoder 96/64/32")
    tr = tc.Trainer(d, blob, 2, 40, 56)
    loss = tr.grad(A.cuda().contiguous(), B.cuda().contiguous(), T.cuda().contiguous())
    g = tr.copy(1).cpu().double().numpy()
    lref, gref = S.loss_and_grad(blob.astype(np.float64), A.double(), B.double(), T.double(), d)
    say(f"   loss gpu={float(loss):.7f} oracle={lref:.7f}")
    assert abs(float(loss) - lref) <= 1e-5 * abs(lref)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    worst = max(np.abs(g[a:b] - gref[a:b]).max() / max(np.abs(gref[a:b]).max(), 1e-12)
                for _, a, b in layer_slices(d, blob))
    say(f"   gradient relative L2 error {rel:.2e}, worst layer {worst:.2e}")
    assert rel <= 1e-4
    assert worst <= 1e-3


def test_adamw_steps_vs_oracle(tc):
    d = synth.load_desc("student")
    blob = synth.he_weights(d)
    A, B, T = (x.cuda().contiguous() for x in batch(2, 24, 32, 9))
    prm = dict(S.TRAIN_DEFAULTS, lr=1e-3)
    tr = tc.Trainer(d, blob, 2, 24, 32, params=tc.train_params(lr=1e-3))
    p, m, v = blob.astype(np.float64), np.zeros(blob.size), np.zeros(blob.size)
    say("[train] three AdamW steps")
    for t in range(1, 4):
        tr.grad(A, B, T)
        g = tr.copy(1).cpu().double().numpy()
        tr.step(A, B, T)        # recomputes the same gradient, then updates
        p, m, v = S.adamw_step(p, g, m, v, t, prm)
        got = tr.copy(0).cpu().double().numpy()
        err = np.abs(got - p).max()
        say(f"   step {t}: max |w_gpu - w_oracle| = {err:.2e}")
        assert err <= 2e-6
    assert tr.steps_done == 3


def test_training_lowers_loss(tc):
    d = synth.load_desc("student")
    A, B, T = (x.cuda().contiguous() for x in batch(4, 64, 96, 13))
    tr = tc.Trainer(d, synth.he_weights(d), 4, 64, 96, params=tc.train_params(lr=2e-3))
    say("[train] 40 steps on one batch")
    first = float(tr.grad(A, B, T))
    for _ in range(40):
        tr.step(A, B, T)
    last = float(tr.grad(A, B, T))
    say(f"   loss {first:.4f} -> {last:.4f}")
    assert np.isfinite(last) and last < 0.9 * first


def test_flow_agreement_counts(tc):
    """Counts equal the consistency step's mask and the oracle's mask away
    from its undecided band."""
    gen = torch.Generator().manual_seed(3)
    h, w = 67, 91
    ffw = 3 * torch.randn(2, 2, h, w, generator=gen)
    fbw = -ffw + 0.5 * torch.randn(2, 2, h, w, generator=gen)
    g = [x.cuda().contiguous() for x in (ffw, fbw)]
    say("[agreement] 2 x 67x91")
    counts = tc.flow_agreement(*g).cpu().numpy()
    P = torch.rand(2, 3, h, w, generator=gen).cuda()
    _, m = tc.consistency_step(P, P.clone(), g[0], g[1], 0.5, mask=True)
    assert np.array_equal(counts, m.reshape(2, -1).sum(1).cpu().numpy())
    for i in range(2):
        _, rm, margin, _ = O.consistency(np.zeros((3, h, w)), np.zeros((3, h, w)),
                                         ffw[i].double().numpy(), fbw[i].double().numpy(), 0.5)
        amb = int((np.abs(margin) <= 1e-4).sum())
        assert abs(int(counts[i]) - int(rm.sum())) <= amb


def test_fallback_switches_to_teacher(tc):
    from paper_2301_00750_amd import student
    sd, td = synth.load_desc("student"), synth.load_desc("tiny")
    s_net, t_net = tc.Net(sd, synth.he_weights(sd)), tc.Net(td, synth.he_weights(td))
    A, B, _ = batch(1, 64, 96, 4)
    A, B = A.cuda().contiguous(), B.cuda().contiguous()
    say("[fallback] thresholds 0 and 1.01")
    never = student.FallbackFlow(s_net, t_net, 64, 96, threshold=0.0)
    fw, bw, agree = never(A, B)
    sfw, sbw = s_net.flow_estimate_pair(A, B)
    assert torch.equal(fw, sfw) and never.fallbacks == 0 and 0.0 <= agree <= 1.0
    always = student.FallbackFlow(s_net, t_net, 64, 96, threshold=1.01)
    fw, bw, _ = always(A, B)
    tfw, tbw = t_net.flow_estimate_pair(A, B)
    assert torch.equal(fw, tfw) and torch.equal(bw, tbw) and always.fallbacks == 1


def test_fallback_threshold_boundary(tc):
    """The rule falls back exactly when the agreement is below the threshold:
    thresholds half a pixel's share above and below the measured agreement
    of a pair flip the decision (agreement = agreeing pixels / h w)."""
    from paper_2301_00750_amd import student
    sd, td = synth.load_desc("student"), synth.load_desc("tiny")
    s_net, t_net = tc.Net(sd, synth.he_weights(sd)), tc.Net(td, synth.he_weights(td))
    h, w = 64, 96
    A, B, _ = batch(1, h, w, 7)
    A, B = A.cuda().contiguous(), B.cuda().contiguous()
    _, _, agree = student.FallbackFlow(s_net, t_net, h, w, threshold=0.0)(A, B)
    say(f"[fallback] agreement {agree:.6f} ({round(agree * h * w)} of {h * w} pixels)")
    half = 0.5 / (h * w)
    above = student.FallbackFlow(s_net, t_net, h, w, threshold=agree + half)
    fw, _, _ = above(A, B)
    assert above.fallbacks == 1 and torch.equal(fw, t_net.flow_estimate_pair(A, B)[0])
    if agree > 0.0:
        below = student.FallbackFlow(s_net, t_net, h, w, threshold=agree - half)
        fw, _, _ = below(A, B)
        assert below.fallbacks == 0 and torch.equal(fw, s_net.flow_estimate_pair(A, B)[0])

