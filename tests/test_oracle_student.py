"""Pins of the student-training oracle (paper Sec. 3.2 "Training" and the
supplementary loss, Eq. S2) against things other than itself: the numpy
oracle's network, central finite differences, closed forms, and torch's
AdamW.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import student_oracle as S
from oracle import tcflow_oracle as O
from paper_2301_00750_amd import synth

RNG = np.random.default_rng(7)


def tiny_student():
    d = synth.load_desc("student")
    return d, synth.he_weights(d).astype(np.float64)


def frames(n, h, w, seed):
    sc = [synth.LayeredScene(w, h, seed=seed + i, max_shift=2.0) for i in range(n)]
    A = torch.stack([s.frame(0) for s in sc]).double()
    B = torch.stack([s.frame(1) for s in sc]).double()
    return A, B


def test_forward_equals_numpy_oracle():
    d, blob = tiny_student()
    A, B = frames(2, 37, 45, 3)          # pads to 40 x 48
    flows = S.student_flows(A, B, S._params(blob, d), d)
    full = 2.0 * S.up2(flows[0])[:, :, :37, :45]
    wts = O.unpack_weights(blob, d)
    for i in range(2):
        ref = O.flow(A[i].numpy(), B[i].numpy(), wts, d)
        assert np.allclose(full[i].detach().numpy(), ref, rtol=0, atol=1e-12)


def test_level_targets_closed_forms():
    T = torch.ones(1, 2, 16, 24, dtype=torch.float64) * torch.tensor([3.0, -2.0]).reshape(1, 2, 1, 1)
    for l, t in enumerate(S.level_targets(T, 3), start=1):
        assert torch.allclose(t, T[:, :, :16 >> l, :24 >> l] / 2 ** l)
    xs = torch.arange(24, dtype=torch.float64)
    R = xs.reshape(1, 1, 1, 24).expand(1, 2, 16, 24).clone()
    for l, t in enumerate(S.level_targets(R, 3), start=1):
        s = 2 ** l
        i = torch.arange(24 // s, dtype=torch.float64)
        assert torch.allclose(t[0, 0, 0], (i * s + (s - 1) / 2) / s)
    # edge padding of a non-multiple size replicates the last row
    Tn = torch.arange(2 * 13 * 8, dtype=torch.float64).reshape(1, 2, 13, 8)
    t1 = S.level_targets(Tn, 3)[0]          # padded to 16 x 8
    last = torch.cat([Tn[:, :, 12:13]] * 2, 2)
    assert torch.allclose(t1[:, :, 7], last.mean(2).reshape(1, 2, 4, 2).mean(3) / 2)


def _const_net(d, b):
    blob = synth.he_weights(d).astype(np.float64) * 0
    wts = O.unpack_weights(blob, d)
    pos, out = 0, blob.copy()
    for name, (w, bb) in wts.items():
        pos += w.size
        if name.endswith("head"):
            out[pos:pos + 2] = b
        pos += bb.size
    return out


def test_constant_network_loss_and_gradient_closed_form():
    """Zero weights and head bias b: flow_l = (2^(L-l+1) - 1) b everywhere;
    a constant teacher c gives targets c / 2^l, so the loss is
    sum_l (|e_l,u| + |e_l,v| + eps)^q, and the gradient with respect to the
    head bias of level m is sum_{l <= m} 2^(m-l) q r_l^(q-1) sign(e_l)."""
    d, _ = tiny_student()
    L = d["levels"]
    b = np.array([0.3, -0.2])
    c = np.array([1.7, 0.9])
    blob = _const_net(d, b)
    A, B = frames(2, 16, 24, 11)
    T = torch.tensor(c).reshape(1, 2, 1, 1).expand(2, 2, 16, 24).clone()
    loss, g = S.loss_and_grad(blob, A, B, T, d)
    eps, q = S.TRAIN_DEFAULTS["loss_eps"], S.TRAIN_DEFAULTS["loss_q"]
    e = {l: (2 ** (L - l + 1) - 1) * b - c / 2 ** l for l in range(1, L + 1)}
    r = {l: np.abs(e[l]).sum() + eps for l in e}
    assert np.isclose(loss, sum(r[l] ** q for l in e), rtol=1e-13)
    wts = O.unpack_weights(blob, d)
    pos = 0
    for name, (w, bb) in wts.items():
        pos += w.size
        if name.endswith("head"):
            m = int(name[3])
            exp = sum(2 ** (m - l) * q * r[l] ** (q - 1) * np.sign(e[l]) for l in range(1, m + 1))
            assert np.allclose(g[pos:pos + 2], exp, rtol=1e-12, atol=1e-14)
        pos += bb.size


def test_gradient_equals_finite_differences():
    d, blob = tiny_student()
    blob = blob * 1.0
    A, B = frames(2, 24, 32, 21)
    T = torch.randn(2, 2, 24, 32, dtype=torch.float64, generator=torch.Generator().manual_seed(2))
    _, g = S.loss_and_grad(blob, A, B, T, d)
    wts = O.unpack_weights(blob, d)
    # a few weights and biases from every layer
    idx, pos = [], 0
    for name, (w, bb) in wts.items():
        for k in RNG.choice(w.size, 2, replace=False):
            idx.append(pos + int(k))
        pos += w.size
        idx.append(pos + int(RNG.integers(bb.size)))
        pos += bb.size
    h = 1e-5
    bad = []
    for i in idx:
        p, m = blob.copy(), blob.copy()
        p[i] += h
        m[i] -= h
        fd = (S.loss_only(p, A, B, T, d) - S.loss_only(m, A, B, T, d)) / (2 * h)
        if abs(fd - g[i]) > 1e-7 + 1e-4 * abs(fd):
            bad.append((i, fd, g[i]))
    assert not bad, bad


def test_adamw_equals_torch():
    p0 = RNG.standard_normal(50)
    prm = dict(S.TRAIN_DEFAULTS, lr=1e-2)
    tp = torch.nn.Parameter(torch.tensor(p0))
    opt = torch.optim.AdamW([tp], lr=prm["lr"], betas=(prm["beta1"], prm["beta2"]),
                            eps=prm["eps"], weight_decay=prm["weight_decay"])
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 4):
        g = RNG.standard_normal(50)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = S.adamw_step(p, g, m, v, t, prm)
        assert np.allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)
