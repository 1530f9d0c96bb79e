"""What the trained student gains over the method without it.

Without the learned part, the method runs the full (teacher) network.  The
student replaces it at a fraction of the cost, so its gain is speed at a
stated accuracy against the teacher.  Frame pairs are held out: their scene
seeds are outside the range the training pairs use.

* accuracy: the trained student's flows are much closer to the teacher's
  than the same network's untrained (seeded He) weights, or a zero flow, are;
* speed: one student flow pair (BF16) takes well under half the time of one
  teacher flow pair (FP32, the plain path), both at 1920 x 1080.
"""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2301_00750_amd import synth

pytestmark = pytest.mark.gpu

HELD_OUT_SEED = 900000  # training scenes use 100000 + k, k < 400


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    from paper_2301_00750_amd import tcflow
    assert torch.cuda.is_available()
    return tcflow


@pytest.fixture(scope="module")
def trained():
    from paper_2301_00750_amd import student as stu
    if not os.path.exists(stu.DEFAULT_WEIGHTS):
        pytest.fail(f"trained student weights missing: {stu.DEFAULT_WEIGHTS}")
    return np.load(stu.DEFAULT_WEIGHTS, allow_pickle=False)


def mean_epe(a, b):
    return float(torch.sqrt(((a - b) ** 2).sum(1)).mean())


def test_trained_student_beats_untrained_and_zero_flow(tc, trained):
    sd = synth.load_desc("student")
    td = synth.load_desc("fullhd")
    h, w = sd["height"], sd["width"]
    teacher = tc.Net(td, synth.he_weights(td))
    student = tc.Net(sd, trained)
    untrained = tc.Net(sd, synth.he_weights(sd))
    e_s, e_u, e_z = [], [], []
    for k in range(4):
        sc = synth.LayeredScene(w, h, seed=HELD_OUT_SEED + k)
        A = sc.frame(0, device="cuda")[None].contiguous()
        B = sc.frame(1, device="cuda")[None].contiguous()
        say(f"[student gain] held-out pair {k} ({w}x{h})")
        tf, tb = teacher.flow_estimate_pair(A, B)
        sf, sb = student.flow_estimate_pair(A, B)
        uf, ub = untrained.flow_estimate_pair(A, B)
        for x, y in ((sf, tf), (sb, tb)):
            e_s.append(mean_epe(x, y))
        for x, y in ((uf, tf), (ub, tb)):
            e_u.append(mean_epe(x, y))
        for y in (tf, tb):
            e_z.append(mean_epe(torch.zeros_like(y), y))
    s, u, z = np.mean(e_s), np.mean(e_u), np.mean(e_z)
    say(f"   EPE vs teacher: trained {s:.3f} px, untrained {u:.3f} px, zero flow {z:.3f} px")
    assert np.isfinite(s)
    assert s <= 0.25 * u
    assert s <= 0.25 * z


def test_student_pair_faster_than_teacher(tc, trained):
    sd = synth.load_desc("student")
    td = synth.load_desc("fullhd")
    H, W = td["height"], td["width"]
    sc = synth.LayeredScene(W, H, seed=HELD_OUT_SEED + 10)
    A = sc.frame(0, device="cuda")[None].contiguous()
    B = sc.frame(1, device="cuda")[None].contiguous()
    nets = {"teacher fp32": tc.Net(dict(td), synth.he_weights(td)),
            "student bf16": tc.Net(dict(sd, height=H, width=W), trained, precision=tc.TC_BF16)}
    ms = {}
    for name, net in nets.items():
        ws = torch.empty(net.flow_workspace_bytes(1, H, W), dtype=torch.uint8, device="cuda")
        fw = torch.empty(1, 2, H, W, device="cuda")
        bw = torch.empty_like(fw)
        for _ in range(3):
            net.flow_estimate_pair(A, B, ws=ws, out_fw=fw, out_bw=bw)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            net.flow_estimate_pair(A, B, ws=ws, out_fw=fw, out_bw=bw)
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / 10
        say(f"[student gain] {name}: {ms[name]:.3f} ms per flow pair at {W}x{H}")
    assert ms["student bf16"] <= 0.5 * ms["teacher fp32"]
