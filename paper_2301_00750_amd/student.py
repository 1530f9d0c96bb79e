"""Distilled student flow network: data, training and inference with fallback.

Teacher: the full network (5 levels, 16..128 channels) with the seeded He
weights.  Student: the same PWC-shaped light network at half width with 3
levels (configs/student.json), trained with the library's trainer
(tc_trainer_*: hand-written backward kernels, AdamW) to reproduce the
teacher's flows on seeded layered-texture frame pairs (Sec. 3.2 "Training":
multi-scale loss, equal weights; supplementary Eq. S2).

At inference the student's forward and backward flows are checked for
agreement (tc_flow_agreement, the consistency step's forward-backward test);
when fewer than ``threshold`` of the pixels agree the frame falls back to the
teacher's flows.

    python -m paper_2301_00750_amd.student --steps 20000 --out weights/student.npy

Every computation runs in libtcflow's kernels; torch holds device memory.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from paper_2301_00750_amd import synth, tcflow

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "student.npy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_pairs(n_pairs, h, w, seed0=100000, pairs_per_scene=5, device="cuda"):
    """n_pairs consecutive-frame pairs (A_i, B_i) from seeded layered scenes,
    pairs_per_scene per scene; returns two (n, 3, h, w) float32 tensors."""
    A = torch.empty(n_pairs, 3, h, w, device=device)
    B = torch.empty(n_pairs, 3, h, w, device=device)
    i, k = 0, 0
    while i < n_pairs:
        sc = synth.LayeredScene(w, h, seed=seed0 + k)
        prev = sc.frame(0, device=device)
        for t in range(1, pairs_per_scene + 1):
            if i >= n_pairs:
                break
            cur = sc.frame(t, device=device)
            A[i] = prev
            B[i] = cur
            prev = cur
            i += 1
        k += 1
    return A, B


def teacher_flows(teacher, A, B, batch=8):
    """Teacher flows A->B and B->A for every pair (FP32 net)."""
    n, _, h, w = A.shape
    fw = torch.empty(n, 2, h, w, device=A.device)
    bw = torch.empty(n, 2, h, w, device=A.device)
    for i in range(0, n, batch):
        j = min(n, i + batch)
        f, b = teacher.flow_estimate_pair(A[i:j], B[i:j])
        fw[i:j] = f
        bw[i:j] = b
    return fw, bw


def train(student_desc, A, B, Tfw, Tbw, steps, batch, seed=0, params=None, weights=None,
          log_every=500):
    """AdamW on random batches drawn from the 2n directed samples (each pair
    in both directions).  Returns (weights, history, seconds)."""
    n, _, h, w = A.shape
    blob = synth.he_weights(student_desc) if weights is None else weights
    tr = tcflow.Trainer(student_desc, blob, batch, h, w, params=params)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        idx = torch.randint(0, 2 * n, (batch,), generator=g)
        fwd = idx < n
        pi = torch.where(fwd, idx, idx - n).cuda()
        fwd = fwd.cuda()
        src = torch.where(fwd[:, None, None, None], A[pi], B[pi]).contiguous()
        dst = torch.where(fwd[:, None, None, None], B[pi], A[pi]).contiguous()
        tgt = torch.where(fwd[:, None, None, None], Tfw[pi], Tbw[pi]).contiguous()
        loss = tr.step(src, dst, tgt)
        if (s + 1) % log_every == 0 or s == 0:
            lv = float(loss)
            hist.append((s + 1, lv))
            log(f"student step {s + 1}/{steps}: loss {lv:.4f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    out = tr.copy(0).cpu().numpy()
    tr.close()
    return out, hist, secs


class FallbackFlow:
    """Student flows with the teacher as fallback for one resolution."""

    def __init__(self, student: tcflow.Net, teacher: tcflow.Net, h, w, threshold=0.9):
        self.student, self.teacher = student, teacher
        self.h, self.w, self.threshold = h, w, threshold
        self.counts = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.fallbacks = 0
        self.frames = 0

    def __call__(self, prev, cur):
        if prev.shape[0] != 1:
            raise ValueError("FallbackFlow decides per pair: one pair (n = 1) per call")
        fw, bw = self.student.flow_estimate_pair(prev, cur)
        tcflow.flow_agreement(fw, bw, counts=self.counts)
        agree = int(self.counts.item()) / float(self.h * self.w)   # host sync: the decision
        self.frames += 1
        if agree < self.threshold:
            self.fallbacks += 1
            fw, bw = self.teacher.flow_estimate_pair(prev, cur)
        return fw, bw, agree


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--pairs", type=int, default=None)
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--init", default=None,
                    help="start from these weights (a fine-tuning stage) instead of He init")
    ap.add_argument("--lr", type=float, default=None, help="learning rate (default: the config's)")
    args = ap.parse_args()
    sd = synth.load_desc("student")
    td = synth.load_desc("fullhd")
    tp = sd["train"]
    steps = args.steps if args.steps is not None else tp["steps"]
    pairs = args.pairs if args.pairs is not None else tp["pairs"]
    batch = args.batch if args.batch is not None else tp["batch"]
    h, w = sd["height"], sd["width"]
    log(f"generating {pairs} pairs {w}x{h}")
    t0 = time.perf_counter()
    A, B = make_pairs(pairs, h, w)
    teacher = tcflow.Net(td, synth.he_weights(td))
    Tfw, Tbw = teacher_flows(teacher, A, B)
    torch.cuda.synchronize()
    log(f"data + teacher flows: {time.perf_counter() - t0:.1f} s")
    lr = args.lr if args.lr is not None else tp["lr"]
    prm = tcflow.train_params(lr=lr, beta1=tp["beta1"], beta2=tp["beta2"], eps=tp["eps"],
                              weight_decay=tp["weight_decay"], loss_eps=tp["loss_eps"],
                              loss_q=tp["loss_q"])
    init = np.load(args.init, allow_pickle=False) if args.init else None
    prior = []
    if args.init:
        prior_meta = os.path.splitext(args.init)[0] + ".json"
        if os.path.exists(prior_meta):
            prior = json.load(open(prior_meta)).get("stages", [])
    wts, hist, secs = train(sd, A, B, Tfw, Tbw, steps, batch, params=prm, weights=init)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, wts.astype(np.float32), allow_pickle=False)
    stage = dict(steps=steps, lr=lr, pairs=pairs, init="he" if init is None else "previous stage",
                 train_seconds=secs, step_ms=1e3 * secs / max(1, steps), loss_history=hist)
    meta = dict(steps=sum(st["steps"] for st in prior) + steps, pairs=pairs, batch=batch,
                resolution=[w, h], train_seconds=secs, step_ms=1e3 * secs / max(1, steps),
                loss_history=hist, params=tp, stages=prior + [stage])
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"saved {args.out}: {steps} steps in {secs:.1f} s ({meta['step_ms']:.2f} ms/step)")


if __name__ == "__main__":
    main()
