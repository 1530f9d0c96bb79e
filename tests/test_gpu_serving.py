"""Serving: continuous batching of concurrent streams of different
resolutions gives every stream the same outputs as serving it alone (bitwise:
each kernel computes an image exactly as it would alone), and the same as
the single-stream driver; every served frame matches the FP64 oracle's
sequence (paper Sec. 3.1: O_1 = P_1, then flow pair and consistency step per
frame); admission under a tight HBM budget still serves every frame."""
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


def make_jobs(serve, specs, nframes=6, keep_flows=False):
    jobs = []
    for sid, (h, w, seed) in enumerate(specs):
        sc = synth.LayeredScene(w, h, seed=seed, max_shift=3.0)
        I = [sc.frame(t, device="cuda")[None].contiguous() for t in range(nframes)]
        P = [synth.stylize(x[0], t)[None].contiguous() for t, x in enumerate(I)]
        jobs.append(serve.StreamJob(sid, I, P, serve.poisson_arrivals(nframes, 30.0, 100 + sid),
                                    alpha=0.25 * (sid % 4), keep_outputs=True,
                                    keep_flows=keep_flows))
    torch.cuda.synchronize()
    return jobs


def f64(t):
    return t.detach().cpu().double().numpy()


_ORACLE_FLOWS = {}


def oracle_flows(job, wts, d):
    """FP64 flow pairs (t-1 -> t, t -> t-1) of a job's frames, cached per stream."""
    key = (job.sid, job.hw)
    if key not in _ORACLE_FLOWS:
        _ORACLE_FLOWS[key] = [O.flow_pair(f64(job.I[t][0]), f64(job.I[t + 1][0]), wts, d)
                              for t in range(job.nframes - 1)]
    return _ORACLE_FLOWS[key]


# Bars per form: max EPE of each served flow; output: max |GPU - oracle| and
# RMS over the frame.  FP32: accumulation over at most 1908 terms per conv
# (max EPE 2e-3 px, the single-pair bar), output at the single-stream bar.
# BF16: the stated mean-EPE bar 0.25 px, and regression guards: max EPE
# 0.1 px (8-bit mantissas through 4 levels; measured 0.016), output within
# |grad O| x max EPE of the oracle's (0.02 max, 1e-3 RMS; measured 7.5e-4 and
# 1.8e-5).  band = the largest fraction of pixels whose decision is left to
# the GPU (measured 0 and 0.019).
SERVE_BARS = {"fp32": dict(epe_mean=0.05, epe_max=2e-3, out_max=1e-3, out_rms=1e-4, band=0.02),
              "bf16": dict(epe_mean=0.25, epe_max=0.1, out_max=0.02, out_rms=1e-3, band=0.1)}


@pytest.mark.parametrize("prec,graphs", [("fp32", False), ("fp32", True), ("bf16", True)])
def test_served_frames_vs_oracle(prec, graphs):
    """Every frame of every stream of the mix against the oracle's sequence on
    the same inputs: the served flow pairs by end-point error, the outputs
    per pixel.  The oracle's recursion feeds back its own O_{t-1}; where the
    visibility test is within the flows' error of its threshold, either
    decision is valid and the oracle takes the GPU's (read back by re-running
    the step on the served inputs, which must reproduce the served output
    bitwise)."""
    from paper_2301_00750_amd import serve, tcflow
    d = synth.load_desc("tiny")
    blob = synth.he_weights(d)
    wts = O.unpack_weights(blob, d)
    net = tcflow.Net(d, blob, precision=tcflow.TC_FP32 if prec == "fp32" else tcflow.TC_BF16)
    specs = [(64, 96, 1), (96, 128, 2), (64, 96, 3), (96, 128, 4), (48, 80, 5)]
    bars = SERVE_BARS[prec]
    jobs = make_jobs(serve, specs, keep_flows=True)
    srv = serve.Server(net, 1 << 40, graphs=graphs)
    say(f"[serving vs oracle] {prec} graphs={graphs}: {srv.run(jobs)}")
    srv.close()
    worst = dict(epe_mean=0.0, epe_max=0.0, out_max=0.0, out_rms=0.0, band=0.0)
    for j in jobs:
        assert len(j.outputs) == j.nframes and len(j.flows) == j.nframes - 1
        rflows = oracle_flows(j, wts, d)
        assert torch.equal(j.outputs[0], j.P[0])
        orc = f64(j.P[0][0])
        for t in range(1, j.nframes):
            fw, bw = j.flows[t - 1]
            rfw, rbw = rflows[t - 1]
            epes = []
            for a, b in ((fw, rfw), (bw, rbw)):
                e = np.sqrt(((f64(a[0]) - b) ** 2).sum(0))
                epes.append((e.mean(), e.max()))
            delta = max(m for _, m in epes)
            worst["epe_mean"] = max(worst["epe_mean"], max(m for m, _ in epes))
            worst["epe_max"] = max(worst["epe_max"], delta)
            # the GPU's decisions, and the served step reproduced from its inputs
            re_out, m_gpu = tcflow.consistency_step(j.P[t], j.outputs[t - 1], fw, bw, j.alpha,
                                                    mask=True)
            torch.cuda.synchronize()
            assert torch.equal(re_out, j.outputs[t])
            m_gpu = m_gpu[0].cpu().numpy().astype(bool)
            P = f64(j.P[t][0])
            _, rm, margin, G = O.consistency(P, orc, rfw, rbw, j.alpha)
            # |change of the test's margin| for flows within delta px of the
            # oracle's (first order, with the change of f~ through the
            # gradient of f_fw at the sample point, plus the second order term)
            # (|grad f_fw| of a bilinear sample is at most sqrt 2 times the
            # largest difference of neighbouring pixels)
            fa = O.warp_clamp(rfw, rbw)
            grad = np.sqrt(2.0) * max(np.abs(np.diff(rfw, axis=1)).max(),
                                      np.abs(np.diff(rfw, axis=2)).max())
            dsum = delta * (2.0 + grad)
            band = (2.0 * np.sqrt(((rbw + fa) ** 2).sum(0)) * dsum + dsum ** 2
                    + 0.02 * (np.sqrt((rbw ** 2).sum(0)) + np.sqrt((fa ** 2).sum(0))) * dsum)
            amb = np.abs(margin) <= 1.01 * band + 1e-6
            assert np.array_equal(m_gpu[~amb], rm[~amb]), \
                f"stream {j.sid} frame {t}: {int((m_gpu[~amb] != rm[~amb]).sum())} decided pixels differ"
            m = np.where(amb, m_gpu, rm)
            orc = np.where(m[None], (1 - j.alpha) * P + j.alpha * G, P)
            diff = f64(j.outputs[t][0]) - orc
            worst["out_max"] = max(worst["out_max"], float(np.abs(diff).max()))
            worst["out_rms"] = max(worst["out_rms"], float(np.sqrt((diff ** 2).mean())))
            worst["band"] = max(worst["band"], float(amb.mean()))
    say("   worst over streams and frames: " + ", ".join(f"{k}={v:.3e}" for k, v in worst.items()))
    for k, v in bars.items():
        assert worst[k] <= v, f"{k} = {worst[k]} above {v}"


@pytest.mark.parametrize("prec,graphs", [("fp32", False), ("bf16", False), ("fp32", True),
                                         ("bf16", True)])
def test_alone_equals_mix(prec, graphs):
    """Mixed serving (eager, or every pass after a stream's first frame a
    replayed HIP graph, with eager copies and other streams' work between the
    replays) against each stream served alone, eagerly: every frame's output
    bitwise equal."""
    from paper_2301_00750_amd import serve, tcflow
    d = synth.load_desc("tiny")
    net = tcflow.Net(d, synth.he_weights(d),
                     precision=tcflow.TC_FP32 if prec == "fp32" else tcflow.TC_BF16)
    specs = [(64, 96, 1), (96, 128, 2), (64, 96, 3), (96, 128, 4), (48, 80, 5)]
    say(f"[serving] {prec} graphs={graphs}: {len(specs)} streams, alone then mixed")
    alone = []
    for j in make_jobs(serve, specs):
        serve.Server(net, 1 << 40).run([j])
        alone.append([o.clone() for o in j.outputs])
    mixed = make_jobs(serve, specs)
    srv = serve.Server(net, 1 << 40, graphs=graphs)
    summary = srv.run(mixed)
    say(f"   mixed: {summary}")
    if graphs:
        assert summary["graphs_captured"] > 0
    # a second session on the same server: its slots are reused, and so are the graphs of
    # slot sets that recur
    again = make_jobs(serve, specs)
    srv.run(again)
    for a, j in zip(alone, again):
        for x, y in zip(a, j.outputs):
            assert torch.equal(x, y)
    srv.close()
    for a, j in zip(alone, mixed):
        assert len(a) == len(j.outputs) == j.nframes
        for x, y in zip(a, j.outputs):
            assert torch.equal(x, y)
    # the single-stream driver gives the same outputs
    j = mixed[1]
    st = tcflow.StreamState(net, 1, *j.hw, pipelined=False)
    for t in range(j.nframes):
        o = st.push(j.I[t], j.P[t], j.alpha)
        torch.cuda.synchronize()
        assert torch.equal(o, j.outputs[t])


@pytest.mark.parametrize("graphs", [False, True])
def test_admission_under_tight_budget(graphs):
    """Room for one slot: the three streams are served one after another in
    the same slot, with the same outputs as with room for all."""
    from paper_2301_00750_amd import serve, tcflow
    d = synth.load_desc("tiny")
    net = tcflow.Net(d, synth.he_weights(d))
    specs = [(64, 96, 1), (64, 96, 2), (64, 96, 3)]
    jobs = make_jobs(serve, specs, nframes=4)
    one = serve._Slot.bytes_for(net, 64, 96, graphs)
    srv = serve.Server(net, srv_budget := one + serve.Server(net, 0).group_bytes((64, 96)) + 16,
                       graphs=graphs)
    summary = srv.run(jobs)
    say(f"[serving] tight budget {srv_budget} B: {summary}")
    assert summary["frames"] == 12
    assert len(srv.groups[(64, 96)]["slots"]) == 1
    ref = make_jobs(serve, specs, nframes=4)
    serve.Server(net, 1 << 40).run(ref)
    for a, b in zip(jobs, ref):
        for x, y in zip(a.outputs, b.outputs):
            assert torch.equal(x, y)


def test_tight_budget_across_resolutions():
    """Room for one slot of the larger resolution: switching resolution frees
    the idle slot (and its graphs) of the other one; outputs unchanged."""
    from paper_2301_00750_amd import serve, tcflow
    d = synth.load_desc("tiny")
    net = tcflow.Net(d, synth.he_weights(d))
    specs = [(64, 96, 1), (96, 128, 2), (64, 96, 3), (96, 128, 4)]
    jobs = make_jobs(serve, specs, nframes=4)
    for i, j in enumerate(jobs):  # one after another, alternating resolution
        j.arrivals = j.arrivals + 0.2 * i
    probe = serve.Server(net, 0)
    budget = (probe.group_bytes((64, 96)) + probe.group_bytes((96, 128))
              + serve._Slot.bytes_for(net, 96, 128, True) + 16)
    srv = serve.Server(net, budget, graphs=True)
    summary = srv.run(jobs)
    say(f"[serving] budget {budget} B across resolutions: {summary}")
    assert summary["frames"] == 16
    assert srv.reserved <= budget
    ref = make_jobs(serve, specs, nframes=4)
    serve.Server(net, 1 << 40).run(ref)
    for a, b in zip(jobs, ref):
        for x, y in zip(a.outputs, b.outputs):
            assert torch.equal(x, y)
    srv.close()
