"""Serving: continuous batching of concurrent streams of different
resolutions gives every stream the same outputs as serving it alone (bitwise:
each kernel computes an image exactly as it would alone), and the same as
the single-stream driver; admission under a tight HBM budget still serves
every frame."""
import sys

import numpy as np
import pytest
import torch

from paper_2301_00750_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_jobs(serve, specs, nframes=6):
    jobs = []
    for sid, (h, w, seed) in enumerate(specs):
        sc = synth.LayeredScene(w, h, seed=seed, max_shift=3.0)
        I = [sc.frame(t, device="cuda")[None].contiguous() for t in range(nframes)]
        P = [synth.stylize(x[0], t)[None].contiguous() for t, x in enumerate(I)]
        jobs.append(serve.StreamJob(sid, I, P, serve.poisson_arrivals(nframes, 30.0, 100 + sid),
                                    alpha=0.25 * (sid % 4), keep_outputs=True))
    torch.cuda.synchronize()
    return jobs


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
