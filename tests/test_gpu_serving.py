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


def make_jobs(serve, specs, nframes=5):
    jobs = []
    for sid, (h, w, seed) in enumerate(specs):
        sc = synth.LayeredScene(w, h, seed=seed, max_shift=3.0)
        I = [sc.frame(t, device="cuda")[None].contiguous() for t in range(nframes)]
        P = [synth.stylize(x[0], t)[None].contiguous() for t, x in enumerate(I)]
        jobs.append(serve.StreamJob(sid, I, P, serve.poisson_arrivals(nframes, 30.0, 100 + sid),
                                    alpha=0.25 * (sid % 4), keep_outputs=True))
    torch.cuda.synchronize()
    return jobs


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_alone_equals_mix(prec):
    from paper_2301_00750_amd import serve, tcflow
    d = synth.load_desc("tiny")
    net = tcflow.Net(d, synth.he_weights(d),
                     precision=tcflow.TC_FP32 if prec == "fp32" else tcflow.TC_BF16)
    specs = [(64, 96, 1), (96, 128, 2), (64, 96, 3), (96, 128, 4), (48, 80, 5)]
    say(f"[serving] {prec}: {len(specs)} streams, alone then mixed")
    alone = []
    for j in make_jobs(serve, specs):
        serve.Server(net, 1 << 40).run([j])
        alone.append([o.clone() for o in j.outputs])
    mixed = make_jobs(serve, specs)
    summary = serve.Server(net, 1 << 40).run(mixed)
    say(f"   mixed: {summary}")
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


def test_admission_under_tight_budget():
    from paper_2301_00750_amd import serve, tcflow
    d = synth.load_desc("tiny")
    net = tcflow.Net(d, synth.he_weights(d))
    specs = [(64, 96, 1), (64, 96, 2), (64, 96, 3)]
    jobs = make_jobs(serve, specs, nframes=4)
    one = serve._Resident.bytes_for(net, 64, 96)
    srv = serve.Server(net, srv_budget := one + serve.Server(net, 0).group_bytes((64, 96)) + 16)
    summary = srv.run(jobs)
    say(f"[serving] tight budget {srv_budget} B: {summary}")
    assert summary["frames"] == 12
    ref = make_jobs(serve, specs, nframes=4)
    serve.Server(net, 1 << 40).run(ref)
    for a, b in zip(jobs, ref):
        for x, y in zip(a.outputs, b.outputs):
            assert torch.equal(x, y)
