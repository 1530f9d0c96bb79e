"""The streaming step replayed as a HIP graph (GraphStreamState) gives
bitwise the outputs of the eager driver, frame after frame, for every
precision form: graphs are replayed many times, with the strength alpha
changing (one graph per buffer parity and alpha), with eager copies and
other eager work on the device between replays."""
import sys

import pytest
import torch

from paper_2301_00750_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_graph_stream_equals_eager(prec):
    from paper_2301_00750_amd import tcflow as tc
    p = {"fp32": tc.TC_FP32, "bf16": tc.TC_BF16, "fp8": tc.TC_FP8_E4M3}[prec]
    d = synth.load_desc("tiny")
    net = tc.Net(d, synth.he_weights(d), precision=p)
    h, w = 96, 128
    sc = synth.LayeredScene(w, h, seed=4, max_shift=3.0)
    I = [sc.frame(t, device="cuda")[None].contiguous() for t in range(5)]
    P = [synth.stylize(x[0], t)[None].contiguous() for t, x in enumerate(I)]
    alphas = [0.5, 0.25, 0.5, 1.0, 0.25, 0.5, 0.0, 0.5, 1.0, 0.5, 0.25, 0.5, 0.75, 0.5]
    say(f"[graph] {prec}: {len(alphas)} frames, graphs vs eager")
    eager = tc.StreamState(net, 1, h, w, pipelined=False)
    graph = tc.GraphStreamState(net, 1, h, w)
    scratch = torch.zeros(1 << 20, device="cuda")
    for t, a in enumerate(alphas):
        f = t % len(I)
        e = eager.push(I[f], P[f], a).clone()
        scratch.add_(1.0)  # other eager work between replays
        g = graph.push(I[f], P[f], a).clone()
        torch.cuda.synchronize()
        assert torch.equal(e, g), f"frame {t} differs"
    assert len(graph.graphs) >= 4
    say(f"   {len(graph.graphs)} graphs captured")
