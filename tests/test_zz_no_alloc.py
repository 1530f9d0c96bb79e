"""tc_flow_estimate_pair_noalloc (the flow pair on the library's static
per-device scratch) against tc_flow_estimate_pair with a caller workspace:
the same kernels on the same inputs, so the flows must be bitwise equal.
Two calls in a row, the second with a smaller input (the scratch keeps the
first call's contents), per precision form; an input beyond the scratch is
rejected before anything runs.  Collected last (test_zz_*) and passes
alone in a fresh process as well as after the other GPU tests.""" 
import sys

import pytest
import torch

from paper_2301_00750_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def frames(n, h, w, seed):
    gen = torch.Generator().manual_seed(seed)
    A = torch.rand(n, 3, h, w, generator=gen).cuda()
    B = torch.rand(n, 3, h, w, generator=gen).cuda()
    return A, B


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_noalloc_equals_workspace_call(prec):
    from paper_2301_00750_amd import tcflow as tc
    p = {"fp32": tc.TC_FP32, "bf16": tc.TC_BF16, "fp8": tc.TC_FP8_E4M3}[prec]
    d = synth.load_desc("tiny")
    net = tc.Net(d, synth.he_weights(d), precision=p)
    for (n, h, w, seed) in [(2, 150, 230, 1), (1, 75, 100, 2)]:
        say(f"[noalloc] {prec} n={n} {h}x{w}: workspace "
            f"{net.flow_workspace_bytes(n, h, w)} B of {tc.NOALLOC_SCRATCH_BYTES}")
        A, B = frames(n, h, w, seed)
        ref = net.flow_estimate_pair(A, B)
        fw = torch.full((n, 2, h, w), float("nan"), device="cuda")
        bw = torch.full((n, 2, h, w), float("nan"), device="cuda")
        net.flow_estimate_pair_noalloc(A, B, fw, bw)
        torch.cuda.synchronize()
        assert torch.equal(fw, ref[0]) and torch.equal(bw, ref[1])


def test_noalloc_fullhd_net_and_limit():
    from paper_2301_00750_amd import tcflow as tc
    d = synth.load_desc("fullhd")
    net = tc.Net(d, synth.he_weights(d))
    h, w = 360, 640
    need = net.flow_workspace_bytes(1, h, w)
    say(f"[noalloc] 5-level net {h}x{w}: workspace {need} B of {tc.NOALLOC_SCRATCH_BYTES}")
    assert need <= tc.NOALLOC_SCRATCH_BYTES
    A, B = frames(1, h, w, 3)
    ref = net.flow_estimate_pair(A, B)
    fw = torch.empty(1, 2, h, w, device="cuda")
    bw = torch.empty(1, 2, h, w, device="cuda")
    net.flow_estimate_pair_noalloc(A, B, fw, bw)
    torch.cuda.synchronize()
    assert torch.equal(fw, ref[0]) and torch.equal(bw, ref[1])
    # 1080p needs more than the static scratch: rejected, outputs untouched
    H, W = 1080, 1920
    assert net.flow_workspace_bytes(1, H, W) > tc.NOALLOC_SCRATCH_BYTES
    A, B = frames(1, H, W, 4)
    fw = torch.full((1, 2, H, W), 5.0, device="cuda")
    bw = torch.full((1, 2, H, W), 5.0, device="cuda")
    with pytest.raises(tc.TcError) as e:
        net.flow_estimate_pair_noalloc(A, B, fw, bw)
    assert e.value.status == tc.TC_ERR_SCRATCH
    torch.cuda.synchronize()
    assert torch.all(fw == 5.0) and torch.all(bw == 5.0)
