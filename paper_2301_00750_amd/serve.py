"""Multi-stream serving over the C ABI: continuous batching of frames from
concurrent video streams of different resolutions.

* Every stream keeps its previous frame's feature pyramid and its previous
  output O_{t-1} resident in HBM (two one-image pyramid buffers and two
  output buffers, used alternately).
* Streams are admitted while their resident memory fits the HBM budget;
  later ones wait in a queue and are admitted as earlier streams finish.
* Frames arrive on the host clock.  Each pass of the serving loop takes, for
  every resolution, the streams whose next frame has arrived, builds their
  pyramids, decodes all their flow pairs in one batched call
  (tc_flow_from_pyramid_list) and runs their consistency steps, on a HIP
  stream of that resolution, so different resolutions overlap on the device
  and frames that arrive while others run join the next pass.
* Per-frame latency = arrival time to the completion of its output (HIP
  events against a common origin).
Every kernel computes each image as it would alone, so a stream's outputs
are bitwise the same alone and in the mix.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import tcflow

MAX_BATCH = 16  # pairs per batched decoder call


@dataclass
class StreamJob:
    """One video stream: frames I[t], stylized P[t] (1 x 3 x h x w device
    tensors, possibly repeating), arrival times in seconds, strength alpha."""
    sid: int
    I: list
    P: list
    arrivals: np.ndarray
    alpha: float = 0.5
    keep_outputs: bool = False
    # filled by the server
    outputs: list = field(default_factory=list)
    latencies_ms: list = field(default_factory=list)

    @property
    def hw(self):
        return tuple(self.I[0].shape[2:])

    @property
    def nframes(self):
        return len(self.arrivals)


class _Resident:
    """Per-stream device state."""

    def __init__(self, net, h, w, device):
        pb = net.pyramid_bytes(1, h, w)
        self.pyr = [torch.empty(pb, dtype=torch.uint8, device=device) for _ in range(2)]
        self.out = [torch.empty(1, 3, h, w, device=device) for _ in range(2)]
        self.fw = torch.empty(1, 2, h, w, device=device)
        self.bw = torch.empty(1, 2, h, w, device=device)
        self.t = 0

    @staticmethod
    def bytes_for(net, h, w):
        return 2 * net.pyramid_bytes(1, h, w) + (2 * 3 + 2 * 2) * h * w * 4


class Server:
    def __init__(self, net: tcflow.Net, hbm_budget_bytes: int, device="cuda"):
        self.net = net
        self.budget = int(hbm_budget_bytes)
        self.device = torch.device(device)
        self.groups = {}  # (h, w) -> dict(stream=HIP stream, ws=workspace)

    def _group(self, hw):
        g = self.groups.get(hw)
        if g is None:
            h, w = hw
            wb = self.net.decoder_list_workspace_bytes(MAX_BATCH, h, w)
            g = dict(stream=torch.cuda.Stream(device=self.device),
                     ws=torch.empty(wb, dtype=torch.uint8, device=self.device), events=[])
            self.groups[hw] = g
        return g

    def group_bytes(self, hw):
        return self.net.decoder_list_workspace_bytes(MAX_BATCH, *hw)

    def run(self, jobs, poll_s=2e-4):
        """Serve all jobs to completion; returns a summary dict."""
        queue = sorted(jobs, key=lambda j: j.arrivals[0])
        active = {}          # sid -> (job, resident, next frame index)
        reserved = 0
        for j in jobs:       # workspaces of the resolutions in use are part of the budget
            if j.hw not in self.groups:
                reserved += self.group_bytes(j.hw)
                self._group(j.hw)
        admitted_late = 0
        pending_events = []  # (job, frame index, event)
        torch.cuda.synchronize(self.device)
        origin = torch.cuda.Event(enable_timing=True)
        origin.record()
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        done = 0
        total = sum(j.nframes for j in jobs)
        while done < total:
            now = time.perf_counter() - t0
            # admission by HBM budget, in arrival order
            while queue and queue[0].arrivals[0] <= now:
                j = queue[0]
                need = _Resident.bytes_for(self.net, *j.hw)
                if reserved + need > self.budget and active:
                    break
                queue.pop(0)
                reserved += need
                if j.arrivals[0] < now - 0.05:
                    admitted_late += 1
                active[j.sid] = [j, _Resident(self.net, *j.hw, self.device), 0]
            # one pass: every stream whose next frame has arrived, by resolution
            batches = {}
            for sid, (j, r, k) in active.items():
                if k < j.nframes and j.arrivals[k] <= now:
                    batches.setdefault(j.hw, []).append(sid)
            if not batches:
                nxt = [j.arrivals[k] for j, r, k in active.values() if k < j.nframes]
                if queue:
                    nxt.append(queue[0].arrivals[0])
                wait = (min(nxt) - now) if nxt else poll_s
                time.sleep(max(0.0, min(wait, 2e-3)))
                continue
            for hw, sids in batches.items():
                for i in range(0, len(sids), MAX_BATCH):
                    evs = self._pass(hw, [active[s] for s in sids[i:i + MAX_BATCH]])
                    pending_events += evs
                    done += len(evs)
            for sid in list(active):
                j, r, k = active[sid]
                if k >= j.nframes:  # finished: its memory returns to the budget
                    del active[sid]
                    reserved -= _Resident.bytes_for(self.net, *j.hw)
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        for j, k, ev in pending_events:
            j.latencies_ms.append(origin.elapsed_time(ev) - 1e3 * float(j.arrivals[k]))
        lat = np.concatenate([np.asarray(j.latencies_ms) for j in jobs])
        return dict(frames=int(total), wall_s=wall, frames_per_s=total / wall,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    admitted_late=admitted_late)

    def _pass(self, hw, members):
        """Enqueue one frame for each member (same resolution) on the group's
        HIP stream; returns (job, frame index, completion event) triples."""
        g = self._group(hw)
        h, w = hw
        out = []
        with torch.cuda.stream(g["stream"]):
            pairs = []
            for m in members:
                j, r, k = m
                cur = r.t % 2
                self.net.pyramid(j.I[k % len(j.I)], out=r.pyr[cur])
                if r.t > 0:
                    pairs.append(m)
            if pairs:
                self.net.flow_from_pyramid_list(
                    [m[1].pyr[(m[1].t - 1) % 2] for m in pairs], [m[1].pyr[m[1].t % 2] for m in pairs],
                    h, w, [m[1].fw for m in pairs], [m[1].bw for m in pairs], g["ws"])
            for m in members:
                j, r, k = m
                cur = r.t % 2
                P = j.P[k % len(j.P)]
                if r.t == 0:
                    r.out[cur].copy_(P)
                else:
                    tcflow.consistency_step(P, r.out[cur ^ 1], r.fw, r.bw, j.alpha, out=r.out[cur])
                if j.keep_outputs:
                    j.outputs.append(r.out[cur].clone())
                ev = torch.cuda.Event(enable_timing=True)
                ev.record()
                out.append((j, k, ev))
                r.t += 1
                m[2] += 1
        return out


def poisson_arrivals(n, fps, seed, start=0.0):
    """Arrival times (s) of n frames with exponential gaps of mean 1 / fps."""
    rng = np.random.default_rng(seed)
    return start + np.cumsum(rng.exponential(1.0 / fps, n))
