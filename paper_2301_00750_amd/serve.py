"""Multi-stream serving over the C ABI: continuous batching of frames from
concurrent video streams of different resolutions.

* Every stream keeps its previous frame's feature pyramid and its previous
  output O_{t-1} resident in HBM (two one-image pyramid buffers and two
  output buffers, used alternately), in a slot of its resolution's pool;
  a finished stream's slot goes to the next stream of that resolution.
* Streams are admitted while the slots fit the HBM budget; later ones wait
  in a queue and are admitted as earlier streams finish (idle slots of other
  resolutions are freed to make room).
* Frames arrive on the host clock.  Each pass of the serving loop takes, for
  every resolution, the streams whose next frame has arrived, builds their
  pyramids, decodes all their flow pairs in one batched call
  (tc_flow_from_pyramid_list) and runs their consistency steps, on a HIP
  stream of that resolution, so different resolutions overlap on the device
  and frames that arrive while others run join the next pass.
* With graphs=True each pass of a resolution is one HIP graph launch,
  captured once per ordered set of slots and buffer parities.
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

MAX_BATCH = 16    # pairs per batched decoder call
MAX_GRAPHS = 256  # captured passes kept per resolution


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
    keep_flows: bool = False
    # filled by the server
    outputs: list = field(default_factory=list)
    flows: list = field(default_factory=list)  # (flow_fw, flow_bw) of frames 1, 2, ...
    latencies_ms: list = field(default_factory=list)

    @property
    def hw(self):
        return tuple(self.I[0].shape[2:])

    @property
    def nframes(self):
        return len(self.arrivals)


class _Slot:
    """Device state of one stream: two one-image pyramid buffers and two
    outputs used alternately, its flow pair, and (graph mode) the input slot
    where its next frame I_t and stylized frame P_t are placed.  A slot
    outlives its stream and is handed to the next stream of that resolution."""

    def __init__(self, net, h, w, device, staging):
        pb = net.pyramid_bytes(1, h, w)
        self.pyr = [torch.empty(pb, dtype=torch.uint8, device=device) for _ in range(2)]
        self.out = [torch.empty(1, 3, h, w, device=device) for _ in range(2)]
        self.fw = torch.empty(1, 2, h, w, device=device)
        self.bw = torch.empty(1, 2, h, w, device=device)
        self.I_in = torch.empty(1, 3, h, w, device=device) if staging else None
        self.P_in = torch.empty(1, 3, h, w, device=device) if staging else None
        self.t = 0

    @staticmethod
    def bytes_for(net, h, w, staging):
        return 2 * net.pyramid_bytes(1, h, w) + (2 * 3 + 2 * 2 + (6 if staging else 0)) * h * w * 4


_GROUP_STREAMS = {}


def _group_stream(device, hw):
    """One HIP stream per (device, resolution), shared by every Server:
    streams are spread over a few hardware queues in creation order, so
    creating new ones per server would crowd queues that other work uses."""
    key = (device.index if device.index is not None else torch.cuda.current_device(), hw)
    if key not in _GROUP_STREAMS:
        _GROUP_STREAMS[key] = torch.cuda.Stream(device=device)
    return _GROUP_STREAMS[key]


class Server:
    """Continuous-batching server over one net.

    graphs=True captures each pass of a resolution in a HIP graph (one per
    ordered set of slots and their buffer parities, captured on first use and
    replayed afterwards): the host then enqueues one graph launch per pass
    instead of every kernel.  The captured kernels read the frames from the
    slots' input buffers, so each frame is first copied there (where a host
    upload would land).  Passes that hold a stream's first frame run eagerly.
    """

    def __init__(self, net: tcflow.Net, hbm_budget_bytes: int, device="cuda", graphs=False):
        self.net = net
        self.budget = int(hbm_budget_bytes)
        self.device = torch.device(device)
        self.graphs = bool(graphs)
        self.groups = {}   # (h, w) -> dict(stream, ws, slots {id: _Slot}, free [ids], graphs)
        self.reserved = 0  # bytes held: group workspaces and slots
        self.graphs_captured = 0

    def group_bytes(self, hw):
        return self.net.decoder_list_workspace_bytes(MAX_BATCH, *hw)

    def _group(self, hw):
        g = self.groups.get(hw)
        if g is None:
            st = _group_stream(self.device, hw)
            wb = self.group_bytes(hw)
            with torch.cuda.stream(st):  # memory is tied to the stream that uses it
                ws = torch.empty(wb, dtype=torch.uint8, device=self.device)
            g = dict(stream=st, ws=ws, slots={}, free=[], graphs={}, next_id=0)
            self.groups[hw] = g
            self.reserved += wb
        return g

    def _release_idle(self, keep):
        """Free the idle slots (and the graphs that use them) of every
        resolution but `keep`."""
        for hw, g in self.groups.items():
            if hw == keep or not g["free"]:
                continue
            g["stream"].synchronize()
            idle = set(g["free"])
            for key in [k for k in g["graphs"] if any(m[0] in idle for m in k)]:
                del g["graphs"][key]
            for sid in idle:
                del g["slots"][sid]
                self.reserved -= _Slot.bytes_for(self.net, *hw, self.graphs)
            g["free"].clear()

    def _acquire(self, hw, others_active):
        """A slot for a new stream of resolution hw, or None if the budget
        has no room while other streams are being served."""
        g = self._group(hw)
        if g["free"]:
            sid = g["free"].pop(0)  # first freed first: stable slot order, recurring graph keys
        else:
            need = _Slot.bytes_for(self.net, *hw, self.graphs)
            if self.reserved + need > self.budget:
                self._release_idle(keep=hw)
            if self.reserved + need > self.budget and others_active:
                return None
            with torch.cuda.stream(g["stream"]):
                slot = _Slot(self.net, *hw, self.device, self.graphs)
            sid = g["next_id"]
            g["next_id"] += 1
            g["slots"][sid] = slot
            self.reserved += need
        g["slots"][sid].t = 0
        return sid

    def close(self):
        """Drop every graph and slot (after the device finishes with them)."""
        torch.cuda.synchronize(self.device)
        self.groups.clear()
        self.reserved = 0

    def run(self, jobs, poll_s=2e-4):
        """Serve all jobs to completion; returns a summary dict."""
        queue = sorted(jobs, key=lambda j: j.arrivals[0])
        active = {}          # stream id -> [job, slot id, next frame index]
        for j in jobs:       # workspaces of the resolutions in use are part of the budget
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
                slot = self._acquire(j.hw, bool(active))
                if slot is None:
                    break
                queue.pop(0)
                if j.arrivals[0] < now - 0.05:
                    admitted_late += 1
                active[j.sid] = [j, slot, 0]
            # one pass: every stream whose next frame has arrived, by resolution
            batches = {}
            for m in active.values():
                j, _, k = m
                if k < j.nframes and j.arrivals[k] <= now:
                    batches.setdefault(j.hw, []).append(m)
            if not batches:
                nxt = [j.arrivals[k] for j, _, k in active.values() if k < j.nframes]
                if queue:
                    nxt.append(queue[0].arrivals[0])
                wait = (min(nxt) - now) if nxt else poll_s
                time.sleep(max(0.0, min(wait, 2e-3)))
                continue
            for hw, members in batches.items():
                for i in range(0, len(members), MAX_BATCH):
                    evs = self._pass(hw, members[i:i + MAX_BATCH])
                    pending_events += evs
                    done += len(evs)
            for sid in list(active):
                j, slot, k = active[sid]
                if k >= j.nframes:  # finished: the slot goes back to its resolution's pool
                    del active[sid]
                    self.groups[j.hw]["free"].append(slot)
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        for j, k, ev in pending_events:
            j.latencies_ms.append(origin.elapsed_time(ev) - 1e3 * float(j.arrivals[k]))
        lat = np.concatenate([np.asarray(j.latencies_ms) for j in jobs])
        return dict(frames=int(total), wall_s=wall, frames_per_s=total / wall,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    admitted_late=admitted_late, graphs_captured=self.graphs_captured)

    def _enqueue(self, hw, g, members, staged):
        """Every kernel of one pass, on the current stream."""
        h, w = hw
        pairs = []
        for j, sid, k in members:
            r = g["slots"][sid]
            frame = r.I_in if staged else j.I[k % len(j.I)]
            self.net.pyramid(frame, out=r.pyr[r.t % 2])
            if r.t > 0:
                pairs.append(r)
        if pairs:
            self.net.flow_from_pyramid_list(
                [r.pyr[(r.t - 1) % 2] for r in pairs], [r.pyr[r.t % 2] for r in pairs],
                h, w, [r.fw for r in pairs], [r.bw for r in pairs], g["ws"])
        for j, sid, k in members:
            r = g["slots"][sid]
            cur = r.t % 2
            P = r.P_in if staged else j.P[k % len(j.P)]
            if r.t == 0:
                r.out[cur].copy_(P)
            else:
                tcflow.consistency_step(P, r.out[cur ^ 1], r.fw, r.bw, j.alpha, out=r.out[cur])

    def _pass(self, hw, members):
        """Enqueue one frame for each member (same resolution) on the group's
        HIP stream; returns (job, frame index, completion event) triples."""
        g = self._group(hw)
        out = []
        # graphs once this resolution has decoded eagerly (its kernels have run) and no
        # member is at its first frame
        use_graph = (self.graphs and g.get("warm", False)
                     and all(g["slots"][sid].t > 0 for _, sid, _ in members))
        with torch.cuda.stream(g["stream"]):
            if use_graph:
                for j, sid, k in members:
                    r = g["slots"][sid]
                    r.I_in.copy_(j.I[k % len(j.I)])
                    r.P_in.copy_(j.P[k % len(j.P)])
                key = tuple((sid, g["slots"][sid].t % 2, float(j.alpha)) for j, sid, _ in members)
                graph = g["graphs"].get(key)
                if graph is None:
                    if len(g["graphs"]) >= MAX_GRAPHS:  # drop the oldest once the group is idle
                        g["stream"].synchronize()
                        del g["graphs"][next(iter(g["graphs"]))]
                    graph = torch.cuda.CUDAGraph()
                    graph.capture_begin(capture_error_mode="thread_local")
                    try:
                        self._enqueue(hw, g, members, staged=True)
                    finally:
                        graph.capture_end()
                    g["graphs"][key] = graph
                    self.graphs_captured += 1
                graph.replay()
            else:
                self._enqueue(hw, g, members, staged=False)
                g["warm"] = g.get("warm", False) or any(g["slots"][sid].t > 0
                                                        for _, sid, _ in members)
            for m in members:
                j, sid, k = m
                r = g["slots"][sid]
                if j.keep_outputs:
                    j.outputs.append(r.out[r.t % 2].clone())
                if j.keep_flows and r.t > 0:
                    j.flows.append((r.fw.clone(), r.bw.clone()))
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
