"""ctypes binding of libtcflow.so (argument marshalling only).

Every function here forwards torch tensors' device pointers and the current
HIP stream to the C ABI declared in include/tcflow.h; all computation happens
in the library's HIP kernels.  If the library is missing or cannot be loaded
the import of this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcflow.so")

(TC_OK, TC_ERR_INVALID_ARG, TC_ERR_SHAPE, TC_ERR_WORKSPACE, TC_ERR_UNSUPPORTED, TC_ERR_HIP,
 TC_ERR_SCRATCH) = range(7)
# static scratch of tc_flow_estimate_pair_noalloc (TC_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 256 << 20
TC_FP32, TC_BF16, TC_FP8_E4M3 = 0, 1, 2
TC_PREC_BF16_FEATURES = 0x100  # OR-ed into TC_BF16 / TC_FP8_E4M3: bfloat16 pyramid features

EXPORTS = (
    "tc_status_str", "tc_version", "tc_weight_floats", "tc_net_create", "tc_net_destroy",
    "tc_pyramid_bytes", "tc_pyramid", "tc_decoder_workspace_bytes", "tc_flow_from_pyramids",
    "tc_flow_workspace_bytes", "tc_flow_estimate", "tc_flow_estimate_pair",
    "tc_consistency_step", "tc_probe_enable", "tc_probe_read", "tc_probe_disable",
    "tc_paper_default_params", "tc_paper_workspace_bytes", "tc_consistency_paper",
    "tc_fp8_e4m3_encode", "tc_decoder_list_workspace_bytes", "tc_flow_from_pyramid_list",
    "tc_train_default_params", "tc_trainer_create", "tc_trainer_destroy", "tc_trainer_grad",
    "tc_trainer_step", "tc_trainer_copy", "tc_trainer_steps_done", "tc_flow_agreement",
    "tc_flow_half_workspace_bytes", "tc_flow_estimate_pair_half", "tc_paper_preset_params",
    "tc_flow_estimate_pair_noalloc",
)

TC_PRESET_FINAL, TC_PRESET_OBJECTIVE, TC_PRESET_FAST = 0, 1, 2
PRESETS = {"final": TC_PRESET_FINAL, "objective": TC_PRESET_OBJECTIVE, "fast": TC_PRESET_FAST}

(TC_OP_PYR_A, TC_OP_PYR_B, TC_OP_UP2, TC_OP_COST_VOLUME, TC_OP_C1, TC_OP_C2, TC_OP_C3, TC_OP_HEAD,
 TC_OP_REFINE) = range(9)
TC_STAGE_INPUT, TC_STAGE_OUTPUT, TC_STAGE_CONSISTENCY, TC_STAGE_PAPER = 1, 2, 3, 4


def stage_id(level, op):
    return level * 16 + op


class TcError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn} failed: {status} ({_lib.tc_status_str(status).decode()})")


class NetDesc(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("ch", ctypes.c_int * 8), ("dec", ctypes.c_int * 3),
                ("radius", ctypes.c_int), ("leaky", ctypes.c_float), ("finest", ctypes.c_int),
                ("ref_layers", ctypes.c_int), ("ref_ch", ctypes.c_int * 8),
                ("ref_dil", ctypes.c_int * 8)]

    @classmethod
    def from_dict(cls, d):
        s = cls()
        s.levels = d["levels"]
        for i, c in enumerate(d["ch"]):
            s.ch[i] = c
        for i, c in enumerate(d["dec"]):
            s.dec[i] = c
        s.radius = d["radius"]
        s.leaky = d["leaky"]
        s.finest = d.get("finest", 1)
        ref = d.get("refine") or {}
        s.ref_layers = len(ref.get("ch", []))
        for i, (c, dl) in enumerate(zip(ref.get("ch", []), ref.get("dil", []))):
            s.ref_ch[i] = c
            s.ref_dil[i] = dl
        return s


class PaperParams(ctypes.Structure):
    """tc_paper_params: k1, k2, a_ph, lambda, eta, kappa, iterations."""
    _fields_ = [("k1", ctypes.c_float), ("k2", ctypes.c_float), ("a_ph", ctypes.c_float),
                ("lam", ctypes.c_float), ("eta", ctypes.c_float), ("kappa", ctypes.c_float),
                ("iterations", ctypes.c_int)]


class TrainParams(ctypes.Structure):
    """tc_train_params: lr, beta1, beta2, eps, weight_decay, loss_eps, loss_q."""
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float),
                ("loss_eps", ctypes.c_float), ("loss_q", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cf, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t
    sig = {
        "tc_status_str": (ctypes.c_char_p, [ci]),
        "tc_version": (ctypes.c_char_p, []),
        "tc_weight_floats": (sz, [ctypes.POINTER(NetDesc)]),
        "tc_net_create": (ci, [ctypes.POINTER(NetDesc), vp, sz, ci, ctypes.POINTER(vp)]),
        "tc_net_destroy": (None, [vp]),
        "tc_pyramid_bytes": (sz, [vp, ci, ci, ci]),
        "tc_pyramid": (ci, [vp, vp, ci, ci, ci, vp, sz, vp]),
        "tc_decoder_workspace_bytes": (sz, [vp, ci, ci, ci]),
        "tc_flow_from_pyramids": (ci, [vp, vp, vp, ci, ci, ci, vp, vp, vp, sz, vp]),
        "tc_flow_workspace_bytes": (sz, [vp, ci, ci, ci]),
        "tc_flow_estimate": (ci, [vp, vp, vp, ci, ci, ci, vp, vp, sz, vp]),
        "tc_flow_estimate_pair": (ci, [vp, vp, vp, ci, ci, ci, vp, vp, vp, sz, vp]),
        "tc_consistency_step": (ci, [vp, vp, vp, vp, cf, ci, ci, ci, vp, vp, vp]),
        "tc_probe_enable": (ci, [ci, ci]),
        "tc_probe_read": (ci, [ctypes.POINTER(ci), ctypes.POINTER(cf)]),
        "tc_probe_disable": (None, []),
        "tc_paper_default_params": (None, [ctypes.POINTER(PaperParams)]),
        "tc_paper_workspace_bytes": (sz, [ci, ci, ci]),
        "tc_fp8_e4m3_encode": (None, [vp, vp, sz]),
        "tc_decoder_list_workspace_bytes": (sz, [vp, ci, ci, ci]),
        "tc_flow_from_pyramid_list": (ci, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ci, ci, ci,
                                           ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp]),
        "tc_consistency_paper": (ci, [vp] * 9 + [ctypes.POINTER(PaperParams), ci, ci, ci, vp, vp,
                                                 sz, vp]),
        "tc_train_default_params": (None, [ctypes.POINTER(TrainParams)]),
        "tc_trainer_create": (ci, [ctypes.POINTER(NetDesc), vp, sz, ctypes.POINTER(TrainParams), ci,
                                   ci, ci, ctypes.POINTER(vp)]),
        "tc_trainer_destroy": (None, [vp]),
        "tc_trainer_grad": (ci, [vp, vp, vp, vp, ci, vp, vp]),
        "tc_trainer_step": (ci, [vp, vp, vp, vp, ci, vp, vp]),
        "tc_trainer_copy": (ci, [vp, ci, vp, vp]),
        "tc_trainer_steps_done": (ci, [vp]),
        "tc_flow_agreement": (ci, [vp, vp, ci, ci, ci, vp, vp]),
        "tc_flow_half_workspace_bytes": (sz, [vp, ci, ci, ci]),
        "tc_flow_estimate_pair_half": (ci, [vp, vp, vp, ci, ci, ci, vp, vp, vp, sz, vp]),
        "tc_paper_preset_params": (ci, [ci, ctypes.POINTER(PaperParams)]),
        "tc_flow_estimate_pair_noalloc": (ci, [vp, vp, vp, ci, ci, ci, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(fn, st):
    if st != TC_OK:
        raise TcError(fn, st)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _frames(t, name, ch):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and t.dim() == 4 and t.shape[1] == ch):
        raise ValueError(f"{name}: expected a contiguous cuda float32 tensor n x {ch} x h x w")
    return t


def _out(t, name, shape, device, dtype=torch.float32):
    """A caller-supplied output: `shape`, `dtype`, contiguous, on `device`
    (the C ABI takes no size for outputs, so a short buffer would be written
    past its end)."""
    if not (isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_contiguous()
            and t.device == device and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor of shape {tuple(shape)} "
                         f"on {device}")
    return t


def _buffer(t, name, nbytes, device):
    """A caller-supplied byte buffer (pyramid, workspace) of at least nbytes."""
    if not (isinstance(t, torch.Tensor) and t.is_contiguous() and t.device == device
            and t.numel() * t.element_size() >= nbytes):
        raise ValueError(f"{name}: expected a contiguous buffer of >= {nbytes} bytes on {device}")
    return t


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Net:
    """A packed network on the current HIP device (tc_net_create)."""

    def __init__(self, desc: dict, weights, precision: int = TC_FP32):
        self.desc = dict(desc)
        self._cdesc = NetDesc.from_dict(desc)
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        h = ctypes.c_void_p()
        _check("tc_net_create", _lib.tc_net_create(ctypes.byref(self._cdesc), w.ctypes.data,
                                                   w.size, precision, ctypes.byref(h)))
        self._h = h
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.tc_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ---- sizes
    def pyramid_bytes(self, n, h, w):
        return _lib.tc_pyramid_bytes(self._h, n, h, w)

    def decoder_workspace_bytes(self, n, h, w):
        return _lib.tc_decoder_workspace_bytes(self._h, n, h, w)

    def flow_workspace_bytes(self, n, h, w):
        return _lib.tc_flow_workspace_bytes(self._h, n, h, w)

    # ---- calls
    def pyramid(self, frames, out=None, stream=None):
        _frames(frames, "frames", 3)
        n, _, h, w = frames.shape
        nb = self.pyramid_bytes(n, h, w)
        if out is None:
            out = _workspace(nb, frames.device)
        _check("tc_pyramid", _lib.tc_pyramid(self._h, _ptr(frames), n, h, w, _ptr(out),
                                             out.numel() * out.element_size(), _stream(stream)))
        return out

    def flow_from_pyramids(self, pyr1, pyr2, n, h, w, both=True, ws=None, out12=None, out21=None,
                           stream=None):
        dev = pyr1.device
        pb = self.pyramid_bytes(n, h, w)
        _buffer(pyr1, "pyr1", pb, dev)
        _buffer(pyr2, "pyr2", pb, dev)
        if ws is None:
            ws = _workspace(self.decoder_workspace_bytes(n, h, w), dev)
        f12 = (_out(out12, "out12", (n, 2, h, w), dev) if out12 is not None
               else torch.empty(n, 2, h, w, device=dev))
        f21 = None
        if both:
            f21 = (_out(out21, "out21", (n, 2, h, w), dev) if out21 is not None
                   else torch.empty(n, 2, h, w, device=dev))
        _check("tc_flow_from_pyramids", _lib.tc_flow_from_pyramids(
            self._h, _ptr(pyr1), _ptr(pyr2), n, h, w, _ptr(f12), _ptr(f21), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream)))
        return (f12, f21) if both else f12

    def decoder_list_workspace_bytes(self, n, h, w):
        return _lib.tc_decoder_list_workspace_bytes(self._h, n, h, w)

    def flow_from_pyramid_list(self, pyr_prev, pyr_cur, h, w, fw, bw, ws, stream=None):
        """One batched decoder pass over per-stream one-image pyramids
        (tc_flow_from_pyramid_list); fw[i], bw[i] are 1 x 2 x h x w outputs."""
        n = len(pyr_prev)
        if not (len(pyr_cur) == len(fw) == len(bw) == n):
            raise ValueError("pyr_prev, pyr_cur, fw and bw differ in length")
        dev = ws.device
        pb = self.pyramid_bytes(1, h, w)
        for i in range(n):
            _buffer(pyr_prev[i], f"pyr_prev[{i}]", pb, dev)
            _buffer(pyr_cur[i], f"pyr_cur[{i}]", pb, dev)
            _out(fw[i], f"fw[{i}]", (1, 2, h, w), dev)
            _out(bw[i], f"bw[{i}]", (1, 2, h, w), dev)
        arr = ctypes.c_void_p * n
        _check("tc_flow_from_pyramid_list", _lib.tc_flow_from_pyramid_list(
            self._h, arr(*[p.data_ptr() for p in pyr_prev]), arr(*[p.data_ptr() for p in pyr_cur]),
            n, h, w, arr(*[f.data_ptr() for f in fw]), arr(*[f.data_ptr() for f in bw]), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream)))

    def flow_half_workspace_bytes(self, n, h, w):
        return _lib.tc_flow_half_workspace_bytes(self._h, n, h, w)

    def flow_estimate_pair_half(self, prev, cur, ws=None, out_fw=None, out_bw=None, stream=None):
        """Flow pair of the fast preset: estimated on 2x2-block-mean half-size
        frames, upsampled back (tc_flow_estimate_pair_half)."""
        _frames(prev, "prev", 3)
        _frames(cur, "cur", 3)
        if prev.shape != cur.shape:
            raise ValueError("prev and cur differ in shape")
        n, _, h, w = prev.shape
        if ws is None:
            ws = _workspace(self.flow_half_workspace_bytes(n, h, w), prev.device)
        fw, bw = self._pair_outputs(out_fw, out_bw, n, h, w, prev.device)
        _check("tc_flow_estimate_pair_half", _lib.tc_flow_estimate_pair_half(
            self._h, _ptr(prev), _ptr(cur), n, h, w, _ptr(fw), _ptr(bw), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream)))
        return fw, bw

    def flow_estimate(self, prev, cur, ws=None, out=None, stream=None):
        _frames(prev, "prev", 3)
        _frames(cur, "cur", 3)
        if prev.shape != cur.shape:
            raise ValueError("prev and cur differ in shape")
        n, _, h, w = prev.shape
        if ws is None:
            ws = _workspace(self.flow_workspace_bytes(n, h, w), prev.device)
        f = (_out(out, "out", (n, 2, h, w), prev.device) if out is not None
             else torch.empty(n, 2, h, w, device=prev.device))
        _check("tc_flow_estimate", _lib.tc_flow_estimate(
            self._h, _ptr(prev), _ptr(cur), n, h, w, _ptr(f), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream)))
        return f

    def flow_estimate_pair(self, prev, cur, ws=None, out_fw=None, out_bw=None, stream=None):
        _frames(prev, "prev", 3)
        _frames(cur, "cur", 3)
        if prev.shape != cur.shape:
            raise ValueError("prev and cur differ in shape")
        n, _, h, w = prev.shape
        if ws is None:
            ws = _workspace(self.flow_workspace_bytes(n, h, w), prev.device)
        fw, bw = self._pair_outputs(out_fw, out_bw, n, h, w, prev.device)
        _check("tc_flow_estimate_pair", _lib.tc_flow_estimate_pair(
            self._h, _ptr(prev), _ptr(cur), n, h, w, _ptr(fw), _ptr(bw), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream)))
        return fw, bw

    def flow_estimate_pair_noalloc(self, prev, cur, out_fw, out_bw, stream=None):
        """tc_flow_estimate_pair_noalloc: the flow pair with the library's
        static per-device scratch instead of a workspace.  The outputs are
        caller-owned (nothing is allocated here either); calls that overlap
        on one GPU race on the shared scratch."""
        _frames(prev, "prev", 3)
        _frames(cur, "cur", 3)
        if prev.shape != cur.shape:
            raise ValueError("prev and cur differ in shape")
        n, _, h, w = prev.shape
        _out(out_fw, "out_fw", (n, 2, h, w), prev.device)
        _out(out_bw, "out_bw", (n, 2, h, w), prev.device)
        _check("tc_flow_estimate_pair_noalloc", _lib.tc_flow_estimate_pair_noalloc(
            self._h, _ptr(prev), _ptr(cur), n, h, w, _ptr(out_fw), _ptr(out_bw), _stream(stream)))
        return out_fw, out_bw

    @staticmethod
    def _pair_outputs(out_fw, out_bw, n, h, w, device):
        fw = (_out(out_fw, "out_fw", (n, 2, h, w), device) if out_fw is not None
              else torch.empty(n, 2, h, w, device=device))
        bw = (_out(out_bw, "out_bw", (n, 2, h, w), device) if out_bw is not None
              else torch.empty(n, 2, h, w, device=device))
        return fw, bw


def consistency_step(stylized, prev_out, flow_fw, flow_bw, alpha, out=None, mask=False,
                     stream=None):
    """out_t (and the uint8 visibility mask if ``mask``) from the C ABI."""
    _frames(stylized, "stylized", 3)
    _frames(prev_out, "prev_out", 3)
    _frames(flow_fw, "flow_fw", 2)
    _frames(flow_bw, "flow_bw", 2)
    n, _, h, w = stylized.shape
    for t in (prev_out, flow_fw, flow_bw):
        if t.shape[0] != n or t.shape[2:] != stylized.shape[2:]:
            raise ValueError("consistency_step: shapes differ")
    o = (_out(out, "out", (n, 3, h, w), stylized.device) if out is not None
         else torch.empty_like(stylized))
    m = torch.empty(n, h, w, dtype=torch.uint8, device=stylized.device) if mask else None
    _check("tc_consistency_step", _lib.tc_consistency_step(
        _ptr(stylized), _ptr(prev_out), _ptr(flow_fw), _ptr(flow_bw), float(alpha), n, h, w,
        _ptr(o), _ptr(m), _stream(stream)))
    return (o, m) if mask else o


def flow_agreement(flow_fw, flow_bw, counts=None, stream=None):
    """Per image, the number of pixels passing the forward-backward test
    (tc_flow_agreement), as a cuda int32 tensor (values are unsigned)."""
    _frames(flow_fw, "flow_fw", 2)
    _frames(flow_bw, "flow_bw", 2)
    n, _, h, w = flow_fw.shape
    if flow_bw.shape != flow_fw.shape:
        raise ValueError("flow_agreement: shapes differ")
    c = (_out(counts, "counts", (n,), flow_fw.device, torch.int32) if counts is not None
         else torch.empty(n, dtype=torch.int32, device=flow_fw.device))
    _check("tc_flow_agreement", _lib.tc_flow_agreement(_ptr(flow_fw), _ptr(flow_bw), n, h, w,
                                                       _ptr(c), _stream(stream)))
    return c


def paper_params(**kw):
    """The paper's final parameter set, with keyword overrides
    (k1, k2, a_ph, lam, eta, kappa, iterations)."""
    p = PaperParams()
    _lib.tc_paper_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def paper_preset(name, **kw):
    """The paper's parameter preset `name` ("final", "objective", "fast";
    tc_paper_preset_params), with keyword overrides."""
    p = PaperParams()
    _check("tc_paper_preset_params", _lib.tc_paper_preset_params(PRESETS[name], ctypes.byref(p)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def consistency_paper(I_prev, I, I_next, P_prev, P, P_next, O_prev, flow_t_prev, flow_t_next,
                      params=None, out=None, ws=None, stream=None):
    """O_t of the paper's full consistency step (tc_consistency_paper)."""
    for name, t in (("I_prev", I_prev), ("I", I), ("I_next", I_next), ("P_prev", P_prev),
                    ("P", P), ("P_next", P_next), ("O_prev", O_prev)):
        _frames(t, name, 3)
    _frames(flow_t_prev, "flow_t_prev", 2)
    _frames(flow_t_next, "flow_t_next", 2)
    n, _, h, w = I.shape
    for t in (I_prev, I_next, P_prev, P, P_next, O_prev, flow_t_prev, flow_t_next):
        if t.shape[0] != n or t.shape[2:] != I.shape[2:]:
            raise ValueError("consistency_paper: shapes differ")
    prm = params if params is not None else paper_params()
    if ws is None:
        ws = _workspace(_lib.tc_paper_workspace_bytes(n, h, w), I.device)
    o = _out(out, "out", (n, 3, h, w), I.device) if out is not None else torch.empty_like(I)
    _check("tc_consistency_paper", _lib.tc_consistency_paper(
        _ptr(I_prev), _ptr(I), _ptr(I_next), _ptr(P_prev), _ptr(P), _ptr(P_next), _ptr(O_prev),
        _ptr(flow_t_prev), _ptr(flow_t_next), ctypes.byref(prm), n, h, w, _ptr(o), _ptr(ws),
        ws.numel() * ws.element_size(), _stream(stream)))
    return o


class Probe:
    """HIP-event timing of every launch of one stage (tc_probe_*)."""

    def __init__(self, stage, max_launches):
        _check("tc_probe_enable", _lib.tc_probe_enable(stage, max_launches))

    def read(self):
        n, ms = ctypes.c_int(), ctypes.c_float()
        _check("tc_probe_read", _lib.tc_probe_read(ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def close(self):
        _lib.tc_probe_disable()


_PIPELINE_STREAMS = {}


def _pipeline_streams(device):
    """The side streams of the pipelined driver (pyramids, two decoder
    lanes), created once per device and shared by every StreamState.  HIP
    spreads streams over a few hardware queues in creation order; streams
    created anew for every driver would, after a few drivers, land on the
    queue of another lane or of the caller's stream and serialise with it."""
    d = torch.device(device)
    key = d.index if d.index is not None else torch.cuda.current_device()
    if key not in _PIPELINE_STREAMS:
        _PIPELINE_STREAMS[key] = tuple(torch.cuda.Stream(device=d) for _ in range(3))
    return _PIPELINE_STREAMS[key]


class StreamState:
    """Streaming driver over the C ABI: O_1 = P_1; for each new frame, the
    pyramid of I_t (the previous frame's pyramid is kept), both flows decoded
    from the two pyramids in one batch, and the consistency step.

    ``pipelined`` spreads the work over HIP streams: pyramids on one side
    stream, the flow decoders of consecutive frames alternately on two more
    (the flows of frame t do not depend on those of frame t - 1; only the
    consistency step is sequential), and the consistency steps in order on
    the caller's current stream.  Events order every buffer reuse.  Results
    are bitwise the same with and without pipelining.  All buffers are
    allocated once."""

    def __init__(self, net: Net, n: int, h: int, w: int, device="cuda", pipelined=True):
        self.net, self.n, self.h, self.w = net, n, h, w
        self.pipelined = pipelined
        pb = net.pyramid_bytes(n, h, w)
        self.ns = 4 if pipelined else 2          # pyramid slots
        self.nd = 2 if pipelined else 1          # decoder lanes
        self.pyr = [_workspace(pb, device) for _ in range(self.ns)]
        wb = net.decoder_workspace_bytes(n, h, w)
        self.ws = [_workspace(wb, device) for _ in range(self.nd)]
        self.fw = [torch.empty(n, 2, h, w, device=device) for _ in range(self.nd)]
        self.bw = [torch.empty(n, 2, h, w, device=device) for _ in range(self.nd)]
        self.out = [torch.empty(n, 3, h, w, device=device), torch.empty(n, 3, h, w, device=device)]
        if pipelined:
            self.s_pyr, *self.s_dec = _pipeline_streams(device)
        self.ev_pyr = [torch.cuda.Event() for _ in range(self.ns)]
        self.ev_dec = [torch.cuda.Event() for _ in range(self.ns)]   # by frame % ns
        self.ev_con = [torch.cuda.Event() for _ in range(self.nd)]   # by frame % nd
        self.t = 0

    def push(self, I, P, alpha, inputs_ready=False, events=None):
        """Enqueue frame t; returns O_t (a view into an internal double buffer),
        ordered on the current stream.  ``events`` = (start, end) CUDA events
        recorded right before this frame's first kernel and after its last
        one (frame latency).

        ``inputs_ready``: I is already complete on the device (no pending
        work on the current stream writes it), so its pyramid may start at
        once on the side stream; otherwise the side stream first waits for
        the current stream, which keeps results correct but removes the
        overlap."""
        main = torch.cuda.current_stream()
        t, ns, nd = self.t, self.ns, self.nd
        slot, lane, o = t % ns, t % nd, t % 2
        if not self.pipelined:
            if events:
                events[0].record(main)
            self.net.pyramid(I, out=self.pyr[slot], stream=main)
            if t > 0:
                self._decode_and_blend(t, P, alpha, main, main)
            else:
                self.out[o].copy_(P)
            if events:
                events[1].record(main)
            self.t += 1
            return self.out[o]

        sp = self.s_pyr
        # slot t % ns last held frame t - ns, read by the decoders of frames
        # t - ns and t - ns + 1
        for k in (t - ns, t - ns + 1):
            if k >= 1:
                sp.wait_event(self.ev_dec[k % ns])
        if not inputs_ready:
            sp.wait_stream(main)
        I.record_stream(sp)
        if events:
            events[0].record(sp)
        self.net.pyramid(I, out=self.pyr[slot], stream=sp)
        self.ev_pyr[slot].record(sp)
        if t == 0:
            main.wait_event(self.ev_pyr[slot])
            self.out[o].copy_(P)
        else:
            sd = self.s_dec[lane]
            sd.wait_event(self.ev_pyr[slot])
            if t - nd >= 1:  # flow buffers of this lane were read by consistency(t - nd)
                sd.wait_event(self.ev_con[lane])
            self._decode(t, sd)
            self.ev_dec[slot].record(sd)
            main.wait_event(self.ev_dec[slot])
            self._blend(t, P, alpha, main)
            self.ev_con[lane].record(main)
        if events:
            events[1].record(main)
        self.t += 1
        return self.out[o]

    def _decode(self, t, stream):
        lane = t % self.nd
        prev, cur = (t - 1) % self.ns, t % self.ns
        self.net.flow_from_pyramids(self.pyr[prev], self.pyr[cur], self.n, self.h, self.w,
                                    both=True, ws=self.ws[lane], out12=self.fw[lane],
                                    out21=self.bw[lane], stream=stream)

    def _blend(self, t, P, alpha, stream):
        lane, o = t % self.nd, t % 2
        consistency_step(P, self.out[o ^ 1], self.fw[lane], self.bw[lane], alpha,
                         out=self.out[o], stream=stream)

    def _decode_and_blend(self, t, P, alpha, sdec, smain):
        self._decode(t, sdec)
        self._blend(t, P, alpha, smain)

    @property
    def flows(self):
        """(flow_fw, flow_bw) of the last pushed frame (after synchronising)."""
        lane = (self.t - 1) % self.nd
        return self.fw[lane], self.bw[lane]


class GraphStreamState:
    """The unpipelined streaming driver with each frame's work (pyramid of
    I_t, the flow pair from the two pyramids, the consistency step) replayed
    as one HIP graph: captured once per buffer parity and strength alpha, then
    launched with a single call.  The frame and the stylized frame are first
    copied into fixed input buffers (where an upload would land), since a
    graph's kernels read fixed addresses.  Frames 0 and 1 run eagerly (the
    first frame only copies P; the second is the first decode, which runs
    every kernel once before any capture).  Outputs are bitwise those of
    StreamState."""

    def __init__(self, net: Net, n: int, h: int, w: int, device="cuda"):
        self.st = StreamState(net, n, h, w, device=device, pipelined=False)
        self.I_in = torch.empty(n, 3, h, w, device=device)
        self.P_in = torch.empty(n, 3, h, w, device=device)
        self.graphs = {}

    @property
    def t(self):
        return self.st.t

    def push(self, I, P, alpha, events=None):
        """Enqueue frame t on the current stream; returns O_t (a view into the
        driver's double buffer).  ``events`` = (start, end) recorded around
        the input copies and the frame's work."""
        main = torch.cuda.current_stream()
        if events:
            events[0].record(main)
        self.I_in.copy_(I)
        self.P_in.copy_(P)
        t = self.st.t
        if t < 2:
            out = self.st.push(self.I_in, self.P_in, alpha)
        else:
            key = (t % 2, float(alpha))
            g = self.graphs.get(key)
            if g is None:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    self.st.push(self.I_in, self.P_in, alpha)
                self.st.t = t  # capture records the frame's work; it runs at replay
                self.graphs[key] = g
            g.replay()
            self.st.t = t + 1
            out = self.st.out[t % 2]
        if events:
            events[1].record(main)
        return out


def train_params(**kw):
    """tc_train_default_params with fields overridden by keyword."""
    p = TrainParams()
    _lib.tc_train_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Trainer:
    """tc_trainer: FP32 training of a network on teacher flows (AdamW)."""

    def __init__(self, desc: dict, weights, max_n: int, h: int, w: int, params=None):
        self.desc = dict(desc)
        self._cdesc = NetDesc.from_dict(desc)
        self._prm = params if params is not None else train_params()
        wb = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        self.n_floats = wb.size
        self.h, self.w, self.max_n = h, w, max_n
        hdl = ctypes.c_void_p()
        _check("tc_trainer_create", _lib.tc_trainer_create(
            ctypes.byref(self._cdesc), wb.ctypes.data, wb.size, ctypes.byref(self._prm), max_n, h,
            w, ctypes.byref(hdl)))
        self._h = hdl
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.tc_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, A, B, T):
        _frames(A, "A", 3)
        _frames(B, "B", 3)
        _frames(T, "teacher", 2)
        if A.shape != B.shape or A.shape[2:] != (self.h, self.w) or T.shape[0] != A.shape[0] \
                or T.shape[2:] != A.shape[2:]:
            raise ValueError("frames and teacher flows must be n x {3,2} x h x w of the trainer")
        return A.shape[0]

    def grad(self, A, B, T, stream=None):
        n = self._args(A, B, T)
        _check("tc_trainer_grad", _lib.tc_trainer_grad(self._h, _ptr(A), _ptr(B), _ptr(T), n,
                                                       _ptr(self.loss), _stream(stream)))
        return self.loss

    def step(self, A, B, T, stream=None):
        n = self._args(A, B, T)
        _check("tc_trainer_step", _lib.tc_trainer_step(self._h, _ptr(A), _ptr(B), _ptr(T), n,
                                                       _ptr(self.loss), _stream(stream)))
        return self.loss

    def copy(self, which: int = 0):
        """Weights (0), gradient (1), Adam moments (2, 3) as a float32 cuda tensor."""
        out = torch.empty(self.n_floats, dtype=torch.float32, device="cuda")
        _check("tc_trainer_copy", _lib.tc_trainer_copy(self._h, which, _ptr(out), _stream()))
        return out

    @property
    def steps_done(self):
        return _lib.tc_trainer_steps_done(self._h)
