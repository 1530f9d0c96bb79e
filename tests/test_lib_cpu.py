"""The C-ABI library loads and exports every symbol include/tcflow.h declares;
host-side argument checks return their documented status codes.  No GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_00750_amd import build_lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_path():
    if not os.path.exists(build_lib.LIB):
        build_lib.build()
    return build_lib.LIB


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"TC_API\s+[\w\s\*]+?\b(tc_\w+)\s*\(", txt))
    return names


def test_header_declares_expected_calls():
    names = declared_symbols()
    for n in ("tc_flow_estimate", "tc_flow_estimate_pair", "tc_consistency_step",
              "tc_net_create", "tc_net_destroy", "tc_flow_workspace_bytes", "tc_status_str"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in sorted(declared_symbols()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    _lib_path()
    from paper_2301_00750_amd import tcflow
    assert set(tcflow.EXPORTS) == declared_symbols()


@pytest.fixture(scope="module")
def tc():
    _lib_path()
    from paper_2301_00750_amd import tcflow
    return tcflow


@pytest.mark.parametrize("name", ["tiny", "fullhd", "tiny_sepref", "fullhd_sepref"])
def test_weight_floats_matches_generator(tc, name):
    d = synth.load_desc(name)
    cd = tc.NetDesc.from_dict(d)
    assert tc.lib().tc_weight_floats(ctypes.byref(cd)) == synth.blob_floats(d)


def test_status_strings(tc):
    for st in range(7):
        assert tc.lib().tc_status_str(st)
    assert tc.lib().tc_status_str(tc.TC_ERR_SCRATCH) != tc.lib().tc_status_str(99)
    assert b"gfx950" in tc.lib().tc_version()


def test_bad_descriptor_and_weight_count(tc):
    d = synth.load_desc("tiny")
    blob = synth.he_weights(d)
    h = ctypes.c_void_p()
    bad = dict(d, ch=[12, 32, 64, 96])  # not a multiple of 8
    cd = tc.NetDesc.from_dict(bad)
    assert tc.lib().tc_weight_floats(ctypes.byref(cd)) == 0
    st = tc.lib().tc_net_create(ctypes.byref(cd), blob.ctypes.data, blob.size, 0, ctypes.byref(h))
    assert st == tc.TC_ERR_SHAPE
    cd = tc.NetDesc.from_dict(d)
    st = tc.lib().tc_net_create(ctypes.byref(cd), blob.ctypes.data, blob.size - 1, 0, ctypes.byref(h))
    assert st == tc.TC_ERR_SHAPE
    st = tc.lib().tc_net_create(ctypes.byref(cd), blob.ctypes.data, blob.size, 7, ctypes.byref(h))
    assert st == tc.TC_ERR_UNSUPPORTED
    st = tc.lib().tc_net_create(ctypes.byref(cd), None, blob.size, 0, ctypes.byref(h))
    assert st == tc.TC_ERR_INVALID_ARG
    assert h.value is None


def test_consistency_argument_checks(tc):
    L = tc.lib()
    p = ctypes.c_void_p(256)  # never dereferenced: every call below fails its checks first
    assert L.tc_consistency_step(None, p, p, p, 0.5, 1, 4, 4, p, None, None) == tc.TC_ERR_INVALID_ARG
    assert L.tc_consistency_step(p, p, p, p, 1.5, 1, 4, 4, ctypes.c_void_p(512), None, None) == tc.TC_ERR_INVALID_ARG
    assert L.tc_consistency_step(p, p, p, p, float("nan"), 1, 4, 4, ctypes.c_void_p(512), None, None) == tc.TC_ERR_INVALID_ARG
    assert L.tc_consistency_step(p, p, p, p, 0.5, 0, 4, 4, ctypes.c_void_p(512), None, None) == tc.TC_ERR_INVALID_ARG
    assert L.tc_consistency_step(p, p, p, p, 0.5, 1, -3, 4, ctypes.c_void_p(512), None, None) == tc.TC_ERR_INVALID_ARG
    # out aliasing prev_out is rejected
    assert L.tc_consistency_step(p, p, ctypes.c_void_p(768), ctypes.c_void_p(1024), 0.5, 1, 4, 4, p, None, None) == tc.TC_ERR_INVALID_ARG


def test_flow_argument_checks(tc):
    L = tc.lib()
    p = ctypes.c_void_p(256)
    assert L.tc_flow_estimate(None, p, p, 1, 8, 8, p, p, 1 << 20, None) == tc.TC_ERR_INVALID_ARG
    assert L.tc_pyramid_bytes(None, 1, 8, 8) == 0
    assert L.tc_flow_workspace_bytes(None, 1, 8, 8) == 0


def test_noalloc_argument_checks(tc):
    """tc_flow_estimate_pair_noalloc rejects null pointers and bad sizes
    before touching the device; its scratch size is the header's."""
    L = tc.lib()
    p = ctypes.c_void_p(256)
    assert L.tc_flow_estimate_pair_noalloc(None, p, p, 1, 8, 8, p, p, None) == tc.TC_ERR_INVALID_ARG
    txt = open(os.path.join(ROOT, "include", "tcflow.h")).read()
    m = re.search(r"#define TC_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == tc.NOALLOC_SCRATCH_BYTES


def test_head_width_limit(tc):
    """The head's input [h2 | h3] is limited to 128 channels (16 blocks of 8
    on the vector-ALU head): a wider descriptor is rejected at creation."""
    d = dict(synth.load_desc("tiny"), dec=[96, 96, 48])
    cd = tc.NetDesc.from_dict(d)
    assert tc.lib().tc_weight_floats(ctypes.byref(cd)) == 0
    ok = dict(synth.load_desc("tiny"), dec=[96, 96, 32])
    assert tc.lib().tc_weight_floats(ctypes.byref(tc.NetDesc.from_dict(ok))) > 0


def test_fp8_encoder_matches_torch_e4m3fn(tc):
    """The host FP8 encoder of the weights equals torch's float8_e4m3fn cast
    (round to nearest even) on normal, subnormal, tie and boundary values;
    beyond 448 it saturates where torch would give NaN."""
    import torch
    rng = np.random.default_rng(3)
    vals = np.concatenate([
        rng.standard_normal(4000) * 10, rng.standard_normal(2000) * 1e-2,
        rng.uniform(-448, 448, 2000), 2.0 ** -np.arange(0, 12),
        [0.0, -0.0, 448.0, -448.0, 240.0, 0.001953125, 0.0009765625, 1.0625, 1.125 * 1.0625],
        (np.arange(1, 64) + 0.5) * 2.0 ** -9,   # subnormal ties
        (np.arange(8, 16) + 0.5) * 2.0 ** -3,   # normal ties
    ]).astype(np.float32)
    out = np.empty(vals.size, np.uint8)
    tc.lib().tc_fp8_e4m3_encode(vals.ctypes.data, out.ctypes.data, vals.size)
    ref = torch.from_numpy(vals).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(out, ref)
    big = np.array([449.0, 1000.0, -5e5], np.float32)
    o2 = np.empty(3, np.uint8)
    tc.lib().tc_fp8_e4m3_encode(big.ctypes.data, o2.ctypes.data, 3)
    assert list(o2) == [0x7e, 0x7e, 0xfe]


@pytest.mark.parametrize("change", [
    dict(finest=0), dict(finest=5),
    dict(refine={"ch": [48, 4], "dil": [1, 1]}),          # last layer must output 2
    dict(refine={"ch": [12, 2], "dil": [1, 1]}),          # widths are multiples of 8
    dict(refine={"ch": [48, 2], "dil": [0, 1]}),          # dilation >= 1
    dict(refine={"ch": [48, 2], "dil": [1, 65]}),
])
def test_bad_variant_descriptors(tc, change):
    d = dict(synth.load_desc("tiny_sepref"), **change)
    cd = tc.NetDesc.from_dict(d)
    assert tc.lib().tc_weight_floats(ctypes.byref(cd)) == 0
