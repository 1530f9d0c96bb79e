"""tcflow: per-frame hot path of streaming temporal consistency on MI355X.

The compute path lives in ``libtcflow.so`` (HIP kernels for gfx950 behind a
C ABI, see ``include/tcflow.h``); ``paper_2301_00750_amd.tcflow`` is the thin
ctypes binding.  ``paper_2301_00750_amd.synth`` draws the seeded inputs.
"""
