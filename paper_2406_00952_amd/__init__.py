"""MI355X (gfx950) block omega-circulant preconditioned all-at-once solver.

The compute path is the HIP library libwcirc.so (C ABI in include/wc.h);
`paper_2406_00952_amd.wc` is its ctypes binding.  Build it with
`python -m paper_2406_00952_amd.build`.
"""
__all__ = ["wc"]
