"""Adaptive randomized HSS compression on AMD MI355X (gfx950).

The compute path is libhss.so (C ABI in include/hss.h, HIP kernels in
csrc/); `hss` is its Python binding and `inputs` draws seeded synthetic
workloads.  Build with `python -m paper_1810_04125_amd.build`.
"""
__all__ = ["hss", "inputs", "build"]
