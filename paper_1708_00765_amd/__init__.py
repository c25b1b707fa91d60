"""MI355X-native Chord Length Sampling (Larmier et al., arXiv 1708.00765, Section 4).

`paper_1708_00765_amd.cls` is the ctypes binding of the C ABI in include/cls.h
(HIP kernels for gfx950 in csrc/). `paper_1708_00765_amd.inputs` draws the seeded
synthetic workloads. The binding is imported lazily so that the input generators
stay importable where the library is not built.
"""
__all__ = ["cls", "inputs"]
