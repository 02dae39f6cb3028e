"""HAMLS hot path for AMD Instinct MI355X (gfx950).

The compute lives in libhamls.so (hand-written HIP behind the C ABI of
include/hamls.h); `paper_2609_39200_amd.hamls` is the thin ctypes binding with
the same entry-point names.  There is no CPU fallback: importing the binding
without the built library raises.
"""
__all__ = ["hamls", "workloads"]
