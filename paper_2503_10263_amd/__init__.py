"""KARL particle-history transport on MI355X (HIP, gfx950).

`workloads` builds seeded synthetic problem descriptions; `karl` is the thin ctypes
binding of the C-ABI library libkarl.so (imported on demand so that the workload
module can be used without a GPU).
"""
__all__ = ["workloads", "karl"]
