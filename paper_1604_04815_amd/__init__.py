"""lscan: a single-pass device-wide scan for AMD MI355X (gfx950).

The scan kernels are hand-written HIP behind a C ABI (``include/lscan.h``);
``binding`` marshals arguments to that library, which must be built
(``__graft_entry__.build()``) -- there is no CPU fallback.
"""
__all__ = ["binding", "workloads"]
