"""lscan: a single-pass device-wide scan for AMD MI355X (gfx950).

The kernels are hand-written HIP behind a C ABI (``include/lscan.h``);
``binding`` marshals arguments to that library, which must be built
(``__graft_entry__.build()``) -- there is no CPU fallback.  The binding
offers, on device tensors: ``inclusive`` / ``exclusive`` (add, max, min,
argmax, argmin; compensated float sums), ``segmented``, ``batched``,
graph-captured scans, the request ``Server``, ``compact``,
``radix_offsets``, ``bfs`` (breadth-first search on the inter-workgroup
hand-off) and ``scan_custom`` (a scan kernel built for a caller's own
operator with ``include/lscan_custom.hpp``).  ``autotune`` picks tile
shapes; ``workloads`` draws the seeded synthetic inputs.
"""
__all__ = ["binding", "workloads"]
