// lscan_custom.hpp -- the persistent single-pass scan for a user-defined
// operator, built in the caller's own HIP translation unit and run through
// lscan_scan_custom (include/lscan.h).
//
// Compile with hipcc for gfx950, with paper_1604_04815_amd/csrc and include/
// on the include path, and with the same flags as the library
// (-Xclang -target-feature -Xclang -packed-fp32-ops).
//
// An operator is a type with
//   using In  = ...;  element type read from x
//   using V   = ...;  value carried through the scan (trivially copyable,
//                     a multiple of 4 bytes)
//   using Out = ...;  element type written to y
//   static constexpr int E = ...;   elements per lane per vector load, with
//                                   E * sizeof(In) of 16 or 8 bytes and
//                                   E * sizeof(Out) of 16 or 32 bytes
//   __device__ static V identity();            the identity e of the operator
//   __device__ static V combine(V a, V b);     a (+) b, a the earlier operand;
//                                              must be associative
//   __device__ static V lift(In x);            element -> value
//   __device__ static Out lower(V v);          value -> output element
// (the same shape as the library's own operators).  Inclusive and exclusive
// plain scans are supported; T threads per workgroup (a multiple of 64, at
// most 1024) and R vector loads per lane fix the tile of T * R * E elements.
//
//   struct MyOp { ... };
//   extern "C" const void* my_scan_kernel() { return lscan_custom::kernel<MyOp, 256, 8>(); }
//   ...
//   lscan_scan_custom((const lscan_custom_kernel*)my_scan_kernel(), x, y, n, 0, nullptr, stream);
#pragma once

#include "lscan.h"
#include "scan_kernel.hpp"

namespace lscan_custom {

template <class Op, int T, int R>
struct Entry {
    static_assert(T % 64 == 0 && T >= 64 && T <= 1024, "wave64 workgroups of up to 1024 threads");
    static_assert(R >= 1, "at least one vector load per lane");
    static_assert(sizeof(typename Op::V) % 4 == 0, "the scan value moves in 32-bit words");

    static lscan::KernelEntry make()
    {
        lscan::KernelEntry k;
        k.abi = lscan::kKernelAbi;
        k.func = reinterpret_cast<const void*>(&lscan::scan_kernel<Op, T, R, lscan::kModePlain>);
        k.launch = &lscan::launch_scan<Op, lscan::kModePlain, T, R>;
        k.block_threads = T;
        k.vectors_per_lane = R;
        k.elems_per_vec = Op::E;
        k.slot_words = int(sizeof(typename Op::V) / 4);
        k.in_bytes = int(sizeof(typename Op::In));
        k.out_bytes = int(sizeof(typename Op::Out));
        k.tile_elems = int64_t(T) * R * Op::E;
        return k;
    }
};

// Handle of the scan kernel for Op with T threads and R vectors per lane
// (one static description per instantiation).
template <class Op, int T = 256, int R = 8>
const lscan_custom_kernel* kernel()
{
    static const lscan::KernelEntry entry = Entry<Op, T, R>::make();
    return reinterpret_cast<const lscan_custom_kernel*>(&entry);
}

}  // namespace lscan_custom
