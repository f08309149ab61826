// affine_scan.hip -- a scan with a user-defined, non-commutative operator,
// built only from the public header lscan_custom.hpp: composition of affine
// maps x -> a*x + b over 32-bit unsigned integers (mod 2^32), the earlier map
// applied first.  The b half of the inclusive scan is the linear recurrence
// h_j = a_j * h_{j-1} + b_j (h_{-1} = 0), a first-order recurrence written
// as a scan.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lscan_custom.hpp"

namespace {

struct Affine {
    uint32_t a, b;  // x -> a*x + b
};

struct AffineOp {
    using In = Affine;
    using V = Affine;
    using Out = Affine;
    static constexpr int E = 2;  // two maps per 16-byte vector
    __device__ static V identity() { return Affine{1u, 0u}; }
    // p first, then q: q(p(x)) = q.a * (p.a * x + p.b) + q.b
    __device__ static V combine(V p, V q) { return Affine{q.a * p.a, q.a * p.b + q.b}; }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};

}  // namespace

// Handles of the operator's scan kernel at three tile shapes.
extern "C" const void* lscan_affine_kernel() { return lscan_custom::kernel<AffineOp, 256, 8>(); }
extern "C" const void* lscan_affine_kernel_small() { return lscan_custom::kernel<AffineOp, 64, 1>(); }
extern "C" const void* lscan_affine_kernel_wide() { return lscan_custom::kernel<AffineOp, 512, 8>(); }
