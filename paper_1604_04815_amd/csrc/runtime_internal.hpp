// runtime_internal.hpp -- helpers of runtime.cpp shared with the server.
#pragma once

#include <cstdint>

#include "lscan.h"

namespace lscan {

// Validate one array request as lscan_inclusive / lscan_batched would
// (dtype, operator, flags, pointers, alignment, overlap).
lscan_status validate_request(const void* x, const void* y, int64_t n, int dt, int op, uint32_t flags);

// Bytes one request moves: n * (sizeof input + sizeof output).
uint64_t request_bytes(int64_t n, int dt);

// Vector registers per lane of the plain (batched = false) or batched
// kernel for (dt, op, flags) and a tile shape, from the code object (-1 if
// unknown).
int kernel_vgprs(bool batched, int dt, int op, uint32_t flags, int threads, int vectors);

// lscan_inclusive / lscan_exclusive (flags & LSCAN_F_EXCLUSIVE) with the
// given parameters (null: the defaults), also raising *status_host on a
// timeout.
lscan_status launch_single(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                           const lscan_params* p, void* stream, uint32_t* status_host);

// lscan_batched_with_params that also raises *status_host (a device-visible
// pointer to host memory, may be null) if a workgroup times out.
lscan_status launch_batched(const lscan_array* arrays, int64_t count, lscan_dtype dt, lscan_op op, uint32_t flags,
                            const lscan_params* p, void* stream, uint32_t* status_host);

}  // namespace lscan
