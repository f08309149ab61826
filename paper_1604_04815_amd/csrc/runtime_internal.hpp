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

}  // namespace lscan
