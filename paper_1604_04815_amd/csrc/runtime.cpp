// runtime.cpp -- host side of the C ABI declared in include/lscan.h:
// argument validation, kernel selection, grid sizing against the occupancy
// limit and a co-residency test, the per-(device, stream) flag workspaces,
// batched descriptors and graph-captured launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>

#include "bfs_kernel.hpp"
#include "kernel_table.hpp"
#include "radix_kernel.hpp"
#include "lscan.h"
#include "lscan_testing.h"
#include "runtime_internal.hpp"

namespace lscan {
namespace {

KernelTable g_table;
std::once_flag g_table_once;

void init_table()
{
    std::memset(&g_table, 0, sizeof(g_table));
    register_i32_kernels(g_table);
    register_i64_kernels(g_table);
    register_f32_kernels(g_table);
    register_bf16_kernels(g_table);
    register_i32_seg_kernels(g_table);
    register_i64_seg_kernels(g_table);
    register_f32_seg_kernels(g_table);
    register_bf16_seg_kernels(g_table);
    register_i32_batch_kernels(g_table);
    register_i64_batch_kernels(g_table);
    register_f32_batch_kernels(g_table);
    register_bf16_batch_kernels(g_table);
    register_compact_kernels(g_table);
    register_arg_kernels(g_table);
    register_arg_short_kernels(g_table);
}

const KernelTable& table()
{
    std::call_once(g_table_once, init_table);
    return g_table;
}

thread_local int32_t t_last_hip_error = 0;
thread_local lscan_launch_info t_last_launch = {};

// A wait for a block aggregate normally lasts microseconds; two seconds means
// the grid is not making progress (e.g. not all workgroups are resident).
constexpr double kSpinLimitSeconds = 2.0;

// The watchdog of the launches made from now on (lscan_set_watchdog_us).
int64_t g_watchdog_us = int64_t(kSpinLimitSeconds * 1e6);

// A co-residency test waits this long for the whole grid to arrive.
constexpr double kResidencyWaitSeconds = 0.02;
// Workgroups per CU a kernel built for a user operator asks for by default
// (the co-residency test may lower it).
constexpr int kCustomGroupsPerCu = 2;

// Tags are 32-bit and 0 marks a never-written slot: reset a workspace well
// before its tag counter could wrap.
constexpr uint64_t kMaxLaunchesPerEpochRun = 0xfffffff0ull;

struct DeviceInfo {
    int cu_count = 0;
    uint64_t spin_limit = 0;
    uint64_t residency_limit = 0;
    uint64_t wall_khz = 0;
    int occupancy[kNumModes][kNumOpCodes][kNumShapes];
    // groups per CU proven resident together (0: none yet) and the smallest
    // count that failed the test (0: none failed)
    int resident_ok[kNumModes][kNumOpCodes][kNumShapes];
    int resident_fail[kNumModes][kNumOpCodes][kNumShapes];
    // the breadth-first search kernel: occupancy and co-residency results
    int bfs_occupancy = -1;
    int bfs_resident_ok = 0;
    int bfs_resident_fail = 0;
    // kernels built for user operators, by entry: occupancy, groups proven
    // resident, smallest failing count
    struct Custom {
        int occupancy = -1;
        int ok = 0;
        int fail = 0;
    };
    std::map<const void*, Custom> custom;
};

// Flag slots, control words and (batched launches) array descriptors of one
// launch sequence.  Launches that share a workspace must be stream-ordered.
struct Workspace {
    uint64_t* slots = nullptr;
    size_t words = 0;
    uint32_t* ctrl = nullptr;   // [0] last tag, [1] exit counter, [2] timeout flag, [4..6] residency test
    uint64_t launches = 0;
    BatchArray* desc = nullptr;        // device copy of the descriptor table
    size_t desc_cap = 0;
    BatchArray* desc_host = nullptr;   // pinned staging copy
    hipEvent_t desc_copied = nullptr;  // recorded after each upload from desc_host
    bool desc_pending = false;
    int64_t* seg_first = nullptr;      // segmented scans: first segment of every block
    size_t seg_cap = 0;
    bool fixed = false;                // slots and ctrl live in memory the library never frees or grows
};

struct Params {
    int shape;
    int groups_per_cu;
    int handoff = LSCAN_HANDOFF_WINDOW;
};

std::mutex g_mu;
std::map<int, DeviceInfo> g_dev;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

// Persistent grids on different streams of one device could each hold part
// of the device and wait for workgroups of their own that cannot become
// resident.  Scans issued through the C ABI are therefore ordered across
// streams: a launch on a stream other than the device's previous one first
// waits (on the device, hipStreamWaitEvent) for that previous launch.
// Launches on one stream need nothing, and the request server, which sizes
// its streams' grids to fit side by side, opts out.
// Until a second stream shows up nothing is recorded (one stream is ordered
// by itself); the first switch drains the device once, and from then on an
// event is recorded after every launch.
struct DeviceOrder {
    hipStream_t last = nullptr;
    bool any = false;
    bool multi = false;         // a second stream has been seen: events are recorded
    hipEvent_t done = nullptr;  // recorded after the device's last ordered launch
};
std::map<int, DeviceOrder> g_order;
Params g_params[kNumModes][kNumOpCodes];
Params g_default_params[kNumModes][kNumOpCodes];  // the library's own, before any lscan_set_params
bool g_params_init = false;

// Plain scans of small arrays: the large-array tiles leave most of the
// device idle, and 1024-thread workgroups with fewer vectors per lane
// finish sooner (MI355X, int32 add, device time per launch: 2^16 6.7 against
// 8.3 us, 2^18 7.2 / 8.4, 2^20 8.3 / 9.1, 2^22 11.4 / 12.5).  Shape index
// for an input of `bytes`, or -1 for the large-array default.
int small_array_shape(int64_t bytes)
{
    if (bytes <= (int64_t(512) << 10)) return 6;  // 512 x 2
    if (bytes <= (int64_t(2) << 20)) return 5;    // 1024 x 2
    if (bytes <= (int64_t(32) << 20)) return 4;   // 1024 x 4
    return -1;
}

lscan_status device_error(hipError_t e)
{
    t_last_hip_error = int32_t(e);
    return LSCAN_ERR_DEVICE;
}

bool capturing(hipStream_t stream)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
}

// Defaults measured on MI355X (gfx950) with N = 2^27..2^28 arrays: shape
// index into kShapeThreads/kShapeVectors and workgroups per CU (capped later
// by the occupancy limit and the co-residency test).  With the prefix of
// each block resolved one round late, one large workgroup per CU (B = 256,
// so a window of 255 aggregates) measured best for every type.
void init_params_locked()
{
    if (g_params_init) return;
    // measured on MI355X (shape x groups/CU sweep of the persistent scan).
    // Kernels reading 16-byte vectors prefetch each workgroup's next block into
    // LDS and fold windows copied into LDS a step earlier; with that, one
    // workgroup of 16 waves per CU measured best: 1024 x 4 for 4-byte types
    // (int32 add 2^28: 6.43 TB/s, 512 x 8 the same), 512 x 8 for int64
    // (6.45 TB/s; 256 x 16 two per CU 5.7) and for the compensated sum, whose
    // 1024 x 4 kernel spills (6.0 TB/s against 4.7)
    const Params t512x8g2{1, 2}, t1024x4{4, 1}, t512x8g1{1, 1};
    g_params[kModePlain][kI32Add] = t1024x4;
    g_params[kModePlain][kI32Max] = t1024x4;
    g_params[kModePlain][kI32Min] = t1024x4;
    for (int o = kI64Add; o <= kI64Min; ++o) g_params[kModePlain][o] = t512x8g1;
    g_params[kModePlain][kF32Add] = t1024x4;
    g_params[kModePlain][kF32AddComp] = t512x8g1;
    g_params[kModePlain][kF32Max] = t1024x4;
    g_params[kModePlain][kF32Min] = t1024x4;
    // bf16 prefetches too (two 8-byte rows per 16-byte LDS load): 2^27 elements,
    // add 127 us at 512 x 8 (1024 x 4 131, 256 x 16 two per CU 143), max 129
    // at 1024 x 4, the compensated sum 166 at 512 x 8 (1024 x 4 spills: 197)
    g_params[kModePlain][kBF16Add] = t512x8g1;
    g_params[kModePlain][kBF16AddComp] = t512x8g1;
    g_params[kModePlain][kBF16Max] = t1024x4;
    g_params[kModePlain][kBF16Min] = t1024x4;
    const Params t1024x2{5, 1};
    for (int o = kI32ArgMax; o <= kF32ArgMin; ++o) g_params[kModePlain][o] = t1024x2;
    // the 32-bit-index argmax / argmin kernels prefetch too (int32 keys, 2^28:
    // 256 x 8 two per CU 773 us, 512 x 8 one per CU 677 us)
    for (int o = kI32ArgMaxS; o <= kF32ArgMinS; ++o) g_params[kModePlain][o] = t512x8g1;
    g_params[kModePlain][kI64ArgMaxS] = t1024x4;
    g_params[kModePlain][kI64ArgMinS] = t1024x4;
    for (int o = 0; o < kNumOpCodes; ++o) {
        // with the per-block segment table and (sums) lane-blocked rows; 512 x 8
        // (4096 segments, int32 add: 5.81 TB/s), whose kernels keep their
        // registers where 1024 x 4 spills
        g_params[kModeSegmented][o] = t512x8g1;
        g_params[kModeBatched][o] = g_params[kModePlain][o];
        g_params[kModeCompact][o] = t1024x4;
    }
    // batches of many int32 arrays: smaller blocks than the single-array
    // 256 x 16 (4096 arrays: 4.93 -> 5.10 TB/s as a graph; 64 arrays: same).
    // The float32 batched kernel at 512 x 8 needs 129 VGPRs (one group per
    // CU); 1024 x 4 measures best for it (4096 arrays: 4.72 -> 4.84 TB/s).
    g_params[kModeBatched][kI32Add] = t512x8g2;
    g_params[kModeBatched][kF32Add] = t1024x4;
    g_params[kModeBatched][kI64Add] = t1024x4;  // 4096 arrays: 4.38 -> 4.60 TB/s
    // max / min batches: 512 x 8 fits one group per CU there too (int32 max
    // 4.75 -> 4.83 TB/s, int64 max 3.95 -> 4.37 at 1024 x 4)
    for (int o : {kI32Max, kI32Min, kI64Max, kI64Min, kF32Max, kF32Min}) g_params[kModeBatched][o] = t1024x4;
    // (float32 max 4.39 -> 4.75); bf16 max / min too, since the y stage of
    // arrays at another phase took their 512 x 8 kernel to 129 VGPRs (4096
    // arrays: 1024 x 4 540 us, 256 x 16 two per CU 564 us)
    g_params[kModeBatched][kBF16Max] = t1024x4;
    g_params[kModeBatched][kBF16Min] = t1024x4;
    for (int m = 0; m < kNumModes; ++m)
        for (int o = 0; o < kNumOpCodes; ++o) g_default_params[m][o] = g_params[m][o];
    g_params_init = true;
}

int opcode_of(int dt, int op, uint32_t flags)
{
    const bool comp = (flags & LSCAN_F_COMPENSATED) != 0;
    if (dt < LSCAN_I32 || dt > LSCAN_BF16 || op < LSCAN_ADD || op > LSCAN_ARGMIN) return -1;
    if (comp && !((dt == LSCAN_F32 || dt == LSCAN_BF16) && op == LSCAN_ADD)) return -2;
    if (op == LSCAN_ARGMAX || op == LSCAN_ARGMIN) {
        const int k = (op == LSCAN_ARGMAX) ? 0 : 1;
        switch (dt) {
        case LSCAN_I32: return kI32ArgMax + k;
        case LSCAN_I64: return kI64ArgMax + k;
        case LSCAN_F32: return kF32ArgMax + k;
        default: return -2;  // bf16 keys are not offered
        }
    }
    switch (dt) {
    case LSCAN_I32: return kI32Add + op;
    case LSCAN_I64: return kI64Add + op;
    case LSCAN_F32: return op == LSCAN_ADD ? (comp ? kF32AddComp : kF32Add) : (op == LSCAN_MAX ? kF32Max : kF32Min);
    case LSCAN_BF16: return op == LSCAN_ADD ? (comp ? kBF16AddComp : kBF16Add) : (op == LSCAN_MAX ? kBF16Max : kBF16Min);
    }
    return -1;
}

int in_bytes_of(int dt) { return dt == LSCAN_I64 ? 8 : dt == LSCAN_BF16 ? 2 : 4; }
// output element size; running argmax / argmin write int64 indices
int out_bytes_of(int dt, int op = LSCAN_ADD)
{
    if (op == LSCAN_ARGMAX || op == LSCAN_ARGMIN) return 8;
    return dt == LSCAN_I64 ? 8 : 4;
}
bool is_arg_op(int op) { return op == LSCAN_ARGMAX || op == LSCAN_ARGMIN; }

int shape_index(int threads, int vectors)
{
    for (int s = 0; s < kNumShapes; ++s)
        if (kShapeThreads[s] == threads && kShapeVectors[s] == vectors) return s;
    return -1;
}

// x / y of one array: element alignment, and no overlap other than in place.
lscan_status check_array(const void* x, const void* y, int64_t n, int dt, int op = LSCAN_ADD)
{
    if (n < 0) return LSCAN_ERR_INVALID_ARG;
    if (n == 0) return LSCAN_OK;
    if (!x || !y) return LSCAN_ERR_INVALID_ARG;
    const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    const int ib = in_bytes_of(dt), ob = out_bytes_of(dt, op);
    if (xa % uintptr_t(ib) || ya % uintptr_t(ob)) return LSCAN_ERR_INVALID_ARG;
    if (uint64_t(n) > (UINT64_MAX / 16)) return LSCAN_ERR_INVALID_ARG;
    const uintptr_t xe = xa + uintptr_t(n) * uintptr_t(ib), ye = ya + uintptr_t(n) * uintptr_t(ob);
    const bool overlap = xa < ye && ya < xe;
    if (overlap && !(xa == ya && ib == ob)) return LSCAN_ERR_INVALID_ARG;
    return LSCAN_OK;
}

lscan_status check_params(const lscan_params* p)
{
    if (!p) return LSCAN_OK;
    if ((p->block_threads != 0 || p->vectors_per_lane != 0) &&
        shape_index(p->block_threads, p->vectors_per_lane) < 0)
        return LSCAN_ERR_UNSUPPORTED;
    if (p->groups_per_cu < 0) return LSCAN_ERR_INVALID_ARG;
    if (p->handoff != LSCAN_HANDOFF_WINDOW && p->handoff != LSCAN_HANDOFF_CHAIN) return LSCAN_ERR_INVALID_ARG;
    return LSCAN_OK;
}

// One validated call.
struct Request {
    int mode = kModePlain;
    int oc = 0;
    const void* x = nullptr;
    void* y = nullptr;
    int64_t n = 0;                       // plain/segmented: elements
    const int64_t* offsets = nullptr;
    int64_t num_segments = 0;
    const lscan_array* arrays = nullptr; // batched (host table)
    int64_t num_arrays = 0;
    bool exclusive = false;
    const lscan_params* p = nullptr;
    bool empty = false;                  // nothing to do
    bool ordered = true;                 // order after other streams' launches (not for the server)
    uint32_t* status_host = nullptr;     // optional host-visible timeout word
    const uint8_t* keep = nullptr;       // compaction: keep flags (may be null)
    int64_t* count = nullptr;            // compaction: device count of kept items
    const KernelEntry* custom = nullptr; // a plain scan kernel built for a user operator
};

lscan_status make_request(int mode, const void* x, void* y, int64_t n, const int64_t* offsets, int64_t num_segments,
                          const lscan_array* arrays, int64_t num_arrays, int dt, int op, uint32_t flags,
                          bool exclusive, const lscan_params* p, Request* r)
{
    const uint32_t allowed = LSCAN_F_COMPENSATED | LSCAN_F_DETERMINISTIC |
                             (mode == kModePlain ? LSCAN_F_INDEX64 : LSCAN_F_EXCLUSIVE);
    if (flags & ~allowed) return LSCAN_ERR_INVALID_ARG;
    if ((flags & LSCAN_F_INDEX64) && !is_arg_op(op)) return LSCAN_ERR_INVALID_ARG;
    const int oc = opcode_of(dt, op, flags);
    if (oc == -1) return LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    if (is_arg_op(op) && mode != kModePlain) return LSCAN_ERR_UNSUPPORTED;  // plain scans only
    lscan_status st = check_params(p);
    if (st != LSCAN_OK) return st;
    r->mode = mode;
    // running argmax / argmin of fewer than 2^31 elements: the 32-bit index kernels
    r->oc = (is_arg_op(op) && n <= int64_t(INT32_MAX) && !(flags & LSCAN_F_INDEX64)) ? oc + kArgShortOffset : oc;
    r->exclusive = exclusive;
    r->p = p;
    if (mode == kModeBatched) {
        if (num_arrays < 0 || (num_arrays > 0 && !arrays)) return LSCAN_ERR_INVALID_ARG;
        int64_t total = 0;
        for (int64_t i = 0; i < num_arrays; ++i) {
            st = check_array(arrays[i].x, arrays[i].y, arrays[i].n, dt);
            if (st != LSCAN_OK) return st;
            total += arrays[i].n;
        }
        r->arrays = arrays;
        r->num_arrays = num_arrays;
        r->empty = (total == 0);
        return LSCAN_OK;
    }
    st = check_array(x, y, n, dt, op);
    if (st != LSCAN_OK) return st;
    if (mode == kModeSegmented) {
        if (num_segments < 0) return LSCAN_ERR_INVALID_ARG;
        if (num_segments == 0 && n != 0) return LSCAN_ERR_INVALID_ARG;
        if (num_segments > 0 && !offsets) return LSCAN_ERR_INVALID_ARG;
        if (reinterpret_cast<uintptr_t>(offsets) % 8) return LSCAN_ERR_INVALID_ARG;
    }
    r->x = x;
    r->y = y;
    r->n = n;
    r->offsets = offsets;
    r->num_segments = num_segments;
    r->empty = (n == 0);
    return LSCAN_OK;
}

// Stream compaction: items of 4 (I32, F32) or 8 (I64) bytes, moved as bits;
// the kernel-table row is the add opcode of that width.
int compact_opcode(int dt)
{
    if (dt == LSCAN_I32 || dt == LSCAN_F32) return kI32Add;
    if (dt == LSCAN_I64) return kI64Add;
    return -1;
}

bool ranges_overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes)
{
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + uintptr_t(bbytes) && b0 < a0 + uintptr_t(abytes);
}

lscan_status make_compact_request(const void* x, const uint8_t* keep, void* out, int64_t* count, int64_t n, int dt,
                                  const lscan_params* p, Request* r)
{
    if (dt < LSCAN_I32 || dt > LSCAN_BF16) return LSCAN_ERR_INVALID_ARG;
    const int oc = compact_opcode(dt);
    if (oc < 0) return LSCAN_ERR_UNSUPPORTED;
    if (n < 0 || !count || reinterpret_cast<uintptr_t>(count) % 8) return LSCAN_ERR_INVALID_ARG;
    lscan_status st = check_params(p);
    if (st != LSCAN_OK) return st;
    if (p && p->handoff != LSCAN_HANDOFF_WINDOW) return LSCAN_ERR_UNSUPPORTED;
    st = check_array(x, out, n, dt);
    if (st != LSCAN_OK) return st;
    const int64_t bytes = n * int64_t(in_bytes_of(dt));
    if (n > 0) {
        // kept items move towards the front: out may not share memory with x,
        // the flags or the count
        if (ranges_overlap(x, bytes, out, bytes)) return LSCAN_ERR_INVALID_ARG;
        if (keep && ranges_overlap(keep, n, out, bytes)) return LSCAN_ERR_INVALID_ARG;
        if (ranges_overlap(count, 8, out, bytes)) return LSCAN_ERR_INVALID_ARG;
    }
    r->mode = kModeCompact;
    r->oc = oc;
    r->p = p;
    r->x = x;
    r->y = out;
    r->n = n;
    r->keep = keep;
    r->count = count;
    r->empty = (n == 0);
    return LSCAN_OK;
}

lscan_status device_info_locked(int dev, DeviceInfo** out)
{
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        DeviceInfo info;
        hipError_t e = hipDeviceGetAttribute(&info.cu_count, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return device_error(e);
        int wall_khz = 0;
        e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess || wall_khz <= 0) wall_khz = 100000;  // 100 MHz constant clock
        info.wall_khz = uint64_t(wall_khz);
        info.spin_limit = uint64_t(double(wall_khz) * double(g_watchdog_us) / 1000.0);
        info.residency_limit = uint64_t(double(wall_khz) * 1000.0 * kResidencyWaitSeconds);
        for (int s = 0; s < kNumModes; ++s)
            for (int o = 0; o < kNumOpCodes; ++o)
                for (int h = 0; h < kNumShapes; ++h) {
                    info.occupancy[s][o][h] = -1;
                    info.resident_ok[s][o][h] = 0;
                    info.resident_fail[s][o][h] = 0;
                }
        it = g_dev.emplace(dev, info).first;
    }
    *out = &it->second;
    return LSCAN_OK;
}

void free_workspace(Workspace& ws)
{
    if (ws.slots && !ws.fixed) (void)hipFree(ws.slots);
    if (ws.ctrl && !ws.fixed) (void)hipFree(ws.ctrl);
    if (ws.desc) (void)hipFree(ws.desc);
    if (ws.desc_host) (void)hipHostFree(ws.desc_host);
    if (ws.desc_copied) (void)hipEventDestroy(ws.desc_copied);
    if (ws.seg_first) (void)hipFree(ws.seg_first);
    ws = Workspace();
}

// Make ws hold a segment table of at least `entries` entries.
lscan_status ensure_segment_table(Workspace& ws, hipStream_t stream, size_t entries)
{
    if (ws.seg_cap >= entries) return LSCAN_OK;
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;  // size the workspace with an eager call first
    hipError_t e;
    const size_t old_cap = ws.seg_cap;
    if (ws.seg_first) {
        e = hipStreamSynchronize(stream);  // an earlier scan on this stream may still read it
        if (e != hipSuccess) return device_error(e);
        e = hipFree(ws.seg_first);
        if (e != hipSuccess) return device_error(e);
        ws.seg_first = nullptr;
        ws.seg_cap = 0;
    }
    const size_t cap = std::max<size_t>(entries, std::max<size_t>(2 * old_cap, 1024));
    e = hipMalloc(reinterpret_cast<void**>(&ws.seg_first), cap * sizeof(int64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ws.seg_first = nullptr;
        return LSCAN_ERR_NO_MEMORY;
    }
    ws.seg_cap = cap;
    return LSCAN_OK;
}

// Start a new epoch run on ws before its 32-bit tag could wrap: clear every
// flag word, restart the tag (word 0) and the exit counter (word 1), and
// forget the tag of the last launch that gave up (word 3), which a restarted
// tag could otherwise meet again and read as its own abort.  The timeout
// flag (word 2) is kept for the next check.  Stream-ordered after the
// launches that used the old tags.  The eager path, graph replays and the
// test hooks all reset through here.
lscan_status reset_epoch(Workspace& ws, hipStream_t stream)
{
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;  // never a memset node in a caller's graph
    hipError_t e = hipSuccess;
    if (ws.slots && ws.words) e = hipMemsetAsync(ws.slots, 0, ws.words * sizeof(uint64_t), stream);
    if (e == hipSuccess && ws.ctrl) e = hipMemsetAsync(ws.ctrl, 0, 2 * sizeof(uint32_t), stream);
    if (e == hipSuccess && ws.ctrl) e = hipMemsetAsync(ws.ctrl + 3, 0, sizeof(uint32_t), stream);
    if (e != hipSuccess) return device_error(e);
    ws.launches = 0;
    return LSCAN_OK;
}

// Make ws hold at least `words` flag words and `desc_entries` descriptors.
lscan_status ensure_workspace(Workspace& ws, hipStream_t stream, size_t words, size_t desc_entries)
{
    hipError_t e;
    const bool need_reset = ws.launches >= kMaxLaunchesPerEpochRun;
    const bool grow_slots = ws.words < words || !ws.ctrl;
    const bool grow_desc = ws.desc_cap < desc_entries;
    if (!grow_slots && !grow_desc && !need_reset) return LSCAN_OK;
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;  // size the workspace with an eager call first
    if (ws.fixed) {  // memory the library does not own: never grown or freed
        if (grow_slots || grow_desc) return LSCAN_ERR_NO_MEMORY;
        return reset_epoch(ws, stream);
    }
    if (ws.slots || ws.ctrl || ws.desc) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return device_error(e);
    }
    if (ws.words < words) {
        const size_t alloc = std::max<size_t>(words, std::max<size_t>(ws.words * 2, size_t(1) << 14));
        if (ws.slots) {
            e = hipFree(ws.slots);
            if (e != hipSuccess) return device_error(e);
            ws.slots = nullptr;
            ws.words = 0;
        }
        e = hipMalloc(reinterpret_cast<void**>(&ws.slots), alloc * sizeof(uint64_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return LSCAN_ERR_NO_MEMORY;
        }
        e = hipMemsetAsync(ws.slots, 0, alloc * sizeof(uint64_t), stream);
        if (e != hipSuccess) {  // never keep flag words that were not cleared
            (void)hipFree(ws.slots);
            ws.slots = nullptr;
            return device_error(e);
        }
        ws.words = alloc;
    }
    if (!ws.ctrl) {
        e = hipMalloc(reinterpret_cast<void**>(&ws.ctrl), 64);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return LSCAN_ERR_NO_MEMORY;
        }
        e = hipMemsetAsync(ws.ctrl, 0, 64, stream);
        if (e != hipSuccess) {
            (void)hipFree(ws.ctrl);
            ws.ctrl = nullptr;
            return device_error(e);
        }
    }
    if (need_reset) {
        const lscan_status st = reset_epoch(ws, stream);
        if (st != LSCAN_OK) return st;
    }
    if (grow_desc) {
        const size_t cap = std::max<size_t>(desc_entries, std::max<size_t>(ws.desc_cap * 2, 256));
        if (ws.desc) (void)hipFree(ws.desc);
        if (ws.desc_host) (void)hipHostFree(ws.desc_host);
        ws.desc = nullptr;
        ws.desc_host = nullptr;
        ws.desc_cap = 0;
        ws.desc_pending = false;
        e = hipMalloc(reinterpret_cast<void**>(&ws.desc), cap * sizeof(BatchArray));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return LSCAN_ERR_NO_MEMORY;
        }
        e = hipHostMalloc(reinterpret_cast<void**>(&ws.desc_host), cap * sizeof(BatchArray), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return LSCAN_ERR_NO_MEMORY;
        }
        if (!ws.desc_copied) {
            e = hipEventCreateWithFlags(&ws.desc_copied, hipEventDisableTiming);
            if (e != hipSuccess) return device_error(e);
        }
        ws.desc_cap = cap;
    }
    return LSCAN_OK;
}

lscan_status workspace_locked(int dev, hipStream_t stream, size_t words, size_t desc_entries, Workspace** out)
{
    Workspace& ws = g_ws[std::make_pair(dev, stream)];
    lscan_status st = ensure_workspace(ws, stream, words, desc_entries);
    if (st != LSCAN_OK) return st;
    *out = &ws;
    return LSCAN_OK;
}

// Launch the kernel in its co-residency test mode with `groups` workgroups
// per CU and report whether they were all resident at once.
lscan_status test_residency_locked(const KernelEntry& k, int cu_count, int groups, uint64_t limit,
                                   Workspace* ws, hipStream_t stream, bool* ok)
{
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;  // run one eager call of this shape first
    hipError_t e = hipMemsetAsync(ws->ctrl + 4, 0, 3 * sizeof(uint32_t), stream);
    if (e != hipSuccess) return device_error(e);
    ScanArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ctrl = ws->ctrl;
    a.slots = ws->slots;
    a.spin_limit = limit;
    a.residency_check = 1;
    e = k.launch(a, groups * cu_count, stream);
    if (e != hipSuccess) return device_error(e);
    uint32_t failed = 1;
    e = hipMemcpyAsync(&failed, ws->ctrl + 5, sizeof(failed), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return device_error(e);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e);
    *ok = (failed == 0);
    return LSCAN_OK;
}

// Largest groups-per-CU count <= want whose grid is known (or now tested)
// to be resident at once.
lscan_status resident_groups_core(DeviceInfo* info, const KernelEntry& k, int want, Workspace* ws,
                                  hipStream_t stream, int& good, int& bad, int* out)
{
    int g = want;
    if (bad > 0 && g >= bad) g = bad - 1;
    while (g > good) {
        bool ok = false;
        lscan_status st = test_residency_locked(k, info->cu_count, g, info->residency_limit, ws, stream, &ok);
        if (st != LSCAN_OK) return st;
        if (ok) {
            good = g;
        } else {
            bad = g;
            --g;
        }
    }
    if (g < 1) return LSCAN_ERR_DEVICE;  // not even one workgroup per CU is resident
    *out = g;
    return LSCAN_OK;
}

lscan_status resident_groups_locked(DeviceInfo* info, int mode, int oc, int shape, const KernelEntry& k,
                                    int want, Workspace* ws, hipStream_t stream, int* out)
{
    return resident_groups_core(info, k, want, ws, stream, info->resident_ok[mode][oc][shape],
                                info->resident_fail[mode][oc][shape], out);
}

// Everything needed to enqueue one launch.
struct Plan {
    const KernelEntry* k = nullptr;
    ScanArgs a;
    int grid = 0;
    int groups = 0;
    int occupancy = 0;
};

// Where full tiles of x (and y) can use the kernel's vectors: 0 when x sits
// on a vector boundary and y on 16 bytes; ph > 0 when both sit ph elements
// past such a boundary (the block grid is then shifted back by ph); -1
// otherwise (the element-by-element path).
int64_t alignment_phase(const KernelEntry& k, const void* x, const void* y)
{
    const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    const uintptr_t vec_bytes = uintptr_t(k.in_bytes) * uintptr_t(k.elems_per_vec);
    if (xa % uintptr_t(k.in_bytes) != 0) return -1;
    const uintptr_t ph = (xa % vec_bytes) / uintptr_t(k.in_bytes);
    return ya % 16 == (ph * uintptr_t(k.out_bytes)) % 16 ? int64_t(ph) : -1;
}

// The path of one array of a batch: x's element phase when x is read with
// vectors (-1: the element path).  *stage_y is set when y sits at another
// phase than x, so that rows read as vectors are written through the LDS
// stage; that needs 16-byte output vectors, else the array takes the element
// path.
int64_t batch_phase(const KernelEntry& k, const lscan_array& arr, bool* stage_y)
{
    *stage_y = false;
    const int64_t ph = alignment_phase(k, arr.x, arr.y);
    if (ph >= 0) return ph;
    const uintptr_t xa = reinterpret_cast<uintptr_t>(arr.x), ya = reinterpret_cast<uintptr_t>(arr.y);
    const uintptr_t vec_bytes = uintptr_t(k.in_bytes) * uintptr_t(k.elems_per_vec);
    if (xa % uintptr_t(k.in_bytes) != 0 || ya % uintptr_t(k.out_bytes) != 0 ||
        k.out_bytes * k.elems_per_vec != 16)
        return -1;
    *stage_y = true;
    return int64_t((xa % vec_bytes) / uintptr_t(k.in_bytes));
}

// Blocks of one array of a batch: its n elements after its alignment phase.
int64_t batch_blocks(const KernelEntry& k, const lscan_array& arr, int64_t L)
{
    if (arr.n <= 0) return 0;
    bool stage_y;
    return (arr.n + std::max<int64_t>(batch_phase(k, arr, &stage_y), 0) + L - 1) / L;
}

// Choose the kernel and grid, size the workspace, run the co-residency test
// if this shape is new, upload batched descriptors, and fill the kernel
// arguments.  Called with g_mu held.  ws_fixed is a workspace owned by a
// graph, or null for the per-stream one.
// The parameters a request runs with: the caller's, else the operator's;
// plain add / max / min scans of small arrays take the small-array tiles
// while the operator's parameters are the library's own.  Host data only
// (no HIP call).  Called with g_mu held.
Params choose_params_locked(const Request& r)
{
    init_params_locked();
    Params prm = r.custom ? Params{0, kCustomGroupsPerCu, LSCAN_HANDOFF_WINDOW} : g_params[r.mode][r.oc];
    const Params& dflt = g_default_params[r.mode][r.oc];
    const bool library_default = prm.shape == dflt.shape && prm.groups_per_cu == dflt.groups_per_cu &&
                                 prm.handoff == dflt.handoff;
    if (!r.custom && r.mode == kModePlain && r.oc < kI32ArgMax && library_default) {
        const int s = small_array_shape(r.n * int64_t(table()[r.mode][r.oc][prm.shape].in_bytes));
        if (s >= 0) {
            prm.shape = s;
            prm.groups_per_cu = 2;
        }
    }
    if (!r.custom && r.p && (r.p->block_threads != 0 || r.p->vectors_per_lane != 0))
        prm.shape = shape_index(r.p->block_threads, r.p->vectors_per_lane);
    if (r.p && r.p->groups_per_cu > 0) prm.groups_per_cu = r.p->groups_per_cu;
    if (r.p) prm.handoff = r.p->handoff;
    return prm;
}

lscan_status plan_locked(const Request& r, int dev, Workspace* ws_fixed, hipStream_t stream, Plan* plan,
                         Workspace** ws_used)
{
    const Params prm = choose_params_locked(r);
    const KernelEntry& k = r.custom ? *r.custom : table()[r.mode][r.oc][prm.shape];
    if (!k.func) return LSCAN_ERR_UNSUPPORTED;  // no kernel of this kind for the operator

    DeviceInfo* info = nullptr;
    lscan_status st = device_info_locked(dev, &info);
    if (st != LSCAN_OK) return st;
    DeviceInfo::Custom* cu = r.custom ? &info->custom[k.func] : nullptr;
    int& occ = cu ? cu->occupancy : info->occupancy[r.mode][r.oc][prm.shape];
    if (occ < 0) {
        int v = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k.func, k.block_threads, 0);
        if (e != hipSuccess) return device_error(e);
        occ = v;
    }
    if (occ <= 0) return LSCAN_ERR_UNSUPPORTED;

    // Plain, segmented and batched scans whose x sits `phase` elements past a vector
    // boundary, with y at the same element phase, shift the block grid back
    // by `phase`: the vector accesses of every full tile are then aligned
    // again, and the blocks cover n + phase positions, the first `phase` of
    // them empty.
    // When y sits at another phase than x, the grid follows x: full blocks
    // still read vectors and write y through an LDS stage.
    int32_t phase = 0;
    bool vec_ok = false, store_vec = false;
    if (r.mode == kModePlain || r.mode == kModeSegmented) {
        const uintptr_t xa = reinterpret_cast<uintptr_t>(r.x);
        const uintptr_t vec_bytes = uintptr_t(k.in_bytes) * uintptr_t(k.elems_per_vec);
        if (xa % uintptr_t(k.in_bytes) == 0) {
            phase = int32_t((xa % vec_bytes) / uintptr_t(k.in_bytes));
            vec_ok = true;
            store_vec = alignment_phase(k, r.x, r.y) >= 0;
        }
    }

    const int64_t L = k.tile_elems;
    int64_t M = 0;
    if (r.mode == kModeBatched) {
        for (int64_t i = 0; i < r.num_arrays; ++i) M += batch_blocks(k, r.arrays[i], L);
    } else {
        M = (r.n + phase + L - 1) / L;
    }
    const size_t desc_entries = (r.mode == kModeBatched) ? size_t(r.num_arrays) + 1 : 0;

    Workspace* ws = ws_fixed;
    if (ws) {
        st = ensure_workspace(*ws, stream, size_t(M) * size_t(k.slot_words), desc_entries);
    } else {
        st = workspace_locked(dev, stream, size_t(M) * size_t(k.slot_words), desc_entries, &ws);
    }
    if (st != LSCAN_OK) return st;

    // The grid must fit on the device at once: cap by the occupancy limit,
    // then by what the co-residency test has shown (a grid no larger than M
    // needs only the groups that M blocks fill).
    int want = std::min<int>(prm.groups_per_cu, occ);
    const int64_t need = (M + info->cu_count - 1) / info->cu_count;
    if (need < want) want = int(need);
    int groups = 0;
    if (cu)
        st = resident_groups_core(info, k, want, ws, stream, cu->ok, cu->fail, &groups);
    else
        st = resident_groups_locked(info, r.mode, r.oc, prm.shape, k, want, ws, stream, &groups);
    if (st != LSCAN_OK) return st;
    const int64_t B = std::max<int64_t>(1, std::min<int64_t>(M, int64_t(groups) * info->cu_count));

    ScanArgs& a = plan->a;
    std::memset(&a, 0, sizeof(a));
    if (r.mode == kModeBatched) {
        if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;  // descriptors are uploaded eagerly
        hipError_t e;
        if (ws->desc_pending) {  // the previous upload must have left the staging buffer
            e = hipEventSynchronize(ws->desc_copied);
            if (e != hipSuccess) return device_error(e);
            ws->desc_pending = false;
        }
        int64_t first = 0;
        for (int64_t i = 0; i < r.num_arrays; ++i) {
            ws->desc_host[i].x = r.arrays[i].x;
            ws->desc_host[i].y = r.arrays[i].y;
            ws->desc_host[i].n = r.arrays[i].n;
            ws->desc_host[i].first_block = first;
            bool stage_y = false;
            ws->desc_host[i].phase = batch_phase(k, r.arrays[i], &stage_y);
            ws->desc_host[i].stage_y = stage_y ? 1 : 0;
            first += batch_blocks(k, r.arrays[i], L);
        }
        ws->desc_host[r.num_arrays] = BatchArray{nullptr, nullptr, 0, first, 0, 0};
        e = hipMemcpyAsync(ws->desc, ws->desc_host, desc_entries * sizeof(BatchArray), hipMemcpyHostToDevice,
                           stream);
        if (e != hipSuccess) return device_error(e);
        e = hipEventRecord(ws->desc_copied, stream);
        if (e != hipSuccess) return device_error(e);
        ws->desc_pending = true;
        a.arrays = ws->desc;
        a.num_arrays = r.num_arrays;
        a.vec_ok = 1;  // decided per array in the kernel
    } else if (r.mode == kModeCompact) {
        // full tiles read 16-byte item vectors and 16-byte flag chunks
        a.x = r.x;
        a.y = r.y;
        a.n = r.n;
        a.keep = r.keep;
        a.count = r.count;
        a.vec_ok = (reinterpret_cast<uintptr_t>(r.x) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(r.keep) % 16 == 0) ? 1 : 0;
    } else {
        a.x = r.x;
        a.y = r.y;
        a.n = r.n;
        a.offsets = r.offsets;
        a.num_segments = r.num_segments;
        a.vec_ok = vec_ok ? 1 : 0;
        a.phase = phase;
        a.store_vec = store_vec ? 1 : 0;
        if (r.mode == kModeSegmented) {  // the first segment of every block, written before the scan
            st = ensure_segment_table(*ws, stream, size_t(M) + 1);
            if (st != LSCAN_OK) return st;
            a.seg_first = ws->seg_first;
        }
    }
    a.num_blocks = M;
    a.slots = ws->slots;
    a.ctrl = ws->ctrl;
    a.spin_limit = info->spin_limit;
    a.exclusive = r.exclusive ? 1 : 0;
    a.chain = (r.mode != kModeCompact && prm.handoff == LSCAN_HANDOFF_CHAIN) ? 1 : 0;
    a.residency_check = 0;
    a.status_host = r.status_host;

    plan->k = &k;
    plan->grid = int(B);
    plan->groups = groups;
    plan->occupancy = occ;
    if (ws_used) *ws_used = ws;

    int64_t total = r.n;
    if (r.mode == kModeBatched) {
        total = 0;
        for (int64_t i = 0; i < r.num_arrays; ++i) total += r.arrays[i].n;
    }
    t_last_launch.n = total;
    t_last_launch.num_blocks = M;
    t_last_launch.tile_elems = L;
    t_last_launch.grid = int32_t(B);
    t_last_launch.block_threads = k.block_threads;
    t_last_launch.slot_words = k.slot_words;
    // 1: vectors both ways; 2: vector reads, element writes; 0: elements
    const bool split = (r.mode == kModePlain || r.mode == kModeSegmented) && !a.store_vec;
    t_last_launch.vector_path = a.vec_ok ? (split ? 2 : 1) : 0;
    t_last_launch.groups_per_cu = groups;
    t_last_launch.occupancy = occ;
    return LSCAN_OK;
}

// Cross-stream ordering of one persistent launch on `stream` (see
// DeviceOrder); *out receives the device's record, to be passed to
// order_after_locked once the launch is enqueued.  Called with g_mu held,
// never on a capturing stream (both callers refuse capture first).
lscan_status order_before_locked(int dev, hipStream_t stream, DeviceOrder** out)
{
    DeviceOrder* order = &g_order[dev];
    hipError_t e = hipSuccess;
    if (order->any && order->last != stream) {  // before the co-residency test, too
        if (!order->multi) {
            if (!order->done) {
                e = hipEventCreateWithFlags(&order->done, hipEventDisableTiming);
                if (e != hipSuccess) {
                    order->done = nullptr;
                    return device_error(e);
                }
            }
            e = hipDeviceSynchronize();  // once: the previous stream's launches have no event
            order->multi = true;
        } else {
            e = hipStreamWaitEvent(stream, order->done, 0);
        }
        if (e != hipSuccess) return device_error(e);
    }
    order->any = true;
    order->last = stream;
    *out = order;
    return LSCAN_OK;
}

lscan_status order_after_locked(DeviceOrder* order, hipStream_t stream)
{
    if (order && order->multi) {
        const hipError_t e = hipEventRecord(order->done, stream);
        if (e != hipSuccess) return device_error(e);
    }
    return LSCAN_OK;
}

// ---------------------------------------------------------------------------
// Flag memory that needs no allocation (lscan_inclusive_noalloc)
// ---------------------------------------------------------------------------

// Control words (the first 256 bytes) and flag slots of the scans that
// lscan_inclusive_noalloc launches.  Every GPU holds its own copy of this
// array for as long as the library is loaded.  In host code `scratch` names
// only a host-side stand-in: its device address on a device comes from
// hipGetSymbolAddress with that device current, and only that address is
// ever handed to HIP (kernel arguments, memsets, copies).
constexpr size_t kNoAllocCtrlWords = 32;               // 256 bytes; the kernels use 7 32-bit words
constexpr size_t kNoAllocSlotWords = size_t(1) << 19;  // 4 MiB of 64-bit flag words
static __device__ __align__(256) uint64_t scratch[kNoAllocCtrlWords + kNoAllocSlotWords];

constexpr int kMaxNoAllocDevices = 64;
// The fixed workspace of each device, set up by its first call (scratch
// address, cleared once); null until then.
Workspace g_noalloc_ws[kMaxNoAllocDevices];
bool g_noalloc_ready[kMaxNoAllocDevices] = {};

// Set up the fixed workspace of device `dev` (current) on its first call:
// look up this device's copy of `scratch` and clear it on the stream.  The
// stream is not capturing (the caller checked).  Called with g_mu held.
lscan_status noalloc_workspace_locked(int dev, hipStream_t stream, Workspace** out)
{
    if (dev < 0 || dev >= kMaxNoAllocDevices) return LSCAN_ERR_UNSUPPORTED;
    Workspace& ws = g_noalloc_ws[dev];
    if (!g_noalloc_ready[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return device_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
        e = hipMemsetAsync(ptr, 0, sizeof(scratch), stream);
        if (e != hipSuccess) return device_error(e);
        ws = Workspace();
        ws.fixed = true;
        ws.ctrl = static_cast<uint32_t*>(ptr);
        ws.slots = static_cast<uint64_t*>(ptr) + kNoAllocCtrlWords;
        ws.words = kNoAllocSlotWords;
        g_noalloc_ready[dev] = true;
    }
    *out = &ws;
    return LSCAN_OK;
}

// Whether the flag words of request r fit the fixed workspace, decided from
// host data before any device work: M blocks of the kernel r would run
// (counting the largest alignment shift of the block grid) times its flag
// words per block.  Called with g_mu held.
bool noalloc_fits_locked(const Request& r)
{
    const Params prm = choose_params_locked(r);
    const KernelEntry& k = table()[r.mode][r.oc][prm.shape];
    if (!k.func) return true;  // refused later as unsupported
    const int64_t M = (r.n + k.elems_per_vec + k.tile_elems - 1) / k.tile_elems;
    return uint64_t(M) * uint64_t(k.slot_words) <= kNoAllocSlotWords;
}

lscan_status run(const Request& r, void* stream_ptr)
{
    if (r.empty) return LSCAN_OK;
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    // A captured kernel node would hold the per-stream workspace's raw
    // pointers, which a later call may free (a larger workspace, or
    // lscan_release_workspaces), and its replays would bypass the host's
    // epoch count.  Captured scans go through lscan_graph_create_*, whose
    // graphs own their workspace.
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceOrder* order = nullptr;
    lscan_status st = LSCAN_OK;
    if (r.ordered) {
        st = order_before_locked(dev, stream, &order);
        if (st != LSCAN_OK) return st;
    }
    Plan plan;
    Workspace* ws = nullptr;
    st = plan_locked(r, dev, nullptr, stream, &plan, &ws);
    if (st != LSCAN_OK) return st;
    if (plan.a.seg_first) {
        e = launch_segment_table(plan.a, plan.k->tile_elems, stream);
        if (e != hipSuccess) return device_error(e);
    }
    e = plan.k->launch(plan.a, plan.grid, stream);
    if (e != hipSuccess) return device_error(e);
    ws->launches++;
    return order_after_locked(order, stream);
}

// One plain scan on the device's fixed workspace: no allocation of any kind
// on the device (the co-residency test of a new shape runs once, eagerly, on
// the same fixed words).  Not ordered after other streams' scans.
lscan_status run_noalloc(const Request& r, void* stream_ptr)
{
    if (r.empty) return LSCAN_OK;
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!noalloc_fits_locked(r)) return LSCAN_ERR_NO_MEMORY;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace* ws = nullptr;
    lscan_status st = noalloc_workspace_locked(dev, stream, &ws);
    if (st != LSCAN_OK) return st;
    Plan plan;
    st = plan_locked(r, dev, ws, stream, &plan, nullptr);
    if (st != LSCAN_OK) return st;
    e = plan.k->launch(plan.a, plan.grid, stream);
    if (e != hipSuccess) return device_error(e);
    ws->launches++;
    return LSCAN_OK;
}

// ---------------------------------------------------------------------------
// Breadth-first search (bfs_kernel.hip)
// ---------------------------------------------------------------------------

// Device state of the search on one stream, in one allocation: the flag
// region (per-chunk words, per-workgroup arrival words, the release word and
// the abort word; zero when allocated), per-workgroup counters, the claim
// words and the two frontier queues, sized for the largest graph seen.
struct BfsWorkspace {
    char* mem = nullptr;
    int64_t cap_v = 0;
    int64_t cap_chunks = 0;  // entries of each chunk table
    int cap_grid = 0;
    size_t flag_bytes = 0;
    uint64_t* slots = nullptr;
    uint64_t* arrive = nullptr;
    uint64_t* go = nullptr;
    uint32_t* abort_word = nullptr;
    int64_t* partial = nullptr;
    uint32_t* visited = nullptr;
    int64_t* edge_off[2] = {nullptr, nullptr};
    int64_t* edge_shift[2] = {nullptr, nullptr};
    int32_t* queue[2] = {nullptr, nullptr};
    int32_t* chunk_first[2] = {nullptr, nullptr};
    uint64_t next_tag = 0;  // the next launch's tags start above this
};
std::map<std::pair<int, hipStream_t>, BfsWorkspace> g_bfs_ws;

// Workgroups per CU the search asks for (the occupancy limit and the
// co-residency test may lower it).
constexpr int kBfsGroupsPerCu = 4;

void free_bfs_workspace(BfsWorkspace& ws)
{
    if (ws.mem) (void)hipFree(ws.mem);
    ws = BfsWorkspace();
}

lscan_status ensure_bfs_workspace(BfsWorkspace& ws, hipStream_t stream, int64_t nv, int64_t chunks, int grid)
{
    if (ws.mem && ws.cap_v >= nv && ws.cap_chunks >= chunks && ws.cap_grid >= grid) return LSCAN_OK;
    hipError_t e;
    if (ws.mem) {
        e = hipStreamSynchronize(stream);  // earlier searches on this stream still use it
        if (e != hipSuccess) return device_error(e);
        nv = std::max(nv, ws.cap_v);
        chunks = std::max(chunks, ws.cap_chunks);
        grid = std::max(grid, ws.cap_grid);
        free_bfs_workspace(ws);
    }
    // flag region first (zeroed), then 8-byte arrays, then 4-byte arrays
    const size_t flag_words = 2 * size_t(chunks) + 4 * size_t(grid) + 4 + 1;
    const size_t bytes = flag_words * 8 + size_t(grid) * 8 + size_t(nv) * 8 * 4 + size_t(nv) * 4 * 2 +
                         size_t(chunks) * 4 * 2 + size_t((nv + 31) / 32) * 4;
    e = hipMalloc(reinterpret_cast<void**>(&ws.mem), bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ws.mem = nullptr;
        return LSCAN_ERR_NO_MEMORY;
    }
    uint64_t* w = reinterpret_cast<uint64_t*>(ws.mem);
    ws.slots = w;
    ws.arrive = ws.slots + 2 * chunks;
    ws.go = ws.arrive + 4 * size_t(grid);
    ws.abort_word = reinterpret_cast<uint32_t*>(ws.go + 4);
    ws.flag_bytes = flag_words * 8;
    ws.partial = reinterpret_cast<int64_t*>(w + flag_words);
    ws.edge_off[0] = ws.partial + grid;
    ws.edge_off[1] = ws.edge_off[0] + nv;
    ws.edge_shift[0] = ws.edge_off[1] + nv;
    ws.edge_shift[1] = ws.edge_shift[0] + nv;
    ws.queue[0] = reinterpret_cast<int32_t*>(ws.edge_shift[1] + nv);
    ws.queue[1] = ws.queue[0] + nv;
    ws.chunk_first[0] = ws.queue[1] + nv;
    ws.chunk_first[1] = ws.chunk_first[0] + chunks;
    ws.visited = reinterpret_cast<uint32_t*>(ws.chunk_first[1] + chunks);
    ws.cap_v = nv;
    ws.cap_chunks = chunks;
    ws.cap_grid = grid;
    ws.next_tag = 0;
    e = hipMemsetAsync(ws.mem, 0, ws.flag_bytes, stream);
    if (e != hipSuccess) {  // never keep flag words that were not cleared
        free_bfs_workspace(ws);
        return device_error(e);
    }
    return LSCAN_OK;
}

// Co-residency test of the search kernel through the scan's test driver.
hipError_t bfs_residency_launch(const ScanArgs& sa, int grid, hipStream_t stream)
{
    BfsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ctrl = sa.ctrl;
    a.spin_limit = sa.spin_limit;
    a.residency_check = 1;
    return launch_bfs(a, grid, stream);
}

lscan_status bfs_run(const int64_t* row, const int32_t* col, int64_t nv, int64_t ne, int32_t src, int32_t* level,
                     int32_t* parent, int64_t* stats, const lscan_params* p, hipStream_t stream)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    if (capturing(stream)) return LSCAN_ERR_UNSUPPORTED;  // each launch takes fresh tags from the host
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceOrder* order = nullptr;
    lscan_status st = order_before_locked(dev, stream, &order);
    if (st != LSCAN_OK) return st;
    DeviceInfo* info = nullptr;
    st = device_info_locked(dev, &info);
    if (st != LSCAN_OK) return st;
    if (info->bfs_occupancy < 0) {
        int v = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, bfs_kernel_func(), kBfsThreads, 0);
        if (e != hipSuccess) return device_error(e);
        info->bfs_occupancy = v;
    }
    if (info->bfs_occupancy <= 0) return LSCAN_ERR_UNSUPPORTED;
    Workspace* ws = nullptr;
    st = workspace_locked(dev, stream, 64, 0, &ws);  // the stream's control words (timeout flag)
    if (st != LSCAN_OK) return st;
    int want = (p && p->groups_per_cu > 0) ? p->groups_per_cu : kBfsGroupsPerCu;
    want = std::min(want, info->bfs_occupancy);
    KernelEntry k;
    std::memset(&k, 0, sizeof(k));
    k.func = bfs_kernel_func();
    k.launch = bfs_residency_launch;
    k.block_threads = kBfsThreads;
    int groups = 0;
    st = resident_groups_core(info, k, want, ws, stream, info->bfs_resident_ok, info->bfs_resident_fail, &groups);
    if (st != LSCAN_OK) return st;
    // no more workgroups than the edges of the largest level can keep busy
    const int64_t chunks = (ne + kBfsChunkEdges - 1) / kBfsChunkEdges + 1;
    const int grid = int(std::max<int64_t>(
        1, std::min<int64_t>({int64_t(groups) * info->cu_count, chunks, int64_t(kBfsMaxGrid)})));

    BfsWorkspace& bw = g_bfs_ws[std::make_pair(dev, stream)];
    st = ensure_bfs_workspace(bw, stream, nv, chunks, grid);
    if (st != LSCAN_OK) return st;
    // tags base + 1 .. base + nv + 2: the start barrier and at most nv levels
    const uint64_t need = uint64_t(nv) + 3;
    if (bw.next_tag + need >= uint64_t(UINT32_MAX)) {
        e = hipMemsetAsync(bw.mem, 0, bw.flag_bytes, stream);
        if (e != hipSuccess) return device_error(e);
        bw.next_tag = 0;
    }
    BfsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row = row;
    a.col = col;
    a.nv = nv;
    a.ne = ne;
    a.src = src;
    a.level = level;
    a.parent = parent;
    a.stats = stats;
    a.visited = bw.visited;
    for (int k = 0; k < 2; ++k) {
        a.queue[k] = bw.queue[k];
        a.edge_off[k] = bw.edge_off[k];
        a.edge_shift[k] = bw.edge_shift[k];
        a.chunk_first[k] = bw.chunk_first[k];
    }
    a.chunk_cap = bw.cap_chunks;
    a.slots = bw.slots;
    a.arrive = bw.arrive;
    a.partial = bw.partial;
    a.go = bw.go;
    a.abort_word = bw.abort_word;
    a.timeout_flag = ws->ctrl + 2;
    a.ctrl = ws->ctrl;
    a.spin_limit = info->spin_limit;
    a.base_tag = uint32_t(bw.next_tag);
    a.residency_check = 0;
    bw.next_tag += need;
    e = launch_bfs(a, grid, stream);
    if (e != hipSuccess) return device_error(e);

    t_last_launch = lscan_launch_info{};
    t_last_launch.n = nv;
    t_last_launch.num_blocks = chunks;
    t_last_launch.tile_elems = kBfsChunkEdges;
    t_last_launch.grid = grid;
    t_last_launch.block_threads = kBfsThreads;
    t_last_launch.slot_words = 1;
    t_last_launch.vector_path = 0;
    t_last_launch.groups_per_cu = groups;
    t_last_launch.occupancy = info->bfs_occupancy;
    return order_after_locked(order, stream);
}

}  // namespace

lscan_status validate_request(const void* x, const void* y, int64_t n, int dt, int op, uint32_t flags)
{
    if (flags & ~(LSCAN_F_COMPENSATED | LSCAN_F_DETERMINISTIC | LSCAN_F_EXCLUSIVE)) return LSCAN_ERR_INVALID_ARG;
    const int oc = opcode_of(dt, op, flags);
    if (oc == -1) return LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    if (is_arg_op(op)) return LSCAN_ERR_UNSUPPORTED;  // the server batches add / max / min scans
    return check_array(x, y, n, dt);
}

uint64_t request_bytes(int64_t n, int dt) { return uint64_t(n) * uint64_t(in_bytes_of(dt) + out_bytes_of(dt)); }

int kernel_vgprs(bool batched, int dt, int op, uint32_t flags, int threads, int vectors)
{
    const int oc = opcode_of(dt, op, flags & LSCAN_F_COMPENSATED);
    const int sh = shape_index(threads, vectors);
    if (oc < 0 || sh < 0) return -1;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, table()[batched ? kModeBatched : kModePlain][oc][sh].func) != hipSuccess)
        return -1;
    return attr.numRegs;
}

lscan_status launch_single(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                           const lscan_params* p, void* stream, uint32_t* status_host)
{
    Request r;
    lscan_status st = make_request(kModePlain, x, y, n, nullptr, 0, nullptr, 0, dt, op, flags & LSCAN_F_COMPENSATED,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, p, &r);
    if (st != LSCAN_OK) return st;
    r.status_host = status_host;
    r.ordered = false;
    return run(r, stream);
}

lscan_status launch_batched(const lscan_array* arrays, int64_t count, lscan_dtype dt, lscan_op op, uint32_t flags,
                            const lscan_params* p, void* stream, uint32_t* status_host)
{
    Request r;
    lscan_status st = make_request(kModeBatched, nullptr, nullptr, 0, nullptr, 0, arrays, count, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, p, &r);
    if (st != LSCAN_OK) return st;
    r.status_host = status_host;
    r.ordered = false;
    return run(r, stream);
}

}  // namespace lscan

using namespace lscan;

// A captured launch with its own workspace (so graph replays never share
// flags with eager launches).
struct lscan_graph {
    int dev = 0;
    hipStream_t prep = nullptr;
    Workspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

lscan_status graph_create(const Request& r, lscan_graph** out)
{
    if (!out) return LSCAN_ERR_INVALID_ARG;
    *out = nullptr;
    if (r.empty) return LSCAN_ERR_INVALID_ARG;  // nothing to capture
    lscan_graph* g = new (std::nothrow) lscan_graph();
    if (!g) return LSCAN_ERR_NO_MEMORY;
    auto fail = [&](lscan_status st) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->prep) (void)hipStreamSynchronize(g->prep);
        free_workspace(g->ws);
        if (g->prep) (void)hipStreamDestroy(g->prep);
        delete g;
        return st;
    };
    hipError_t e = hipGetDevice(&g->dev);
    if (e != hipSuccess) return fail(device_error(e));
    e = hipStreamCreateWithFlags(&g->prep, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(device_error(e));
    Plan plan;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        lscan_status st = plan_locked(r, g->dev, &g->ws, g->prep, &plan, nullptr);
        if (st != LSCAN_OK) return fail(st);
    }
    e = hipStreamSynchronize(g->prep);  // workspace zeroed, descriptors uploaded, residency known
    if (e != hipSuccess) return fail(device_error(e));
    e = hipStreamBeginCapture(g->prep, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(device_error(e));
    if (plan.a.seg_first) e = launch_segment_table(plan.a, plan.k->tile_elems, g->prep);  // part of every replay
    if (e == hipSuccess) e = plan.k->launch(plan.a, plan.grid, g->prep);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(g->prep, &graph);
    g->graph = graph;
    if (e != hipSuccess) return fail(device_error(e));
    if (e2 != hipSuccess) return fail(device_error(e2));
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(device_error(e));
    *out = g;
    return LSCAN_OK;
}

}  // namespace

extern "C" {

lscan_status lscan_inclusive(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                             void* stream)
{
    Request r;
    lscan_status st = make_request(kModePlain, x, y, n, nullptr, 0, nullptr, 0, dt, op, flags, false, nullptr, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_exclusive(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                             void* stream)
{
    Request r;
    lscan_status st = make_request(kModePlain, x, y, n, nullptr, 0, nullptr, 0, dt, op, flags, true, nullptr, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_inclusive_noalloc(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op,
                                     uint32_t flags, void* stream)
{
    Request r;
    lscan_status st = make_request(kModePlain, x, y, n, nullptr, 0, nullptr, 0, dt, op, flags, false, nullptr, &r);
    return st != LSCAN_OK ? st : run_noalloc(r, stream);
}

lscan_status lscan_segmented(const void* x, void* y, int64_t n_total, const int64_t* offsets,
                             int64_t num_segments, lscan_dtype dt, lscan_op op, uint32_t flags, void* stream)
{
    Request r;
    lscan_status st = make_request(kModeSegmented, x, y, n_total, offsets, num_segments, nullptr, 0, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, nullptr, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_batched(const lscan_array* arrays, int64_t count, lscan_dtype dt, lscan_op op, uint32_t flags,
                           void* stream)
{
    Request r;
    lscan_status st = make_request(kModeBatched, nullptr, nullptr, 0, nullptr, 0, arrays, count, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, nullptr, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_scan_with_params(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op,
                                    uint32_t flags, int32_t exclusive, const lscan_params* p, void* stream)
{
    Request r;
    lscan_status st = make_request(kModePlain, x, y, n, nullptr, 0, nullptr, 0, dt, op, flags, exclusive != 0, p, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_segmented_with_params(const void* x, void* y, int64_t n_total, const int64_t* offsets,
                                         int64_t num_segments, lscan_dtype dt, lscan_op op, uint32_t flags,
                                         const lscan_params* p, void* stream)
{
    Request r;
    lscan_status st = make_request(kModeSegmented, x, y, n_total, offsets, num_segments, nullptr, 0, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, p, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_batched_with_params(const lscan_array* arrays, int64_t count, lscan_dtype dt, lscan_op op,
                                       uint32_t flags, const lscan_params* p, void* stream)
{
    Request r;
    lscan_status st = make_request(kModeBatched, nullptr, nullptr, 0, nullptr, 0, arrays, count, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, p, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_graph_create_scan(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                                     const lscan_params* p, lscan_graph** out)
{
    Request r;
    const bool exclusive = (flags & LSCAN_F_EXCLUSIVE) != 0;
    lscan_status st = make_request(kModePlain, x, y, n, nullptr, 0, nullptr, 0, dt, op, flags & ~LSCAN_F_EXCLUSIVE,
                                   exclusive, p, &r);
    return st != LSCAN_OK ? st : graph_create(r, out);
}

lscan_status lscan_graph_create_segmented(const void* x, void* y, int64_t n_total, const int64_t* offsets,
                                          int64_t num_segments, lscan_dtype dt, lscan_op op, uint32_t flags,
                                          const lscan_params* p, lscan_graph** out)
{
    Request r;
    lscan_status st = make_request(kModeSegmented, x, y, n_total, offsets, num_segments, nullptr, 0, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, p, &r);
    return st != LSCAN_OK ? st : graph_create(r, out);
}

lscan_status lscan_graph_create_batched(const lscan_array* arrays, int64_t count, lscan_dtype dt, lscan_op op,
                                        uint32_t flags, const lscan_params* p, lscan_graph** out)
{
    Request r;
    lscan_status st = make_request(kModeBatched, nullptr, nullptr, 0, nullptr, 0, arrays, count, dt, op, flags,
                                   (flags & LSCAN_F_EXCLUSIVE) != 0, p, &r);
    return st != LSCAN_OK ? st : graph_create(r, out);
}

lscan_status lscan_graph_launch(lscan_graph* g, void* stream_ptr)
{
    if (!g || !g->exec) return LSCAN_ERR_INVALID_ARG;
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    if (g->ws.launches >= kMaxLaunchesPerEpochRun) {
        const lscan_status st = reset_epoch(g->ws, stream);
        if (st != LSCAN_OK) return st;
    }
    const hipError_t e = hipGraphLaunch(g->exec, stream);
    if (e != hipSuccess) return device_error(e);
    g->ws.launches++;
    return LSCAN_OK;
}

lscan_status lscan_graph_check(lscan_graph* g, void* stream_ptr)
{
    if (!g) return LSCAN_ERR_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream_ptr));
    if (e != hipSuccess) return device_error(e);
    uint32_t flag = 0;
    e = hipMemcpy(&flag, g->ws.ctrl + 2, sizeof(flag), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_error(e);
    if (flag) {
        const uint32_t zero = 0;
        e = hipMemcpy(g->ws.ctrl + 2, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (e != hipSuccess) return device_error(e);
        return LSCAN_ERR_TIMEOUT;
    }
    return LSCAN_OK;
}

lscan_status lscan_graph_destroy(lscan_graph* g)
{
    if (!g) return LSCAN_ERR_INVALID_ARG;
    hipError_t e = hipDeviceSynchronize();  // no replay may still use the workspace
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    free_workspace(g->ws);
    if (g->prep) (void)hipStreamDestroy(g->prep);
    delete g;
    return e == hipSuccess ? LSCAN_OK : device_error(e);
}

// ---------------------------------------------------------------------------
// Test hooks (include/lscan_testing.h)
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

// Seed ws after the work that used it has finished: all flag words cleared,
// the tag and launch count set, the exit counter zeroed.
lscan_status seed_epoch(Workspace& ws, uint64_t launches, uint32_t tag, uint32_t abort_tag)
{
    if (!ws.ctrl || !ws.slots) return LSCAN_ERR_NOT_FOUND;
    if (launches > kMaxLaunchesPerEpochRun) return LSCAN_ERR_INVALID_ARG;
    if (uint64_t(tag) + (kMaxLaunchesPerEpochRun - launches) + 1 >= uint64_t(UINT32_MAX)) return LSCAN_ERR_INVALID_ARG;
    hipError_t e = hipMemset(ws.slots, 0, ws.words * sizeof(uint64_t));
    const uint32_t words[2] = {tag, 0u};
    if (e == hipSuccess) e = hipMemcpy(ws.ctrl, words, sizeof(words), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ws.ctrl + 3, &abort_tag, sizeof(abort_tag), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return device_error(e);
    ws.launches = launches;
    return LSCAN_OK;
}

lscan_status epoch_state(const Workspace& ws, uint64_t* launches, uint32_t* ctrl)
{
    if (!launches || !ctrl) return LSCAN_ERR_INVALID_ARG;
    if (!ws.ctrl) return LSCAN_ERR_NOT_FOUND;
    const hipError_t e = hipMemcpy(ctrl, ws.ctrl, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_error(e);
    *launches = ws.launches;
    return LSCAN_OK;
}

// The per-stream workspace of (current device, stream), after the stream
// has drained; null if there is none.
lscan_status stream_workspace_synced(void* stream_ptr, Workspace** out)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e);
    auto it = g_ws.find(std::make_pair(dev, stream));
    *out = (it == g_ws.end()) ? nullptr : &it->second;
    return LSCAN_OK;
}

}  // namespace

extern "C" {

uint64_t lscan_test_epoch_limit(void) { return kMaxLaunchesPerEpochRun; }

lscan_status lscan_test_seed_epoch(void* stream, uint64_t launches, uint32_t tag, uint32_t abort_tag)
{
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace* ws = nullptr;
    lscan_status st = stream_workspace_synced(stream, &ws);
    if (st != LSCAN_OK) return st;
    return ws ? seed_epoch(*ws, launches, tag, abort_tag) : LSCAN_ERR_NOT_FOUND;
}

lscan_status lscan_test_graph_seed_epoch(lscan_graph* g, uint64_t launches, uint32_t tag, uint32_t abort_tag)
{
    if (!g) return LSCAN_ERR_INVALID_ARG;
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return device_error(e);
    return seed_epoch(g->ws, launches, tag, abort_tag);
}

lscan_status lscan_test_epoch_state(void* stream, uint64_t* launches, uint32_t ctrl[4])
{
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace* ws = nullptr;
    lscan_status st = stream_workspace_synced(stream, &ws);
    if (st != LSCAN_OK) return st;
    return ws ? epoch_state(*ws, launches, ctrl) : LSCAN_ERR_NOT_FOUND;
}

lscan_status lscan_test_graph_epoch_state(lscan_graph* g, uint64_t* launches, uint32_t ctrl[4])
{
    if (!g) return LSCAN_ERR_INVALID_ARG;
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return device_error(e);
    return epoch_state(g->ws, launches, ctrl);
}

int32_t lscan_num_tile_shapes(void) { return kNumShapes; }

lscan_status lscan_tile_shape(int32_t idx, lscan_params* out)
{
    if (!out || idx < 0 || idx >= kNumShapes) return LSCAN_ERR_INVALID_ARG;
    out->block_threads = kShapeThreads[idx];
    out->vectors_per_lane = kShapeVectors[idx];
    out->groups_per_cu = 0;
    out->handoff = LSCAN_HANDOFF_WINDOW;
    return LSCAN_OK;
}

lscan_status lscan_get_params(lscan_dtype dt, lscan_op op, uint32_t flags, int32_t kind, lscan_params* out)
{
    if (!out || kind < 0 || kind >= kNumModes) return LSCAN_ERR_INVALID_ARG;
    const int oc = (kind == kModeCompact) ? compact_opcode(dt) : opcode_of(dt, op, flags & LSCAN_F_COMPENSATED);
    if (oc == -1) return (kind == kModeCompact && dt == LSCAN_BF16) ? LSCAN_ERR_UNSUPPORTED : LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    init_params_locked();
    // running argmax / argmin: the 32-bit index row (what arrays below 2^31 elements use)
    const Params& p = g_params[kind][is_arg_op(op) && kind != kModeCompact ? oc + kArgShortOffset : oc];
    out->block_threads = kShapeThreads[p.shape];
    out->vectors_per_lane = kShapeVectors[p.shape];
    out->groups_per_cu = p.groups_per_cu;
    out->handoff = p.handoff;
    return LSCAN_OK;
}

lscan_status lscan_set_params(lscan_dtype dt, lscan_op op, uint32_t flags, int32_t kind, const lscan_params* p)
{
    if (!p || kind < 0 || kind >= kNumModes) return LSCAN_ERR_INVALID_ARG;
    const int oc = (kind == kModeCompact) ? compact_opcode(dt) : opcode_of(dt, op, flags & LSCAN_F_COMPENSATED);
    if (oc == -1) return (kind == kModeCompact && dt == LSCAN_BF16) ? LSCAN_ERR_UNSUPPORTED : LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    if (kind == kModeCompact && p->handoff != LSCAN_HANDOFF_WINDOW) return LSCAN_ERR_UNSUPPORTED;
    const int s = shape_index(p->block_threads, p->vectors_per_lane);
    if (s < 0) return LSCAN_ERR_UNSUPPORTED;
    if (p->groups_per_cu <= 0) return LSCAN_ERR_INVALID_ARG;
    if (p->handoff != LSCAN_HANDOFF_WINDOW && p->handoff != LSCAN_HANDOFF_CHAIN) return LSCAN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    init_params_locked();
    g_params[kind][oc] = Params{s, p->groups_per_cu, p->handoff};
    if (is_arg_op(op) && kind != kModeCompact) g_params[kind][oc + kArgShortOffset] = g_params[kind][oc];  // both index widths
    return LSCAN_OK;
}

lscan_status lscan_compact_with_params(const void* x, const uint8_t* keep, void* out, int64_t* count, int64_t n,
                                       lscan_dtype dt, const lscan_params* p, void* stream)
{
    Request r;
    lscan_status st = make_compact_request(x, keep, out, count, n, dt, p, &r);
    if (st != LSCAN_OK) return st;
    if (r.empty) {  // nothing is launched: the count is zero
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (capturing(s)) return LSCAN_ERR_UNSUPPORTED;  // no memset node in a caller's graph
        hipError_t e = hipMemsetAsync(count, 0, sizeof(int64_t), s);
        return e == hipSuccess ? LSCAN_OK : device_error(e);
    }
    return run(r, stream);
}

lscan_status lscan_compact(const void* x, const uint8_t* keep, void* out, int64_t* count, int64_t n, lscan_dtype dt,
                           void* stream)
{
    return lscan_compact_with_params(x, keep, out, count, n, dt, nullptr, stream);
}

lscan_status lscan_radix_offsets(const void* keys, int64_t n, lscan_dtype dt, int32_t shift, int32_t bits,
                                 int64_t block_items, int64_t* offsets, void* stream)
{
    if (dt < LSCAN_I32 || dt > LSCAN_BF16) return LSCAN_ERR_INVALID_ARG;
    if (dt == LSCAN_BF16) return LSCAN_ERR_UNSUPPORTED;
    const int kb = (dt == LSCAN_I64) ? 8 : 4;
    if (n < 0 || bits < 1 || bits > 8 || shift < 0 || shift + bits > 8 * kb || block_items < 1)
        return LSCAN_ERR_INVALID_ARG;
    if (n == 0) return LSCAN_OK;
    if (!keys || !offsets || reinterpret_cast<uintptr_t>(keys) % uintptr_t(kb) ||
        reinterpret_cast<uintptr_t>(offsets) % 8)
        return LSCAN_ERR_INVALID_ARG;
    const int64_t m = (n - 1) / block_items + 1;
    const int64_t digits = int64_t(1) << bits;
    if (m > (INT64_MAX / 16) / digits) return LSCAN_ERR_INVALID_ARG;
    const int64_t total = digits * m;
    if (ranges_overlap(keys, n * kb, offsets, total * 8)) return LSCAN_ERR_INVALID_ARG;
    if (capturing(static_cast<hipStream_t>(stream))) return LSCAN_ERR_UNSUPPORTED;  // as every eager scan
    RadixArgs a;
    a.keys = keys;
    a.n = n;
    a.block_items = block_items;
    a.num_blocks = m;
    // enough workgroups to fill the device, each writing a run of counts per
    // digit; the table of a workgroup stays within 32 KiB of LDS
    const int64_t want = (m + 1023) / 1024;
    a.group = std::max<int64_t>(1, std::min<int64_t>(want, 8192 / digits));
    a.counts = offsets;
    a.key_bytes = kb;
    a.shift = shift;
    a.bits = bits;
    a.vec_ok = (reinterpret_cast<uintptr_t>(keys) % 16 == 0 && block_items % (16 / kb) == 0) ? 1 : 0;
    hipError_t e = lscan::launch_digit_counts(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e);
    // the offsets: exclusive +-scan of the digit-major counts, in place
    Request r;
    lscan_status st = make_request(kModePlain, offsets, offsets, total, nullptr, 0, nullptr, 0, LSCAN_I64, LSCAN_ADD, 0,
                                   true, nullptr, &r);
    return st != LSCAN_OK ? st : run(r, stream);
}

lscan_status lscan_bfs_with_params(const int64_t* row_offsets, const int32_t* cols, int64_t num_vertices,
                                   int64_t num_edges, int32_t source, int32_t* levels, int32_t* parents,
                                   int64_t* stats, const lscan_params* p, void* stream)
{
    if (num_vertices < 0 || num_vertices > int64_t(INT32_MAX) - 1 || num_edges < 0 ||
        num_edges >= (int64_t(1) << 42))
        return LSCAN_ERR_INVALID_ARG;
    if (p) {
        lscan_status st = check_params(p);
        if (st != LSCAN_OK) return st;
        if (p->block_threads != 0 || p->vectors_per_lane != 0 || p->handoff != LSCAN_HANDOFF_WINDOW)
            return LSCAN_ERR_UNSUPPORTED;
    }
    auto mis = [](const void* q, uintptr_t al) { return reinterpret_cast<uintptr_t>(q) % al != 0; };
    if (stats && mis(stats, 8)) return LSCAN_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (num_vertices == 0) {
        if (capturing(s)) return LSCAN_ERR_UNSUPPORTED;  // no memset node in a caller's graph
        if (stats) {
            const hipError_t e = hipMemsetAsync(stats, 0, 4 * sizeof(int64_t), s);
            if (e != hipSuccess) return device_error(e);
        }
        return LSCAN_OK;
    }
    if (source < 0 || int64_t(source) >= num_vertices) return LSCAN_ERR_INVALID_ARG;
    if (!row_offsets || !levels || (num_edges > 0 && !cols)) return LSCAN_ERR_INVALID_ARG;
    if (mis(row_offsets, 8) || mis(cols, 4) || mis(levels, 4) || mis(parents, 4)) return LSCAN_ERR_INVALID_ARG;
    const int64_t rb = (num_vertices + 1) * 8, cb = num_edges * 4, vb = num_vertices * 4;
    if (ranges_overlap(levels, vb, row_offsets, rb) || ranges_overlap(levels, vb, cols, cb))
        return LSCAN_ERR_INVALID_ARG;
    if (parents && (ranges_overlap(parents, vb, row_offsets, rb) || ranges_overlap(parents, vb, cols, cb) ||
                    ranges_overlap(parents, vb, levels, vb)))
        return LSCAN_ERR_INVALID_ARG;
    if (stats && (ranges_overlap(stats, 32, row_offsets, rb) || ranges_overlap(stats, 32, cols, cb) ||
                  ranges_overlap(stats, 32, levels, vb) || (parents && ranges_overlap(stats, 32, parents, vb))))
        return LSCAN_ERR_INVALID_ARG;
    return bfs_run(row_offsets, cols, num_vertices, num_edges, source, levels, parents, stats, p, s);
}

lscan_status lscan_bfs(const int64_t* row_offsets, const int32_t* cols, int64_t num_vertices, int64_t num_edges,
                       int32_t source, int32_t* levels, int32_t* parents, int64_t* stats, void* stream)
{
    return lscan_bfs_with_params(row_offsets, cols, num_vertices, num_edges, source, levels, parents, stats,
                                 nullptr, stream);
}

lscan_status lscan_scan_custom(const lscan_custom_kernel* kernel, const void* x, void* y, int64_t n,
                               uint32_t flags, const lscan_params* p, void* stream)
{
    const KernelEntry* k = reinterpret_cast<const KernelEntry*>(kernel);
    if (!k || (k->abi & 0xFFFF0000u) != kKernelAbiMark) return LSCAN_ERR_INVALID_ARG;
    if (k->abi != kKernelAbi) return LSCAN_ERR_UNSUPPORTED;  // built against another layout of the headers
    if (!k->func || !k->launch) return LSCAN_ERR_INVALID_ARG;
    if (k->block_threads < 64 || k->block_threads > 1024 || k->block_threads % 64 != 0 || k->vectors_per_lane < 1 ||
        k->elems_per_vec < 1 || k->in_bytes < 1 || k->out_bytes < 1 || k->slot_words < 1 ||
        k->tile_elems != int64_t(k->block_threads) * k->vectors_per_lane * k->elems_per_vec)
        return LSCAN_ERR_INVALID_ARG;  // not an entry made by lscan_custom.hpp
    if (flags & ~(LSCAN_F_EXCLUSIVE | LSCAN_F_DETERMINISTIC)) return LSCAN_ERR_INVALID_ARG;
    lscan_status st = check_params(p);
    if (st != LSCAN_OK) return st;
    if (p && (p->block_threads != 0 || p->vectors_per_lane != 0)) return LSCAN_ERR_UNSUPPORTED;  // fixed by the kernel
    if (n < 0) return LSCAN_ERR_INVALID_ARG;
    if (n > 0) {
        if (!x || !y) return LSCAN_ERR_INVALID_ARG;
        const uintptr_t ax = uintptr_t(std::min(k->in_bytes, 16)), ay = uintptr_t(std::min(k->out_bytes, 16));
        if (reinterpret_cast<uintptr_t>(x) % ax || reinterpret_cast<uintptr_t>(y) % ay) return LSCAN_ERR_INVALID_ARG;
        if (x == y) {
            if (k->in_bytes != k->out_bytes) return LSCAN_ERR_INVALID_ARG;
        } else if (ranges_overlap(x, n * k->in_bytes, y, n * k->out_bytes)) {
            return LSCAN_ERR_INVALID_ARG;
        }
    }
    Request r;
    r.mode = kModePlain;
    r.custom = k;
    r.x = x;
    r.y = y;
    r.n = n;
    r.exclusive = (flags & LSCAN_F_EXCLUSIVE) != 0;
    r.p = p;
    r.empty = (n == 0);
    return run(r, stream);
}

lscan_status lscan_set_watchdog_us(int64_t us)
{
    if (us < 0 || us > int64_t(3600) * 1000000) return LSCAN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    g_watchdog_us = us;
    for (auto& kv : g_dev) kv.second.spin_limit = uint64_t(double(kv.second.wall_khz) * double(us) / 1000.0);
    return LSCAN_OK;
}

int64_t lscan_get_watchdog_us(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    return g_watchdog_us;
}

lscan_status lscan_last_launch(lscan_launch_info* out)
{
    if (!out) return LSCAN_ERR_INVALID_ARG;
    *out = t_last_launch;
    return LSCAN_OK;
}

lscan_status lscan_check(void* stream_ptr)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e);
    // the stream's workspace, and the device's fixed one (shared by every
    // stream) once lscan_inclusive_noalloc has set it up
    uint32_t* ctrls[2] = {nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_ws.find(std::make_pair(dev, stream));
        if (it != g_ws.end()) ctrls[0] = it->second.ctrl;
        if (dev >= 0 && dev < kMaxNoAllocDevices && g_noalloc_ready[dev]) ctrls[1] = g_noalloc_ws[dev].ctrl;
    }
    bool timed_out = false;
    for (uint32_t* ctrl : ctrls) {
        if (!ctrl) continue;
        uint32_t flag = 0;
        e = hipMemcpy(&flag, ctrl + 2, sizeof(flag), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return device_error(e);
        if (flag) {
            const uint32_t zero = 0;
            e = hipMemcpy(ctrl + 2, &zero, sizeof(zero), hipMemcpyHostToDevice);
            if (e != hipSuccess) return device_error(e);
            timed_out = true;
        }
    }
    return timed_out ? LSCAN_ERR_TIMEOUT : LSCAN_OK;
}

lscan_status lscan_release_workspaces(void)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return device_error(e);
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first == dev) {
            free_workspace(it->second);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = g_bfs_ws.begin(); it != g_bfs_ws.end();) {
        if (it->first.first == dev) {
            free_bfs_workspace(it->second);
            it = g_bfs_ws.erase(it);
        } else {
            ++it;
        }
    }
    g_order[dev].any = false;  // the device is idle: nothing to order after
    g_order[dev].multi = false;
    return LSCAN_OK;
}

const char* lscan_status_string(lscan_status s)
{
    switch (s) {
    case LSCAN_OK: return "ok";
    case LSCAN_PENDING: return "pending";
    case LSCAN_ERR_INVALID_ARG: return "invalid argument";
    case LSCAN_ERR_UNSUPPORTED: return "unsupported combination";
    case LSCAN_ERR_NO_MEMORY: return "out of memory or over budget";
    case LSCAN_ERR_DEVICE: return "HIP runtime error";
    case LSCAN_ERR_AGAIN: return "queue full, try again";
    case LSCAN_ERR_TIMEOUT: return "a workgroup timed out waiting for a block prefix";
    case LSCAN_ERR_NOT_FOUND: return "unknown ticket";
    default: return "unknown status";
    }
}

int32_t lscan_last_device_error(void) { return t_last_hip_error; }

}  // extern "C"
