// runtime.cpp -- host side of the C ABI declared in include/lscan.h:
// argument validation, kernel selection, grid sizing against the occupancy
// limit, and the per-(device, stream) flag workspaces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "kernel_table.hpp"
#include "lscan.h"

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

// A co-residency test waits this long for the whole grid to arrive.
constexpr double kResidencyWaitSeconds = 0.02;

struct DeviceInfo {
    int cu_count = 0;
    uint64_t spin_limit = 0;
    uint64_t residency_limit = 0;
    int occupancy[2][kNumOpCodes][kNumShapes];
    // groups per CU proven resident together (0: none yet) and the smallest
    // count that failed the test (0: none failed)
    int resident_ok[2][kNumOpCodes][kNumShapes];
    int resident_fail[2][kNumOpCodes][kNumShapes];
};

struct Workspace {
    uint64_t* slots = nullptr;
    size_t words = 0;
    uint32_t* ctrl = nullptr;   // [0] last tag, [1] exit counter, [2] timeout flag
    uint64_t launches = 0;
};

struct Params {
    int shape;
    int groups_per_cu;
};

std::mutex g_mu;
std::map<int, DeviceInfo> g_dev;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
Params g_params[2][kNumOpCodes];
bool g_params_init = false;

// Tags are 32-bit and 0 marks a never-written slot: reset a workspace well
// before its tag counter could wrap.
constexpr uint64_t kMaxLaunchesPerEpochRun = 0xfffffff0ull;

lscan_status device_error(hipError_t e)
{
    t_last_hip_error = int32_t(e);
    return LSCAN_ERR_DEVICE;
}

// Defaults measured on MI355X (gfx950) with N = 2^27..2^28 arrays: shape
// index into kShapeThreads/kShapeVectors and workgroups per CU (capped later
// by the occupancy limit and the co-residency test).
void init_params_locked()
{
    if (g_params_init) return;
    const Params t256x8{0, 5}, t256x16{3, 3}, t1024x4{4, 1}, comp_bf16{3, 2};
    for (int o = kI32Add; o <= kI32Min; ++o) g_params[0][o] = t256x8;
    for (int o = kI64Add; o <= kI64Min; ++o) g_params[0][o] = t256x16;
    g_params[0][kF32Add] = t256x8;
    g_params[0][kF32AddComp] = t1024x4;
    g_params[0][kF32Max] = t256x8;
    g_params[0][kF32Min] = t256x8;
    g_params[0][kBF16Add] = t256x16;
    g_params[0][kBF16AddComp] = comp_bf16;
    g_params[0][kBF16Max] = t256x16;
    g_params[0][kBF16Min] = t256x16;
    // segmented kernels: the per-tile head search adds latency, so fewer
    // groups per CU measured best
    for (int o = 0; o < kNumOpCodes; ++o) {
        g_params[1][o] = g_params[0][o];
        if (g_params[1][o].groups_per_cu > 3) g_params[1][o].groups_per_cu = 3;
    }
    g_params_init = true;
}

int opcode_of(int dt, int op, uint32_t flags)
{
    const bool comp = (flags & LSCAN_F_COMPENSATED) != 0;
    if (dt < LSCAN_I32 || dt > LSCAN_BF16 || op < LSCAN_ADD || op > LSCAN_MIN) return -1;
    if (comp && !((dt == LSCAN_F32 || dt == LSCAN_BF16) && op == LSCAN_ADD)) return -2;
    switch (dt) {
    case LSCAN_I32: return kI32Add + op;
    case LSCAN_I64: return kI64Add + op;
    case LSCAN_F32: return op == LSCAN_ADD ? (comp ? kF32AddComp : kF32Add) : (op == LSCAN_MAX ? kF32Max : kF32Min);
    case LSCAN_BF16: return op == LSCAN_ADD ? (comp ? kBF16AddComp : kBF16Add) : (op == LSCAN_MAX ? kBF16Max : kBF16Min);
    }
    return -1;
}

int in_bytes_of(int dt) { return dt == LSCAN_I64 ? 8 : dt == LSCAN_BF16 ? 2 : 4; }
int out_bytes_of(int dt) { return dt == LSCAN_I64 ? 8 : 4; }

int shape_index(int threads, int vectors)
{
    for (int s = 0; s < kNumShapes; ++s)
        if (kShapeThreads[s] == threads && kShapeVectors[s] == vectors) return s;
    return -1;
}

lscan_status check_common(const void* x, const void* y, int64_t n, int dt, int op, uint32_t flags,
                          uint32_t allowed_flags, int* opcode)
{
    if (flags & ~allowed_flags) return LSCAN_ERR_INVALID_ARG;
    const int oc = opcode_of(dt, op, flags);
    if (oc == -1) return LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    if (n < 0) return LSCAN_ERR_INVALID_ARG;
    *opcode = oc;
    if (n == 0) return LSCAN_OK;
    if (!x || !y) return LSCAN_ERR_INVALID_ARG;
    const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    const int ib = in_bytes_of(dt), ob = out_bytes_of(dt);
    if (xa % uintptr_t(ib) || ya % uintptr_t(ob)) return LSCAN_ERR_INVALID_ARG;
    if (uint64_t(n) > (UINT64_MAX / 16)) return LSCAN_ERR_INVALID_ARG;
    const uintptr_t xe = xa + uintptr_t(n) * uintptr_t(ib), ye = ya + uintptr_t(n) * uintptr_t(ob);
    const bool overlap = xa < ye && ya < xe;
    if (overlap && !(xa == ya && ib == ob)) return LSCAN_ERR_INVALID_ARG;
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
        info.spin_limit = uint64_t(double(wall_khz) * 1000.0 * kSpinLimitSeconds);
        info.residency_limit = uint64_t(double(wall_khz) * 1000.0 * kResidencyWaitSeconds);
        for (int s = 0; s < 2; ++s)
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

lscan_status workspace_locked(int dev, hipStream_t stream, size_t words, Workspace** out)
{
    Workspace& ws = g_ws[std::make_pair(dev, stream)];
    hipError_t e;
    const bool need_reset = ws.launches >= kMaxLaunchesPerEpochRun;
    if (ws.words < words || !ws.ctrl || need_reset) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
            return LSCAN_ERR_UNSUPPORTED;  // size the workspace with an eager call before capturing
        if (ws.slots || ws.ctrl) {
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
            ws.words = alloc;
            e = hipMemsetAsync(ws.slots, 0, alloc * sizeof(uint64_t), stream);
            if (e != hipSuccess) return device_error(e);
        } else if (need_reset) {
            e = hipMemsetAsync(ws.slots, 0, ws.words * sizeof(uint64_t), stream);
            if (e != hipSuccess) return device_error(e);
        }
        if (!ws.ctrl) {
            e = hipMalloc(reinterpret_cast<void**>(&ws.ctrl), 64);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return LSCAN_ERR_NO_MEMORY;
            }
            e = hipMemsetAsync(ws.ctrl, 0, 64, stream);
            if (e != hipSuccess) return device_error(e);
        } else if (need_reset) {
            // keep the timeout flag (word 2); restart the tag and exit counter
            e = hipMemsetAsync(ws.ctrl, 0, 2 * sizeof(uint32_t), stream);
            if (e != hipSuccess) return device_error(e);
        }
        if (need_reset) ws.launches = 0;
    }
    *out = &ws;
    return LSCAN_OK;
}

// Launch the kernel in its co-residency test mode with `groups` workgroups
// per CU and report whether they were all resident at once.
lscan_status test_residency_locked(const KernelEntry& k, int cu_count, int groups, uint64_t limit,
                                   Workspace* ws, hipStream_t stream, bool* ok)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        return LSCAN_ERR_UNSUPPORTED;  // run one eager call of this shape before capturing
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
lscan_status resident_groups_locked(DeviceInfo* info, int sg, int oc, int shape, const KernelEntry& k,
                                    int want, Workspace* ws, hipStream_t stream, int* out)
{
    int& good = info->resident_ok[sg][oc][shape];
    int& bad = info->resident_fail[sg][oc][shape];
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

lscan_status run_scan(bool segmented, const void* x, void* y, int64_t n, const int64_t* offsets,
                      int64_t num_segments, int dt, int op, uint32_t flags, bool exclusive,
                      const lscan_params* p, void* stream_ptr)
{
    int oc = 0;
    const uint32_t allowed = segmented ? (LSCAN_F_COMPENSATED | LSCAN_F_EXCLUSIVE) : LSCAN_F_COMPENSATED;
    lscan_status st = check_common(x, y, n, dt, op, flags, allowed, &oc);
    if (st != LSCAN_OK) return st;
    if (segmented) {
        if (num_segments < 0) return LSCAN_ERR_INVALID_ARG;
        if (num_segments == 0 && n != 0) return LSCAN_ERR_INVALID_ARG;
        if (num_segments > 0 && !offsets) return LSCAN_ERR_INVALID_ARG;
        if (reinterpret_cast<uintptr_t>(offsets) % 8) return LSCAN_ERR_INVALID_ARG;
    }
    if (p && (p->block_threads != 0 || p->vectors_per_lane != 0) &&
        shape_index(p->block_threads, p->vectors_per_lane) < 0)
        return LSCAN_ERR_UNSUPPORTED;
    if (p && p->groups_per_cu < 0) return LSCAN_ERR_INVALID_ARG;
    if (n == 0) return LSCAN_OK;

    const int sg = segmented ? 1 : 0;
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    const KernelTable& tab = table();

    std::lock_guard<std::mutex> lock(g_mu);
    init_params_locked();
    Params prm = g_params[sg][oc];
    if (p && (p->block_threads != 0 || p->vectors_per_lane != 0))
        prm.shape = shape_index(p->block_threads, p->vectors_per_lane);
    if (p && p->groups_per_cu > 0) prm.groups_per_cu = p->groups_per_cu;
    const KernelEntry& k = tab[sg][oc][prm.shape];

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e);
    DeviceInfo* info = nullptr;
    st = device_info_locked(dev, &info);
    if (st != LSCAN_OK) return st;
    int& occ = info->occupancy[sg][oc][prm.shape];
    if (occ < 0) {
        int v = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k.func, k.block_threads, 0);
        if (e != hipSuccess) return device_error(e);
        occ = v;
    }
    if (occ <= 0) return LSCAN_ERR_UNSUPPORTED;

    const int64_t L = k.tile_elems;
    const int64_t M = (n + L - 1) / L;

    Workspace* ws = nullptr;
    st = workspace_locked(dev, stream, size_t(M) * size_t(k.slot_words), &ws);
    if (st != LSCAN_OK) return st;

    // The grid must fit on the device at once: cap by the occupancy limit,
    // then by what the co-residency test has shown (a grid no larger than M
    // needs only the groups that M blocks fill).
    int want = std::min<int>(prm.groups_per_cu, occ);
    const int64_t need = (M + info->cu_count - 1) / info->cu_count;
    if (need < want) want = int(need);
    int groups = 0;
    st = resident_groups_locked(info, sg, oc, prm.shape, k, want, ws, stream, &groups);
    if (st != LSCAN_OK) return st;
    const int64_t B = std::max<int64_t>(1, std::min<int64_t>(M, int64_t(groups) * info->cu_count));

    const int vec_bytes = k.in_bytes * k.elems_per_vec;
    ScanArgs a;
    a.x = x;
    a.y = y;
    a.n = n;
    a.num_blocks = M;
    a.offsets = offsets;
    a.num_segments = num_segments;
    a.slots = ws->slots;
    a.ctrl = ws->ctrl;
    a.spin_limit = info->spin_limit;
    a.exclusive = exclusive ? 1 : 0;
    a.vec_ok = (reinterpret_cast<uintptr_t>(x) % uintptr_t(vec_bytes) == 0 &&
                reinterpret_cast<uintptr_t>(y) % 16 == 0) ? 1 : 0;
    a.residency_check = 0;
    a.pad_ = 0;

    e = k.launch(a, int(B), stream);
    if (e != hipSuccess) return device_error(e);
    ws->launches++;

    t_last_launch.n = n;
    t_last_launch.num_blocks = M;
    t_last_launch.tile_elems = L;
    t_last_launch.grid = int32_t(B);
    t_last_launch.block_threads = k.block_threads;
    t_last_launch.slot_words = k.slot_words;
    t_last_launch.vector_path = a.vec_ok;
    t_last_launch.groups_per_cu = groups;
    t_last_launch.occupancy = occ;
    return LSCAN_OK;
}

}  // namespace
}  // namespace lscan

using namespace lscan;

extern "C" {

lscan_status lscan_inclusive(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                             void* stream)
{
    return run_scan(false, x, y, n, nullptr, 0, dt, op, flags, false, nullptr, stream);
}

lscan_status lscan_exclusive(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op, uint32_t flags,
                             void* stream)
{
    return run_scan(false, x, y, n, nullptr, 0, dt, op, flags, true, nullptr, stream);
}

lscan_status lscan_segmented(const void* x, void* y, int64_t n_total, const int64_t* offsets,
                             int64_t num_segments, lscan_dtype dt, lscan_op op, uint32_t flags, void* stream)
{
    return run_scan(true, x, y, n_total, offsets, num_segments, dt, op, flags,
                    (flags & LSCAN_F_EXCLUSIVE) != 0, nullptr, stream);
}

lscan_status lscan_scan_with_params(const void* x, void* y, int64_t n, lscan_dtype dt, lscan_op op,
                                    uint32_t flags, int32_t exclusive, const lscan_params* p, void* stream)
{
    return run_scan(false, x, y, n, nullptr, 0, dt, op, flags, exclusive != 0, p, stream);
}

lscan_status lscan_segmented_with_params(const void* x, void* y, int64_t n_total, const int64_t* offsets,
                                         int64_t num_segments, lscan_dtype dt, lscan_op op, uint32_t flags,
                                         const lscan_params* p, void* stream)
{
    return run_scan(true, x, y, n_total, offsets, num_segments, dt, op, flags,
                    (flags & LSCAN_F_EXCLUSIVE) != 0, p, stream);
}

int32_t lscan_num_tile_shapes(void) { return kNumShapes; }

lscan_status lscan_tile_shape(int32_t idx, lscan_params* out)
{
    if (!out || idx < 0 || idx >= kNumShapes) return LSCAN_ERR_INVALID_ARG;
    out->block_threads = kShapeThreads[idx];
    out->vectors_per_lane = kShapeVectors[idx];
    out->groups_per_cu = 0;
    out->reserved = 0;
    return LSCAN_OK;
}

lscan_status lscan_get_params(lscan_dtype dt, lscan_op op, uint32_t flags, int32_t segmented, lscan_params* out)
{
    if (!out) return LSCAN_ERR_INVALID_ARG;
    const int oc = opcode_of(dt, op, flags);
    if (oc == -1) return LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    init_params_locked();
    const Params& p = g_params[segmented ? 1 : 0][oc];
    out->block_threads = kShapeThreads[p.shape];
    out->vectors_per_lane = kShapeVectors[p.shape];
    out->groups_per_cu = p.groups_per_cu;
    out->reserved = 0;
    return LSCAN_OK;
}

lscan_status lscan_set_params(lscan_dtype dt, lscan_op op, uint32_t flags, int32_t segmented, const lscan_params* p)
{
    if (!p) return LSCAN_ERR_INVALID_ARG;
    const int oc = opcode_of(dt, op, flags);
    if (oc == -1) return LSCAN_ERR_INVALID_ARG;
    if (oc == -2) return LSCAN_ERR_UNSUPPORTED;
    const int s = shape_index(p->block_threads, p->vectors_per_lane);
    if (s < 0) return LSCAN_ERR_UNSUPPORTED;
    if (p->groups_per_cu <= 0) return LSCAN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    init_params_locked();
    g_params[segmented ? 1 : 0][oc] = Params{s, p->groups_per_cu};
    return LSCAN_OK;
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
    uint32_t* ctrl = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_ws.find(std::make_pair(dev, stream));
        if (it == g_ws.end() || !it->second.ctrl) return LSCAN_OK;
        ctrl = it->second.ctrl;
    }
    uint32_t flag = 0;
    e = hipMemcpy(&flag, ctrl + 2, sizeof(flag), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_error(e);
    if (flag) {
        const uint32_t zero = 0;
        e = hipMemcpy(ctrl + 2, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (e != hipSuccess) return device_error(e);
        return LSCAN_ERR_TIMEOUT;
    }
    return LSCAN_OK;
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
            if (it->second.slots) (void)hipFree(it->second.slots);
            if (it->second.ctrl) (void)hipFree(it->second.ctrl);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
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
