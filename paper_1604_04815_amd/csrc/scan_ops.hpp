// scan_ops.hpp -- scan operators and wave64 cross-lane building blocks for
// gfx950 (CDNA4).
//
// An operator type describes one (+) of the paper's problem statement
// (Section 1) as the kernel sees it:
//   In        element type read from x (float types are read as raw bits)
//   V         value carried through the scan (may differ from In: f32
//             max/min scan an integer order key, compensated add carries an
//             (s, c) pair, segmented scans carry a head flag)
//   Out       element type written to y
//   E         elements per lane per vector load (16-byte loads, 8-byte for
//             bf16, so every lane-row writes 16 bytes of output)
//   identity  the identity e of (+)
//   combine   a (+) b, with a the earlier (left) operand
//   lift      In -> V;  lower  V -> Out
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lscan {

// ---------------------------------------------------------------------------
// Cross-lane moves (DPP, data-parallel primitives of the GFX9 ISA family).
// The paper's intra-warp step uses shuffle-up and broadcast on 32 lanes
// (Section 4.1); wave64 on CDNA uses DPP row shifts, row broadcasts and a
// whole-wave shift instead, which read a neighbour's register in the same
// instruction with no LDS traffic.
// ---------------------------------------------------------------------------
enum : int {
    kDppRowShr1 = 0x111,
    kDppRowShr2 = 0x112,
    kDppRowShr4 = 0x114,
    kDppRowShr8 = 0x118,
    kDppWaveShr1 = 0x138,
    kDppRowBcast15 = 0x142,
    kDppRowBcast31 = 0x143,
};

// Lane-wise DPP move of any 4-byte-multiple value: lanes whose source lane
// is out of range, or whose row is masked off, receive `old`.
template <int CTRL, int ROW_MASK, class V>
__device__ __forceinline__ V dpp_move(const V& old, const V& src)
{
    static_assert(sizeof(V) % 4 == 0, "DPP moves 32-bit words");
    constexpr int NW = sizeof(V) / 4;
    int o[NW], s[NW];
    __builtin_memcpy(o, &old, sizeof(V));
    __builtin_memcpy(s, &src, sizeof(V));
#pragma unroll
    for (int k = 0; k < NW; ++k)
        s[k] = __builtin_amdgcn_update_dpp(o[k], s[k], CTRL, ROW_MASK, 0xf, false);
    V r;
    __builtin_memcpy(&r, s, sizeof(V));
    return r;
}

// Value of lane `lane` (wave-uniform result).
template <class V>
__device__ __forceinline__ V read_lane(const V& v, int lane)
{
    constexpr int NW = sizeof(V) / 4;
    int s[NW];
    __builtin_memcpy(s, &v, sizeof(V));
#pragma unroll
    for (int k = 0; k < NW; ++k) s[k] = __builtin_amdgcn_readlane(s[k], lane);
    V r;
    __builtin_memcpy(&r, s, sizeof(V));
    return r;
}

// Inclusive scan across the 64 lanes of a wave (Hillis-Steele steps, as the
// paper's intra-warp row scan, Section 4.1): four row shifts build the scan
// inside each 16-lane row, then two row broadcasts carry row totals into the
// following rows.  Lane 63 ends with the wave total.
template <class Op>
__device__ __forceinline__ typename Op::V wave_inclusive_scan(typename Op::V v)
{
    using V = typename Op::V;
    const V e = Op::identity();
    v = Op::combine(dpp_move<kDppRowShr1, 0xf>(e, v), v);
    v = Op::combine(dpp_move<kDppRowShr2, 0xf>(e, v), v);
    v = Op::combine(dpp_move<kDppRowShr4, 0xf>(e, v), v);
    v = Op::combine(dpp_move<kDppRowShr8, 0xf>(e, v), v);
    v = Op::combine(dpp_move<kDppRowBcast15, 0xa>(e, v), v);
    v = Op::combine(dpp_move<kDppRowBcast31, 0xc>(e, v), v);
    return v;
}

// Shift an inclusive lane scan to the exclusive one (lane 0 gets e).
template <class Op>
__device__ __forceinline__ typename Op::V wave_shift_right(typename Op::V v)
{
    return dpp_move<kDppWaveShr1, 0xf>(Op::identity(), v);
}

// ---------------------------------------------------------------------------
// Operators
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bits_to_f32(uint32_t b) { return __uint_as_float(b); }
__device__ __forceinline__ uint32_t f32_to_bits(float f) { return __float_as_uint(f); }

// IEEE 754 totalOrder on non-NaN floats as a signed integer key: for a
// negative float the 31 magnitude bits are flipped, so larger magnitudes
// sort lower and -0 sorts below +0.  The map is its own inverse.
__device__ __forceinline__ int32_t order_key(uint32_t bits)
{
    return (int32_t)(bits ^ ((uint32_t)((int32_t)bits >> 31) >> 1));
}
__device__ __forceinline__ uint32_t key_bits(int32_t key)
{
    return (uint32_t)key ^ ((uint32_t)(key >> 31) >> 1);
}

struct AddI32 {
    using In = int32_t; using V = int32_t; using Out = int32_t;
    static constexpr int E = 4;
    __device__ static V identity() { return 0; }
    __device__ static V combine(V a, V b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};
struct MaxI32 {
    using In = int32_t; using V = int32_t; using Out = int32_t;
    static constexpr int E = 4;
    __device__ static V identity() { return INT32_MIN; }
    __device__ static V combine(V a, V b) { return a > b ? a : b; }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};
struct MinI32 {
    using In = int32_t; using V = int32_t; using Out = int32_t;
    static constexpr int E = 4;
    __device__ static V identity() { return INT32_MAX; }
    __device__ static V combine(V a, V b) { return a < b ? a : b; }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};
struct AddI64 {
    using In = int64_t; using V = int64_t; using Out = int64_t;
    static constexpr int E = 2;
    __device__ static V identity() { return 0; }
    __device__ static V combine(V a, V b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};
struct MaxI64 {
    using In = int64_t; using V = int64_t; using Out = int64_t;
    static constexpr int E = 2;
    __device__ static V identity() { return INT64_MIN; }
    __device__ static V combine(V a, V b) { return a > b ? a : b; }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};
struct MinI64 {
    using In = int64_t; using V = int64_t; using Out = int64_t;
    static constexpr int E = 2;
    __device__ static V identity() { return INT64_MAX; }
    __device__ static V combine(V a, V b) { return a < b ? a : b; }
    __device__ static V lift(In x) { return x; }
    __device__ static Out lower(V v) { return v; }
};

// float32 add (rounded; the association is fixed by the launch shape).
struct AddF32 {
    using In = uint32_t; using V = float; using Out = float;
    static constexpr int E = 4;
    __device__ static V identity() { return 0.0f; }
    __device__ static V combine(V a, V b) { return a + b; }
    __device__ static V lift(In x) { return bits_to_f32(x); }
    __device__ static Out lower(V v) { return v; }
};

// Compensated float32 add: the state is (s, c) with s + c the running sum.
// Combining two states adds the s parts with TwoSum (Knuth), which also
// yields the exact rounding error of that addition, and folds that error
// together with both c parts into c.  The output is fl(s + c).
//
// A lifted element carries c = -0.0: x + (-0.0) == x for every x (signed
// zeros included), so the compiler drops the c addition of every combine
// with a freshly lifted element.  (The identity keeps c = +0.0, which the
// cross-lane moves supply for free to lanes without a source.)
//
// finish(q, e), the output of q (+) e, is fl(fl(q.s + e.s) + fl(q.c + e.c))
// instead of a full TwoSum followed by fl(s + c): three additions instead
// of nine.  With q the prefix before a lane's vector and e the in-lane
// partial sum, |q.s + e.s| exceeds the result |y| only by the small
// compensation terms, so the two extra roundings add at most about
// u * |y| (u = 2^-24) to the rounding of the result itself.
struct F32Pair {
    float s, c;
};
__device__ __forceinline__ F32Pair two_sum_combine(F32Pair a, F32Pair b)
{
#pragma clang fp contract(off)
    const float s = a.s + b.s;
    const float bb = s - a.s;
    const float err = (a.s - (s - bb)) + (b.s - bb);
    F32Pair r;
    r.s = s;
    r.c = (a.c + b.c) + err;
    return r;
}
struct AddF32Comp {
    using In = uint32_t; using V = F32Pair; using Out = float;
    static constexpr int E = 4;
    // a lane scans R consecutive vectors (a zero input word lifts to an identity)
    static constexpr bool kBlockedLanes = true;
    __device__ static V identity() { return F32Pair{0.0f, 0.0f}; }
    __device__ static V combine(V a, V b) { return two_sum_combine(a, b); }
    __device__ static V lift(In x) { return F32Pair{bits_to_f32(x), -0.0f}; }
    __device__ static Out lower(V v) { return v.s + v.c; }
    __device__ static Out finish(V q, V e) { return (q.s + e.s) + (q.c + e.c); }
};

// float32 max / min under totalOrder, scanned on integer keys (exact).
struct MaxF32 {
    using In = uint32_t; using V = int32_t; using Out = float;
    static constexpr int E = 4;
    __device__ static V identity() { return order_key(0xff800000u); }  // -inf
    __device__ static V combine(V a, V b) { return a > b ? a : b; }
    __device__ static V lift(In x) { return order_key(x); }
    __device__ static Out lower(V v) { return bits_to_f32(key_bits(v)); }
};
struct MinF32 {
    using In = uint32_t; using V = int32_t; using Out = float;
    static constexpr int E = 4;
    __device__ static V identity() { return order_key(0x7f800000u); }  // +inf
    __device__ static V combine(V a, V b) { return a < b ? a : b; }
    __device__ static V lift(In x) { return order_key(x); }
    __device__ static Out lower(V v) { return bits_to_f32(key_bits(v)); }
};

// Running argmax / argmin: the value carries the element's index, and the
// scan keeps the best (key, index) pair, the earlier one among equal keys
// (a is always the earlier operand, so ties keep a).  An index < 0 marks
// the identity, which loses to every element.  The output is the int64
// index.  Keys: int32 / int64 values, float32 as totalOrder keys.  The
// index is kept as two 32-bit halves so that a 32-bit key gives a
// three-word value (three DPP moves per step).
template <class KeyT>
struct ArgValue;
template <>
struct ArgValue<int32_t> {
    int32_t key;
    uint32_t lo, hi;
    __device__ int64_t index() const { return int64_t((uint64_t(hi) << 32) | lo); }
};
template <>
struct ArgValue<int64_t> {
    int64_t key;
    uint32_t lo, hi;
    __device__ int64_t index() const { return int64_t((uint64_t(hi) << 32) | lo); }
};

template <class In_, class KeyT, bool MAX, bool FLOAT_KEY>
struct ArgOp {
    using In = In_; using V = ArgValue<KeyT>; using Out = int64_t;
    static constexpr int E = 16 / int(sizeof(In));
    static constexpr bool kIndexed = true;
    __device__ static V identity()
    {
        V v;
        v.key = 0;
        v.lo = 0xffffffffu;
        v.hi = 0xffffffffu;
        return v;
    }
    __device__ static V combine(V a, V b)
    {
        // field by field: a select of whole structs would go through memory
        const bool a_id = int32_t(a.hi) < 0, b_id = int32_t(b.hi) < 0;
        const bool take_b = a_id || (!b_id && (MAX ? (b.key > a.key) : (b.key < a.key)));
        V r;
        r.key = take_b ? b.key : a.key;
        r.lo = take_b ? b.lo : a.lo;
        r.hi = take_b ? b.hi : a.hi;
        return r;
    }
    __device__ static V lift_at(In x, int64_t i)
    {
        V v;
        if constexpr (FLOAT_KEY)
            v.key = order_key(x);
        else
            v.key = KeyT(x);
        v.lo = uint32_t(uint64_t(i));
        v.hi = uint32_t(uint64_t(i) >> 32);
        return v;
    }
    __device__ static Out lower(const V& v) { return v.index(); }
};
using ArgMaxI32 = ArgOp<int32_t, int32_t, true, false>;
using ArgMinI32 = ArgOp<int32_t, int32_t, false, false>;
using ArgMaxI64 = ArgOp<int64_t, int64_t, true, false>;
using ArgMinI64 = ArgOp<int64_t, int64_t, false, false>;
using ArgMaxF32 = ArgOp<uint32_t, int32_t, true, true>;
using ArgMinF32 = ArgOp<uint32_t, int32_t, false, true>;

// Arrays of fewer than 2^31 elements carry the index in one 32-bit word: a
// 32-bit key then makes a two-word value, a 64-bit key three words (kept
// as two halves so the value has no padding).  idx < 0 marks the identity.
template <class KeyT>
struct ArgValueS;
template <>
struct ArgValueS<int32_t> {
    int32_t k;
    int32_t idx;
    __device__ int32_t key() const { return k; }
    __device__ void set_key(int32_t v) { k = v; }
};
template <>
struct ArgValueS<int64_t> {
    uint32_t klo, khi;
    int32_t idx;
    __device__ int64_t key() const { return int64_t((uint64_t(khi) << 32) | klo); }
    __device__ void set_key(int64_t v)
    {
        klo = uint32_t(uint64_t(v));
        khi = uint32_t(uint64_t(v) >> 32);
    }
};

template <class In_, class KeyT, bool MAX, bool FLOAT_KEY>
struct ArgOpS {
    using In = In_; using V = ArgValueS<KeyT>; using Out = int64_t;
    static constexpr int E = 16 / int(sizeof(In));
    static constexpr bool kIndexed = true;
    __device__ static V identity()
    {
        V v;
        v.set_key(0);
        v.idx = -1;
        return v;
    }
    __device__ static V combine(V a, V b)
    {
        const KeyT ka = a.key(), kb = b.key();
        const bool take_b = a.idx < 0 || (b.idx >= 0 && (MAX ? (kb > ka) : (kb < ka)));
        V r;
        r.set_key(take_b ? kb : ka);
        r.idx = take_b ? b.idx : a.idx;
        return r;
    }
    __device__ static V lift_at(In x, int64_t i)
    {
        V v;
        if constexpr (FLOAT_KEY)
            v.set_key(order_key(x));
        else
            v.set_key(KeyT(x));
        v.idx = int32_t(i);
        return v;
    }
    __device__ static Out lower(const V& v) { return int64_t(v.idx); }
};
using ArgMaxI32S = ArgOpS<int32_t, int32_t, true, false>;
using ArgMinI32S = ArgOpS<int32_t, int32_t, false, false>;
using ArgMaxI64S = ArgOpS<int64_t, int64_t, true, false>;
using ArgMinI64S = ArgOpS<int64_t, int64_t, false, false>;
using ArgMaxF32S = ArgOpS<uint32_t, int32_t, true, true>;
using ArgMinF32S = ArgOpS<uint32_t, int32_t, false, true>;

// Element lift for operators with (kIndexed) or without the element index.
template <class Op, class = void>
struct is_indexed_op : std::false_type {};
template <class Op>
struct is_indexed_op<Op, std::void_t<decltype(Op::kIndexed)>> : std::integral_constant<bool, Op::kIndexed> {};

template <class Op>
__device__ __forceinline__ typename Op::V lift_elem(typename Op::In x, int64_t i)
{
    if constexpr (is_indexed_op<Op>::value)
        return Op::lift_at(x, i);
    else
        return Op::lift(x);
}

// Output of q (+) e: the operator's own finish when it has one, else
// lower(combine(q, e)).
template <class Op, class = void>
struct has_finish : std::false_type {};
template <class Op>
struct has_finish<Op, std::void_t<decltype(Op::finish(Op::identity(), Op::identity()))>> : std::true_type {};

template <class Op>
__device__ __forceinline__ typename Op::Out finish_of(const typename Op::V& q, const typename Op::V& e)
{
    if constexpr (has_finish<Op>::value)
        return Op::finish(q, e);
    else
        return Op::lower(Op::combine(q, e));
}

// bfloat16 input: the 16 bits become the high half of an f32 (exact), then
// the f32 operator runs.  Loads are 8 bytes (4 elements) per lane so that
// the 4 float32 outputs fill one 16-byte store.
__device__ __forceinline__ uint32_t bf16_bits_to_f32_bits(uint16_t h) { return (uint32_t)h << 16; }

// Whether an operator asks for lane-blocked rows (its kBlockedLanes member).
template <class Op, class = void>
struct blocked_lanes : std::false_type {};
template <class Op>
struct blocked_lanes<Op, std::void_t<decltype(Op::kBlockedLanes)>> : std::bool_constant<Op::kBlockedLanes> {};
template <class F32Op>
struct FromBF16 {
    using In = uint16_t; using V = typename F32Op::V; using Out = typename F32Op::Out;
    static constexpr int E = 4;
    __device__ static V identity() { return F32Op::identity(); }
    __device__ static V combine(V a, V b) { return F32Op::combine(a, b); }
    __device__ static V lift(In x) { return F32Op::lift(bf16_bits_to_f32_bits(x)); }
    __device__ static Out lower(V v) { return F32Op::lower(v); }
    __device__ static Out finish(V q, V e) { return finish_of<F32Op>(q, e); }
    static constexpr bool kBlockedLanes = blocked_lanes<F32Op>::value;
};
using AddBF16 = FromBF16<AddF32>;
using AddBF16Comp = FromBF16<AddF32Comp>;
using MaxBF16 = FromBF16<MaxF32>;
using MinBF16 = FromBF16<MinF32>;

// Segmented operator on (value, head flag) pairs: a head starts a new
// segment, so  (a, fa) (+) (b, fb) = (fb ? b : a (+) b, fa | fb).
// It is associative whenever (+) is, with identity (e, 0).
template <class VV, bool PAD>
struct SegValue;
template <class VV>
struct SegValue<VV, false> {
    VV v;
    uint32_t f;
    __device__ void clear_pad() {}
};
template <class VV>
struct SegValue<VV, true> {  // 8-byte values: keep sizeof free of padding
    VV v;
    uint32_t f;
    uint32_t pad;
    __device__ void clear_pad() { pad = 0; }
};

template <class Op>
struct Seg {
    using In = typename Op::In; using Out = typename Op::Out;
    static constexpr int E = Op::E;
    using V = SegValue<typename Op::V, alignof(typename Op::V) == 8>;
    __device__ static V make(typename Op::V v, uint32_t head)
    {
        V r;
        r.v = v;
        r.f = head;
        r.clear_pad();
        return r;
    }
    __device__ static V identity() { return make(Op::identity(), 0u); }
    __device__ static V combine(const V& a, const V& b)
    {
        return make(b.f ? b.v : Op::combine(a.v, b.v), a.f | b.f);
    }
};

}  // namespace lscan
