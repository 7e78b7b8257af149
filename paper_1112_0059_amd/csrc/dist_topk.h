// Distance + top-(k+1) kernel (K1) of the local NBNN hot path for gfx950:
// operand policies, the selection helpers, the pipelined kernel template and
// its per-variant instantiation.  Each (format, list length) instance set is
// compiled in its own translation unit (dist_inst.hip).
//
// Distances.  For a query q and reference r the kernels rank by
//     d'(q, r) = ||r||^2 - 2 q.r  =  ||q - r||^2 - ||q||^2,
// which orders references exactly like the squared distance of Algorithm 2
// and leaves every difference dist_C - dist_B unchanged.  The MFMA
// accumulator is seeded with ||r||^2 and the query operand carries -2q, so
// one chain of MFMAs yields d' with no extra vector work.  For u8 data every
// product and partial sum is an integer below 2^24 in magnitude, so FP16 and
// BF16 operands with FP32 accumulation are exact in any summation order.
#pragma once
#include "internal.h"
#include <type_traits>

namespace lnbnn {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4v __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ uint32_t byte_at(uint2 r, int e)
{
    return ((e < 4 ? r.x : r.y) >> (8 * (e & 3))) & 0xffu;
}

// ---------------------------------------------------------------------------
// Operand policies.
//
// FP16/BF16 (v_mfma_f32_32x32x16_{f16,bf16}): a K step covers 16 elements;
// lane l supplies row (l & 31) and K elements 16*s + 8*(l >> 5) + e,
// e = 0..7, for both operands (one uint4 per lane per step), so packing the
// references and loading the queries with the same rule pairs them.
//
// FP8 (v_mfma_scale_f32_32x32x64_f8f6f4, OCP e4m3 operands): a K step
// covers 64 elements; lane l supplies 32 bytes (two uint4) of row (l & 31),
// K elements 64*s + 32*(l >> 5) + e.  Every lane also supplies an E8M0
// scale (2^(v-127)) for its row; the hardware applies the scale of lane i to
// bytes 0..15 and that of lane i+32 to bytes 16..31 of every lane of row i,
// so a per-row scale must be (and is) supplied by both lanes of the row.
// References carry 2^-e_r, queries 2^(1-e_q) on codes of -q * 2^e_q, so the
// accumulator seeded with ||r~||^2 yields ||r~||^2 - 2 q~.r~ of the
// dequantised values.
// ---------------------------------------------------------------------------
// Float minima of accumulator values use the NaN-propagating minimum
// (v_minimum3_f32): the accumulators are never NaN (finite FP8/16-bit
// products, finite or +inf seeds), so it equals the IEEE minNum there, and
// unlike minNum it takes raw operands without a canonicalising v_max first
// (16 values: 8 vector ops instead of 10; 8 values: 4 instead of 6).
static __device__ __forceinline__ float fmin_acc(float a, float b) { return __builtin_elementwise_minimum(a, b); }

static __device__ __forceinline__ float min16(const f32x16 &acc)
{
    const float m0 = fmin_acc(fmin_acc(acc[0], acc[1]), acc[2]);
    const float m1 = fmin_acc(fmin_acc(acc[3], acc[4]), acc[5]);
    const float m2 = fmin_acc(fmin_acc(acc[6], acc[7]), acc[8]);
    const float m3 = fmin_acc(fmin_acc(acc[9], acc[10]), acc[11]);
    const float m4 = fmin_acc(fmin_acc(acc[12], acc[13]), acc[14]);
    const float m5 = fmin_acc(fmin_acc(m0, m1), acc[15]);
    const float m6 = fmin_acc(fmin_acc(m2, m3), m4);
    return fmin_acc(m5, m6);
}

static __device__ __forceinline__ int min16(const i32x16 &a)
{
    const int m0 = min(min(a[0], a[1]), a[2]);
    const int m1 = min(min(a[3], a[4]), a[5]);
    const int m2 = min(min(a[6], a[7]), a[8]);
    const int m3 = min(min(a[9], a[10]), a[11]);
    const int m4 = min(min(a[12], a[13]), a[14]);
    const int mn = min(min(m0, m1), min(m2, m3));
    return min(min(mn, m4), a[15]);
}

// Chains of three-operand minima (v_min3 / v_minimum3): 4 vector ops for
// eight values, where a pairwise tree takes 5 (INT8) or, with minNum's
// canonicalising v_max on raw operands, 11 (float).
static __device__ __forceinline__ float min8(const f32x8 &a)
{
    const float m0 = fmin_acc(fmin_acc(a[0], a[1]), a[2]);
    const float m1 = fmin_acc(fmin_acc(a[3], a[4]), a[5]);
    const float m2 = fmin_acc(fmin_acc(m0, a[6]), a[7]);
    return fmin_acc(m2, m1);
}

static __device__ __forceinline__ int min8(const i32x8 &a)
{
    const int m0 = min(min(a[0], a[1]), a[2]);
    const int m1 = min(min(a[3], a[4]), a[5]);
    const int m2 = min(min(m0, a[6]), a[7]);
    return min(m2, m1);
}

// Float formats: the accumulator is the ranking key d' itself.  The gate
// compares a tile's smallest key with the list's KP-th key.
struct FloatKeys {
    static constexpr int kRow = kDim;     // elements per descriptor
    static constexpr bool kNbnn = false;  // per-class minima (original NBNN) instead of k+1 lists
    // 32x32 output blocks: lanes l and l+32 share query column l & 31; each
    // holds 16 rows of a tile, register r being row 8*(r/4) + 4*(l/32) + r%4
    static constexpr int kQT = 32;        // query columns per MFMA
    static constexpr int kGroups = 2;     // lanes (and so lists) per query
    static constexpr int kAccN = 16;      // accumulator registers per tile and query tile
    static constexpr int kRowStride = 8;  // row distance between register groups of four
    static constexpr int kMfma = 1;       // MFMA instructions per K step
    using acc_t = f32x16;
    using seed_t = f32x16;
    using gate_t = float;
    static constexpr bool kParity = false;
    static __device__ __forceinline__ float init() { return __builtin_inff(); }
    static __device__ __forceinline__ float gate_min(const f32x16 &acc) { return min16(acc); }
    static __device__ __forceinline__ float group_min(const f32x16 &a, int g)
    {
        return fmin_acc(fmin_acc(fmin_acc(a[4 * g], a[4 * g + 1]), a[4 * g + 2]), a[4 * g + 3]);
    }
    static __device__ __forceinline__ float gate_thr(float thr) { return thr; }
    static __device__ __forceinline__ float key(const f32x16 &acc, int r, uint32_t, int) { return acc[r]; }
    // key of one accumulator value of tile row `row` (one list per query)
    static __device__ __forceinline__ float key_at(float v, int, uint32_t) { return v; }
};

struct OpF16 : FloatKeys {
    static constexpr int kFmt = FMT_F16;
    static constexpr int kSteps = 8;
    static constexpr int kAU = 1;          // uint4 per lane per step
    static constexpr int kBU = 1;          // query uint4 per lane per step
    static constexpr bool kScaled = false;
    static __device__ __forceinline__ uint4 cvt8(uint2 raw, float mul)
    {
        f16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (_Float16)(mul * (float)byte_at(raw, e));
        return __builtin_bit_cast(uint4, v);
    }
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint8_t *qrow = static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim + 8 * h;
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            uint2 raw = make_uint2(0u, 0u);
            if (ok) raw = *reinterpret_cast<const uint2 *>(qrow + 16 * s);
            b[s][0] = cvt8(raw, -2.0f);
        }
        sb = 127;
    }
    // A fragment of K step s for one reference row (zeros past the end)
    static __device__ __forceinline__ uint4 pack_frag(const uint8_t *row, bool ok, int s, int h)
    {
        uint2 raw = make_uint2(0u, 0u);
        if (ok) raw = *reinterpret_cast<const uint2 *>(row + 16 * s + 8 * h);
        return cvt8(raw, 1.0f);
    }
    static __device__ __forceinline__ f32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], f32x16 c, int, int)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a[0]),
                                                      __builtin_bit_cast(f16x8, b[0]), c, 0, 0, 0);
    }
};

struct OpBF16 : FloatKeys {
    static constexpr int kFmt = FMT_BF16;
    static constexpr int kSteps = 8;
    static constexpr int kAU = 1;
    static constexpr int kBU = 1;
    static constexpr bool kScaled = false;
    static __device__ __forceinline__ uint4 cvt8(uint2 raw, float mul)
    {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)(mul * (float)byte_at(raw, e));
        return __builtin_bit_cast(uint4, v);
    }
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint8_t *qrow = static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim + 8 * h;
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            uint2 raw = make_uint2(0u, 0u);
            if (ok) raw = *reinterpret_cast<const uint2 *>(qrow + 16 * s);
            b[s][0] = cvt8(raw, -2.0f);
        }
        sb = 127;
    }
    // A fragment of K step s for one reference row (zeros past the end)
    static __device__ __forceinline__ uint4 pack_frag(const uint8_t *row, bool ok, int s, int h)
    {
        uint2 raw = make_uint2(0u, 0u);
        if (ok) raw = *reinterpret_cast<const uint2 *>(row + 16 * s + 8 * h);
        return cvt8(raw, 1.0f);
    }
    static __device__ __forceinline__ f32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], f32x16 c, int, int)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                       __builtin_bit_cast(bf16x8, b[0]), c, 0, 0, 0);
    }
};

struct OpFP8 : FloatKeys {
    static constexpr int kFmt = FMT_FP8;
    static constexpr int kSteps = 2;
    static constexpr int kAU = 2;
    static constexpr int kBU = 2;
    static constexpr bool kScaled = true;
    // queries: FP8 codes [n_q][128] in natural K order, E8M0 scale per query
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *qsc, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim);
#pragma unroll
        for (int s = 0; s < kSteps; ++s)
#pragma unroll
            for (int u = 0; u < kAU; ++u) b[s][u] = ok ? qrow[4 * s + 2 * h + u] : make_uint4(0u, 0u, 0u, 0u);
        sb = ok ? qsc[qi] : 127;
    }
    static __device__ __forceinline__ f32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], f32x16 c, int sa,
                                                 int sb)
    {
        i32x8 av, bv;
        av[0] = (int)a[0].x; av[1] = (int)a[0].y; av[2] = (int)a[0].z; av[3] = (int)a[0].w;
        av[4] = (int)a[1].x; av[5] = (int)a[1].y; av[6] = (int)a[1].z; av[7] = (int)a[1].w;
        bv[0] = (int)b[0].x; bv[1] = (int)b[0].y; bv[2] = (int)b[0].z; bv[3] = (int)b[0].w;
        bv[4] = (int)b[1].x; bv[5] = (int)b[1].y; bv[6] = (int)b[1].z; bv[7] = (int)b[1].w;
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, sa, 0, sb);
    }
};

// INT8 (v_mfma_i32_32x32x32_i8, INT32 accumulation: exact).  With s = r - 128
// and t = q - 128 (both int8), ||q - r||^2 = ||t - s||^2 = ||t||^2 + key with
//     key = ||s||^2 - 2 t.s,
// a per-query shift of the squared distance.  The factor 2 does not fit an
// int8 operand, so the accumulator carries
//     D = floor(||s||^2 / 2) - t.s,   key = 2 D + b,   b = ||s||^2 mod 2,
// from the seed floor(||s||^2 / 2) + sum(s) and the query operand
// u = 127 - q = -t - 1 (so u.s = -t.s - sum(s)).  |D| < 2^22, so every
// key is an exact FP32 integer.  The per-row bit b lives in a per-tile
// mask that only the (rare) insertion path reads.  A K step covers 32
// elements: lane l supplies 16 bytes of row (l & 31), K elements
// 32*s + 16*(l >> 5) + e.  Padding rows carry the seed 2^30, whose D never
// makes a key (see key()).  S K steps: S = 4 for 128-element rows, S = 5
// for the 160-element location-augmented rows (|D| < 2^23 there, and every
// key and distance stays below 2^24, still exact in FP32).
// NBN: the class-sorted index of the original NBNN rule (Algorithm 1): the
// kernel keeps each query's running minimum key per class instead of a
// neighbour list (see k_dist_topk).
template <int S, int FMT, bool NBN = false>
struct OpI8T {
    static constexpr int kFmt = FMT;
    static constexpr bool kNbnn = NBN;
    static constexpr int kSteps = S;
    static constexpr int kRow = 32 * S;      // bytes per descriptor
    static constexpr int kAU = 1;
    static constexpr int kBU = 1;
    static constexpr bool kScaled = false;
    static constexpr int kQT = 32;           // as for the float formats
    static constexpr int kGroups = 2;
    static constexpr int kAccN = 16;
    static constexpr int kRowStride = 8;
    static constexpr int kMfma = 1;
    using acc_t = i32x16;
    using seed_t = f32x16;
    using gate_t = int;
    static constexpr bool kParity = true;
    static constexpr int kPadSeed = 1 << 30;
    static __device__ __forceinline__ int init() { return 0x7fffffff; }
    static __device__ __forceinline__ int gate_min(const i32x16 &acc) { return min16(acc); }
    static __device__ __forceinline__ int group_min(const i32x16 &a, int g)
    {
        return min(min(min(a[4 * g], a[4 * g + 1]), a[4 * g + 2]), a[4 * g + 3]);
    }
    // key = 2D + b < thr implies D < ceil(thr / 2); no bound while the list
    // is not full (thr = +inf)
    static __device__ __forceinline__ int gate_thr(float thr)
    {
        return thr < 1e30f ? (int)__builtin_ceilf(0.5f * thr) : 0x7fffffff;
    }
    static __device__ __forceinline__ float key(const i32x16 &acc, int r, uint32_t parity, int h)
    {
        const int d = acc[r];
        const int row = 8 * (r >> 2) + 4 * h + (r & 3);
        return d >= (1 << 29) ? __builtin_inff() : (float)(2 * d + (int)((parity >> row) & 1u));
    }
    static __device__ __forceinline__ float key_at(int d, int row, uint32_t parity)
    {
        return d >= (1 << 29) ? __builtin_inff() : (float)(2 * d + (int)((parity >> row) & 1u));
    }
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kRow);
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            // bytes 127 - q: q ^ 0x7f reads as that int8 for every q in 0..255
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (ok) v = qrow[2 * s + h];
            const uint32_t m = 0x7f7f7f7fu;
            b[s][0] = ok ? make_uint4(v.x ^ m, v.y ^ m, v.z ^ m, v.w ^ m) : make_uint4(0u, 0u, 0u, 0u);
        }
        sb = 127;
    }
    static __device__ __forceinline__ uint4 pack_frag(const uint8_t *row, bool ok, int s, int h)
    {
        // bytes r ^ 0x80 read as the int8 r - 128
        if (!ok) return make_uint4(0u, 0u, 0u, 0u);
        const uint4 v = *reinterpret_cast<const uint4 *>(row + 32 * s + 16 * h);
        const uint32_t m = 0x80808080u;
        return make_uint4(v.x ^ m, v.y ^ m, v.z ^ m, v.w ^ m);
    }
    static __device__ __forceinline__ i32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], i32x16 c, int, int)
    {
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i32x4v, a[0]), __builtin_bit_cast(i32x4v, b[0]),
                                                     c, 0, 0, 0);
    }
};
using OpI8 = OpI8T<4, FMT_I8>;
using OpI8L = OpI8T<5, FMT_I8L>;
using OpI8N = OpI8T<4, FMT_I8N, true>;

// 16x16 output blocks (v_mfma_i32_16x16x64_i8, v_mfma_f32_16x16x32_{f16,bf16}).
// A 32-row tile is two 16-row blocks b = 0, 1; lane l holds query column
// l & 15, and register 4b + i is row 16b + 4*(l/16) + i, so four lanes (and
// four lists) share each query.  Each block MFMA reads K elements
// K0 + 16*(l/16) + e (INT8, e < 16) or K0 + 8*(l/16) + e (16-bit, e < 8) of
// row 16b + (l & 15): in the 32x32 packing that chunk sits in K step
// 2 s + (l/16)/2, lane 16 b + (l & 15) + 32 ((l/16) & 1), so both shapes read
// the same packed index.
template <class Op>
static __device__ __forceinline__ int frag_off(int s, int u, int lane)
{
    if constexpr (Op::kQT == 16 && Op::kScaled) {
        // FP8: u = 2 * (row block) + (16-byte half); one K step
        const int g = lane >> 4;
        return (2 * (g >> 1) + (u & 1)) * 64 + 16 * (u >> 1) + (lane & 15) + 32 * (g & 1);
    } else if constexpr (Op::kQT == 16) {
        const int g = lane >> 4;
        return (2 * s + (g >> 1)) * 64 + 16 * u + (lane & 15) + 32 * (g & 1);
    } else {
        return (s * Op::kAU + u) * 64 + lane;
    }
}

template <int FMT, bool NBN>
struct OpI8Q : OpI8T<4, FMT, NBN> {
    using Base = OpI8T<4, FMT, NBN>;
    static constexpr int kSteps = 2;         // K = 64 per step
    static constexpr int kAU = 2;            // one uint4 per row block
    static constexpr int kBU = 1;
    static constexpr int kQT = 16;
    static constexpr int kGroups = 4;
    static constexpr int kAccN = 8;
    static constexpr int kRowStride = 16;
    static constexpr int kMfma = 2;
    using acc_t = i32x8;
    using seed_t = f32x8;
    static __device__ __forceinline__ int gate_min(const i32x8 &acc) { return min8(acc); }
    static __device__ __forceinline__ int group_min(const i32x8 &a, int g)
    {
        return min(min(min(a[4 * g], a[4 * g + 1]), a[4 * g + 2]), a[4 * g + 3]);
    }
    static __device__ __forceinline__ float key(const i32x8 &acc, int r, uint32_t parity, int h)
    {
        const int d = acc[r];
        const int row = 16 * (r >> 2) + 4 * h + (r & 3);
        return d >= (1 << 29) ? __builtin_inff() : (float)(2 * d + (int)((parity >> row) & 1u));
    }
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim);
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (ok) v = qrow[4 * s + h];
            const uint32_t m = 0x7f7f7f7fu;
            b[s][0] = ok ? make_uint4(v.x ^ m, v.y ^ m, v.z ^ m, v.w ^ m) : make_uint4(0u, 0u, 0u, 0u);
        }
        sb = 127;
    }
    static __device__ __forceinline__ i32x8 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], i32x8 c, int, int)
    {
        const i32x4v bv = __builtin_bit_cast(i32x4v, b[0]);
        const i32x4v lo = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i32x4v, a[0]), bv,
                                                                __builtin_shufflevector(c, c, 0, 1, 2, 3), 0, 0, 0);
        const i32x4v hi = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i32x4v, a[1]), bv,
                                                                __builtin_shufflevector(c, c, 4, 5, 6, 7), 0, 0, 0);
        return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    }
};

// Members of the 16x16 layout shared by the float formats.
template <class Base>
struct FloatQ : Base {
    static constexpr int kQT = 16;
    static constexpr int kGroups = 4;
    static constexpr int kAccN = 8;
    static constexpr int kRowStride = 16;
    static constexpr int kMfma = 2;
    using acc_t = f32x8;
    using seed_t = f32x8;
    static __device__ __forceinline__ float gate_min(const f32x8 &acc) { return min8(acc); }
    static __device__ __forceinline__ float group_min(const f32x8 &a, int g)
    {
        return fmin_acc(fmin_acc(fmin_acc(a[4 * g], a[4 * g + 1]), a[4 * g + 2]), a[4 * g + 3]);
    }
    static __device__ __forceinline__ float key(const f32x8 &acc, int r, uint32_t, int) { return acc[r]; }
};

template <class Base16, bool BF>
struct OpH16Q : FloatQ<Base16> {
    static constexpr int kSteps = 4;         // K = 32 per step
    static constexpr int kAU = 2;
    static constexpr int kBU = 1;
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint8_t *qrow = static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim + 8 * h;
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            uint2 raw = make_uint2(0u, 0u);
            if (ok) raw = *reinterpret_cast<const uint2 *>(qrow + 32 * s);
            b[s][0] = Base16::cvt8(raw, -2.0f);
        }
        sb = 127;
    }
    static __device__ __forceinline__ f32x8 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], f32x8 c, int, int)
    {
        f32x4v lo, hi;
        if constexpr (BF) {
            const bf16x8 bv = __builtin_bit_cast(bf16x8, b[0]);
            lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[0]), bv,
                                                         __builtin_shufflevector(c, c, 0, 1, 2, 3), 0, 0, 0);
            hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[1]), bv,
                                                         __builtin_shufflevector(c, c, 4, 5, 6, 7), 0, 0, 0);
        } else {
            const f16x8 bv = __builtin_bit_cast(f16x8, b[0]);
            lo = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a[0]), bv,
                                                        __builtin_shufflevector(c, c, 0, 1, 2, 3), 0, 0, 0);
            hi = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a[1]), bv,
                                                        __builtin_shufflevector(c, c, 4, 5, 6, 7), 0, 0, 0);
        }
        return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    }
};

// FP8, 16x16 blocks (v_mfma_scale_f32_16x16x128_f8f6f4: the whole K = 128
// in one instruction per 16-row block).  Lane l supplies 32 codes of row
// 16 b + (l & 15), K elements 32 (l/16) + e: in the 32x32 packing those are
// the two 16-byte chunks of K step (l/16)/2 at lane 32 ((l/16) & 1) + 16 b +
// (l & 15), so both shapes read the same packed index.  The two blocks' E8M0
// row scales travel in bytes 0 and 1 of one register, picked by the scale
// byte select of each block's instruction.
struct OpFP8Q : FloatQ<OpFP8> {
    static constexpr int kSteps = 1;
    static constexpr int kAU = 4;            // (row block, 16-byte half)
    static constexpr int kBU = 2;
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *qsc, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kBU], int &sb)
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim);
#pragma unroll
        for (int u = 0; u < kBU; ++u) b[0][u] = ok ? qrow[2 * h + u] : make_uint4(0u, 0u, 0u, 0u);
        sb = ok ? qsc[qi] : 127;
    }
    static __device__ __forceinline__ i32x8 cat(const uint4 &x, const uint4 &y)
    {
        i32x8 v;
        v[0] = (int)x.x; v[1] = (int)x.y; v[2] = (int)x.z; v[3] = (int)x.w;
        v[4] = (int)y.x; v[5] = (int)y.y; v[6] = (int)y.z; v[7] = (int)y.w;
        return v;
    }
    static __device__ __forceinline__ f32x8 mma(const uint4 (&a)[kAU], const uint4 (&b)[kBU], f32x8 c, int sa,
                                                int sb)
    {
        const i32x8 bv = cat(b[0], b[1]);
        const f32x4v lo = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
            cat(a[0], a[1]), bv, __builtin_shufflevector(c, c, 0, 1, 2, 3), 0, 0, 0, sa, 0, sb);
        const f32x4v hi = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
            cat(a[2], a[3]), bv, __builtin_shufflevector(c, c, 4, 5, 6, 7), 0, 0, 1, sa, 0, sb);
        return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    }
};

// The 16x16 form of each operand policy that has one (void: none).
template <class Op> struct Square16 { using type = void; };
template <> struct Square16<OpI8> { using type = OpI8Q<FMT_I8, false>; };
template <> struct Square16<OpI8N> { using type = OpI8Q<FMT_I8N, true>; };
template <> struct Square16<OpF16> { using type = OpH16Q<OpF16, false>; };
template <> struct Square16<OpBF16> { using type = OpH16Q<OpBF16, true>; };
template <> struct Square16<OpFP8> { using type = OpFP8Q; };

// ---------------------------------------------------------------------------
// K1: distances + top-(k+1).
//
// Work item = (query block of W * kQT * NT queries, reference slice).
// Each wave keeps kQT*NT queries' operand fragments in registers; the
// workgroup streams 32-row reference tiles through NB LDS stages of MT
// tiles.  With references as the MFMA M dimension and queries as N, lane l's
// accumulator registers are references of one query: in the 32x32 shape 16
// registers, column l & 31, register r being row 8*(r/4) + 4*(l/32) + r%4;
// in the 16x16 shape 8 registers, column l & 15, row 16*(r/4) + 4*(l/16) + r%4.
//
// Selection.  Each lane keeps a sorted register list of the KP best
// (d', index) pairs of its query among the rows it has seen (the kGroups
// lanes of a query each see their share of every tile and keep separate
// lists).  A tile is gated by the minimum of the lane's values: only when
// some lane of the wave beats its current KP-th value does the wave walk the
// registers and insert.  Rows reach a lane in increasing index order, so "strictly less
// than" on d' alone realises the (distance, index) order.
//
// Original NBNN (Op::kNbnn, Algorithm 1).  The index holds the references
// sorted by class, every class padded to a multiple of 8 tiles, so a class
// boundary is always a stage boundary.  The list is one entry long: the
// query's smallest key in the current class.  When a stage starts a new
// class (and at the end of an item), the entry is flushed into
// cls_min[class][query] with an atomic minimum and reset; slices and chunks
// of one class therefore combine exactly.
// ---------------------------------------------------------------------------
template <int KP>
static __device__ __forceinline__ void list_insert(float v, int idx, float (&ld)[KP], int (&li)[KP],
                                                   float &thr)
{
#pragma unroll
    for (int p = KP - 1; p > 0; --p) {
        const bool shift = v < ld[p - 1];
        const bool here = v < ld[p];
        const float nd = shift ? ld[p - 1] : (here ? v : ld[p]);
        const int ni = shift ? li[p - 1] : (here ? idx : li[p]);
        ld[p] = nd;
        li[p] = ni;
    }
    const bool first = v < ld[0];
    ld[0] = first ? v : ld[0];
    li[0] = first ? idx : li[0];
    thr = ld[KP - 1];
}

// Load through the scalar cache (uniform index).
static __device__ __forceinline__ uint32_t load_uniform(const uint32_t *p, int i)
{
    return ((const __attribute__((address_space(4))) uint32_t *)p)[i];
}

// Insert every key of one tile that beats the list's current KP-th key;
// gt is the gate threshold that goes with the list's new KP-th key.
template <class Op, int KP>
static __device__ __forceinline__ void tile_insert(const typename Op::acc_t &acc, float &thr,
                                                   typename Op::gate_t &gt,
                                                   float (&ld)[KP], int (&li)[KP], int row0, int h,
                                                   const uint32_t *parity)
{
    uint32_t pm = 0;
    if constexpr (Op::kParity) pm = load_uniform(parity, __builtin_amdgcn_readfirstlane(row0 >> 5));
    // the row base is made opaque here so the 16 index computations stay on
    // this (rarely taken) path instead of being hoisted into the gate
    int base = row0;
    asm volatile("" : "+v"(base));
    // registers 4g..4g+3 hold rows kRowStride*g + 4h + 0..3: only the groups
    // whose minimum passes the gate are walked (usually one)
#pragma unroll
    for (int g = 0; g < Op::kAccN / 4; ++g) {
        if (__builtin_amdgcn_ballot_w64(Op::group_min(acc, g) < gt) == 0) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * g + i;
            const float v = Op::key(acc, r, pm, h);
            const bool take = v < thr;
            if (__builtin_amdgcn_ballot_w64(take) != 0) {
                if (take) list_insert<KP>(v, base + Op::kRowStride * g + i, ld, li, thr);
            }
        }
    }
    gt = Op::gate_thr(thr);
}

static __device__ __forceinline__ float lmin(float a, float b) { return __builtin_fminf(a, b); }
static __device__ __forceinline__ int lmin(int a, int b) { return min(a, b); }

template <class Op> using AccT = typename Op::acc_t;
template <class Op, int NT> using AccArr = typename Op::acc_t[NT];

// Lists each lane keeps: one per query tile, or (PL, shared lists) one for the
// query it owns.
template <bool PL, int NT>
constexpr int lists_per_lane() { return PL ? 1 : NT; }

// Shared lists: the kGroups lanes of a query (2 with 32x32 blocks, 4 with
// 16x16) keep one list, held by one of them, over NT = kGroups query tiles:
// lane l owns the list of query (tile l / kQT, column l % kQT), which sees
// every row of every tile.  Its values of a tile sit in the kGroups lanes of
// its column, each in the accumulator of its query tile, so the insertion
// path first transposes the accumulators across the lane groups in place
// (the accumulators are dead after their gate): one v_permlane32_swap round
// for two groups; for four, a v_permlane32_swap round (tiles j, j+2) and a
// v_permlane16_swap round (tiles 2k, 2k+1).  Then every lane holds its own
// query's values, acc[j] register r being row kRowStride*(r/4) + 4j + r%4.
// The gate needs no exchange: each lane compares its values of tile nt with
// the gate threshold of that tile's query (gq[nt], exchanged after every
// insertion).
template <class Op>
static __device__ __forceinline__ void swap_lanes32(AccT<Op> &x, AccT<Op> &y)
{
    using E = typename Op::gate_t;                 // accumulator element type
#pragma unroll
    for (int r = 0; r < Op::kAccN; ++r) {
        const auto p = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, (E)x[r]),
                                                        __builtin_bit_cast(uint32_t, (E)y[r]), false, false);
        x[r] = __builtin_bit_cast(E, (uint32_t)p[0]);
        y[r] = __builtin_bit_cast(E, (uint32_t)p[1]);
    }
}

template <class Op>
static __device__ __forceinline__ void swap_lanes16(AccT<Op> &x, AccT<Op> &y)
{
    using E = typename Op::gate_t;
#pragma unroll
    for (int r = 0; r < Op::kAccN; ++r) {
        const auto p = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(uint32_t, (E)x[r]),
                                                        __builtin_bit_cast(uint32_t, (E)y[r]), false, false);
        x[r] = __builtin_bit_cast(E, (uint32_t)p[0]);
        y[r] = __builtin_bit_cast(E, (uint32_t)p[1]);
    }
}

// the gate thresholds of the query tiles' queries, from their owner lanes
template <class Op, int NT>
static __device__ __forceinline__ void share_gate_thr(typename Op::gate_t gt, typename Op::gate_t (&gq)[NT], int col)
{
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) gq[nt] = __shfl(gt, Op::kQT * nt + col);
}

template <class Op, int KP, int NT>
static __device__ __forceinline__ void tile_insert_pl(AccArr<Op, NT> &acc, float &thr, typename Op::gate_t &gt,
                                                      typename Op::gate_t (&gq)[NT], float (&ld)[KP], int (&li)[KP],
                                                      int row0, int col, const uint32_t *parity)
{
    static_assert(NT == Op::kGroups && (NT == 2 || NT == 4), "one query tile per lane group");
    if constexpr (NT == 2) {
        swap_lanes32<Op>(acc[0], acc[1]);
    } else {
        swap_lanes32<Op>(acc[0], acc[2]);
        swap_lanes32<Op>(acc[1], acc[3]);
        swap_lanes16<Op>(acc[0], acc[1]);
        swap_lanes16<Op>(acc[2], acc[3]);
    }
    uint32_t pm = 0;
    if constexpr (Op::kParity) pm = load_uniform(parity, __builtin_amdgcn_readfirstlane(row0 >> 5));
    int base = row0;                               // opaque, as in tile_insert
    asm volatile("" : "+v"(base));
#pragma unroll
    for (int g = 0; g < Op::kAccN / 4; ++g) {
        typename Op::gate_t m = Op::group_min(acc[0], g);
#pragma unroll
        for (int j = 1; j < NT; ++j) m = lmin(m, Op::group_min(acc[j], g));
        if (__builtin_amdgcn_ballot_w64(m < gt) == 0) continue;
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = Op::kRowStride * g + 4 * j + i;
                const float v = Op::key_at(acc[j][4 * g + i], row, pm);
                const bool take = v < thr;
                if (__builtin_amdgcn_ballot_w64(take) != 0) {
                    if (take) list_insert<KP>(v, base + row, ld, li, thr);
                }
            }
    }
    gt = Op::gate_thr(thr);
    share_gate_thr<Op, NT>(gt, gq, col);
}

// Gate of the NT query tiles of one reference tile: does some lane hold a
// value below its list's gate threshold?  (Shared lists: one answer for all
// tiles, in any[0].)
template <class Op, int NT, bool PL>
static __device__ __forceinline__ void gate_any(const typename Op::acc_t (&acc)[NT],
                                                const typename Op::gate_t (&gt)[lists_per_lane<PL, NT>()],
                                                const typename Op::gate_t (&gq)[NT], bool (&any)[NT])
{
    if constexpr (PL) {
        bool below = Op::gate_min(acc[0]) < gq[0];
#pragma unroll
        for (int nt = 1; nt < NT; ++nt) below = below | (Op::gate_min(acc[nt]) < gq[nt]);
        any[0] = __builtin_amdgcn_ballot_w64(below) != 0;
#pragma unroll
        for (int nt = 1; nt < NT; ++nt) any[nt] = false;
    } else {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) any[nt] = __builtin_amdgcn_ballot_w64(Op::gate_min(acc[nt]) < gt[nt]) != 0;
    }
}

// Insertions for the tiles whose gate passed (rare).
template <class Op, int KP, int NT, bool PL>
static __device__ __forceinline__ void gate_insert(AccArr<Op, NT> &acc, const bool (&any)[NT],
                                                   float (&thr)[lists_per_lane<PL, NT>()],
                                                   typename Op::gate_t (&gt)[lists_per_lane<PL, NT>()],
                                                   typename Op::gate_t (&gq)[NT],
                                                   float (&ld)[lists_per_lane<PL, NT>()][KP],
                                                   int (&li)[lists_per_lane<PL, NT>()][KP], int row0, int h,
                                                   const uint32_t *parity)
{
    if constexpr (PL) {
        if (__builtin_expect(any[0], 0))
            tile_insert_pl<Op, KP, NT>(acc, thr[0], gt[0], gq, ld[0], li[0], row0,
                                       (int)(threadIdx.x & (Op::kQT - 1)), parity);
    } else {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            if (__builtin_expect(any[nt], 0))
                tile_insert<Op, KP>(acc[nt], thr[nt], gt[nt], ld[nt], li[nt], row0, h, parity);
    }
}

// Original NBNN: one running minimum key per query tile (in mk), no list.
// Every stage of the class-sorted copy holds one class and one parity of
// ||r - 128||^2, so the smallest exact key of a tile's rows is
// 2 x (the smallest accumulator value) + that parity.  Padding rows (seed
// 2^30) are clamped to 2^28 first: their keys stay above every real key and
// no sum overflows.  The update sits behind a wave-uniform branch, taken
// only when some lane improves: written branch-free, the pipelined loop was
// allocated differently and spilled the query operands.
template <class Op, int NT>
static __device__ __forceinline__ void nbnn_tile_min(const AccArr<Op, NT> &acc, typename Op::gate_t (&mk)[NT],
                                                     int par)
{
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int key = 2 * min(Op::gate_min(acc[nt]), 1 << 28) + par;
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(key < mk[nt]) != 0, 0)) mk[nt] = min(mk[nt], key);
    }
}

// Gate + insert for the NT query tiles of one reference tile.  All gates
// are computed before any branch so they can overlap the next MFMA chain.
// (Original NBNN: the running minimum keys instead.)
template <class Op, int KP, int NT, bool PL>
static __device__ __forceinline__ void tiles_select(AccArr<Op, NT> &acc,
                                                    float (&thr)[lists_per_lane<PL, NT>()],
                                                    typename Op::gate_t (&gt)[lists_per_lane<PL, NT>()],
                                                    typename Op::gate_t (&gq)[NT],
                                                    float (&ld)[lists_per_lane<PL, NT>()][KP],
                                                    int (&li)[lists_per_lane<PL, NT>()][KP], int row0, int h,
                                                    const uint32_t *parity, int nb_par = 0)
{
    if constexpr (Op::kNbnn) {
        nbnn_tile_min<Op, NT>(acc, gq, nb_par);
    } else {
        bool any[NT];
        gate_any<Op, NT, PL>(acc, gt, gq, any);
        gate_insert<Op, KP, NT, PL>(acc, any, thr, gt, gq, ld, li, row0, h, parity);
    }
}


// Asynchronous copy of one LDS stage (MT tiles of fragments, their seeds
// and, for scaled formats, their row scales) straight from global memory into
// LDS (global_load_lds).  A fragment instruction moves 64 lanes x 16 B to
// consecutive LDS addresses; every wave also copies its share of the
// stage's MT*32 seeds (and scales) with one partial-lane 4-byte instruction.
// Each wave therefore issues exactly StageLoads::total instructions per
// stage, which is what the vmcnt waits count on.
template <class Op, int MT, int W>
struct StageLoads {
    static constexpr int tile_chunks = Op::kSteps * Op::kAU;           // 1 KB chunks per tile
    static constexpr int frag = MT * tile_chunks / W;                  // chunks per wave
    static_assert(frag * W == MT * tile_chunks, "stage chunks must split evenly over the waves");
    static constexpr int seeds_per_wave = MT * kTileRows / W;
    static_assert(seeds_per_wave <= 64 && seeds_per_wave * W == MT * kTileRows, "seed split");
    static constexpr int total = frag + 1 + (Op::kScaled ? 1 : 0);
};

static __device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)p;
}

// Asynchronous global-to-LDS copies (global_load_lds: every lane moves its
// bytes to M0 + lane * size), written as inline assembly so that the
// compiler does not count them against its own LDS accesses: it would
// otherwise make every LDS read wait for all copies in flight, including
// the prefetch of later stages.  The stage loop orders each read after the
// copy it needs with its own vmcnt wait and barrier.  One wait state
// separates the M0 write from the copy.
static __device__ __forceinline__ void dma16(const void *src, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off"
                 :: "s"(lds), "v"(src) : "memory", "m0");
}

static __device__ __forceinline__ void dma4(const void *src, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dword %1, off"
                 :: "s"(lds), "v"(src) : "memory", "m0");
}

template <class Op, int MT, int W, int TILE_U4>
static __device__ __forceinline__ void stage_copy(const uint4 *src, uint4 *dst, const float *seed_src, float *seed_dst,
                                                  const int32_t *rsc_src, int32_t *rsc_dst, int wave, int lane)
{
    using SL = StageLoads<Op, MT, W>;
#pragma unroll
    for (int c = 0; c < SL::frag; ++c) {
        const int chunk = c * W + wave;
        dma16(src + chunk * 64 + lane, lds_addr(dst + chunk * 64));
    }
    const int s0 = wave * SL::seeds_per_wave;
    if (lane < SL::seeds_per_wave) dma4(seed_src + s0 + lane, lds_addr(seed_dst + s0));
    if constexpr (Op::kScaled) {
        if (lane < SL::seeds_per_wave) dma4(rsc_src + s0 + lane, lds_addr(rsc_dst + s0));
    }
}

// s_waitcnt with only the vector-memory counter limited (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at maximum).
template <int N>
static __device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));


// All LDS reads of one tile (A fragments, seeds, row scales) as one block
// that also waits for them.  The compiler cannot tell which of the stage
// buffers an asynchronous global-to-LDS copy is still filling, so reads it
// emits itself would wait for every copy in flight, including the prefetch
// of later stages; the stage loop's own vmcnt wait and barrier already
// order each read after the copy it needs.
template <class Op>
static __device__ __forceinline__ void tile_reads(const uint4 *frag, const float4 *seed, const int32_t *rsc,
                                                  int lane, int h, uint4 (&av)[Op::kSteps][Op::kAU],
                                                  typename Op::seed_t &sd, int &sa)
{
    const uint32_t fa = lds_addr(frag + frag_off<Op>(0, 0, lane));
    const uint32_t ea = lds_addr(seed + h);
    u32x4 a0, a1, a2, a3, a4, a5, a6, a7;
    f32x4 s0, s1, s2, s3;
    if constexpr (Op::kQT == 16 && Op::kScaled) {
        // FP8, 16x16 blocks: (row block b, half j) at byte offset 256 b +
        // 1024 j from the lane's base; the two blocks' row scales 64 bytes apart
        static_assert(Op::kSteps == 1 && Op::kAU == 4, "16x16 FP8 layout");
        const uint32_t ra = lds_addr(rsc + (lane & 15));
        int r0, r1;
        asm volatile(
            "ds_read_b128 %0, %8\n\t"
            "ds_read_b128 %1, %8 offset:1024\n\t"
            "ds_read_b128 %2, %8 offset:256\n\t"
            "ds_read_b128 %3, %8 offset:1280\n\t"
            "ds_read_b128 %4, %9\n\t"
            "ds_read_b128 %5, %9 offset:64\n\t"
            "ds_read_b32 %6, %10\n\t"
            "ds_read_b32 %7, %10 offset:64\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(s0), "=&v"(s1), "=&v"(r0), "=&v"(r1)
            : "v"(fa), "v"(ea), "v"(ra)
            : "memory");
        av[0][0] = __builtin_bit_cast(uint4, a0);
        av[0][1] = __builtin_bit_cast(uint4, a1);
        av[0][2] = __builtin_bit_cast(uint4, a2);
        av[0][3] = __builtin_bit_cast(uint4, a3);
        sa = r0 | (r1 << 8);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sd[j] = s0[j];
            sd[4 + j] = s1[j];
        }
        return;
    } else if constexpr (Op::kQT == 16) {
        // 16-bit formats, 16x16 blocks: K step s, row block u at byte
        // offset 2048 s + 256 u from the lane's base; the lane's two seed
        // groups are 64 bytes apart
        static_assert(Op::kSteps == 4 && Op::kAU == 2 && !Op::kScaled, "16x16 16-bit layout");
        asm volatile(
            "ds_read_b128 %0, %10\n\t"
            "ds_read_b128 %1, %10 offset:256\n\t"
            "ds_read_b128 %2, %10 offset:2048\n\t"
            "ds_read_b128 %3, %10 offset:2304\n\t"
            "ds_read_b128 %4, %10 offset:4096\n\t"
            "ds_read_b128 %5, %10 offset:4352\n\t"
            "ds_read_b128 %6, %10 offset:6144\n\t"
            "ds_read_b128 %7, %10 offset:6400\n\t"
            "ds_read_b128 %8, %11\n\t"
            "ds_read_b128 %9, %11 offset:64\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(a4), "=&v"(a5), "=&v"(a6), "=&v"(a7),
              "=&v"(s0), "=&v"(s1)
            : "v"(fa), "v"(ea)
            : "memory");
        const u32x4 a[8] = {a0, a1, a2, a3, a4, a5, a6, a7};
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int u = 0; u < 2; ++u) av[s][u] = __builtin_bit_cast(uint4, a[2 * s + u]);
        sa = 127;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sd[j] = s0[j];
            sd[4 + j] = s1[j];
        }
        return;
    } else if constexpr (Op::kSteps * Op::kAU == 8) {
        static_assert(!Op::kScaled, "unscaled formats only");
        asm volatile(
            "ds_read_b128 %0, %12\n\t"
            "ds_read_b128 %1, %12 offset:1024\n\t"
            "ds_read_b128 %2, %12 offset:2048\n\t"
            "ds_read_b128 %3, %12 offset:3072\n\t"
            "ds_read_b128 %4, %12 offset:4096\n\t"
            "ds_read_b128 %5, %12 offset:5120\n\t"
            "ds_read_b128 %6, %12 offset:6144\n\t"
            "ds_read_b128 %7, %12 offset:7168\n\t"
            "ds_read_b128 %8, %13\n\t"
            "ds_read_b128 %9, %13 offset:32\n\t"
            "ds_read_b128 %10, %13 offset:64\n\t"
            "ds_read_b128 %11, %13 offset:96\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(a4), "=&v"(a5), "=&v"(a6), "=&v"(a7),
              "=&v"(s0), "=&v"(s1), "=&v"(s2), "=&v"(s3)
            : "v"(fa), "v"(ea)
            : "memory");
        const u32x4 a[8] = {a0, a1, a2, a3, a4, a5, a6, a7};
#pragma unroll
        for (int s = 0; s < 8; ++s) av[s][0] = __builtin_bit_cast(uint4, a[s]);
        sa = 127;
    } else if constexpr (!Op::kScaled) {
        static_assert(Op::kSteps * Op::kAU == 4, "INT8 layout");
        asm volatile(
            "ds_read_b128 %0, %8\n\t"
            "ds_read_b128 %1, %8 offset:1024\n\t"
            "ds_read_b128 %2, %8 offset:2048\n\t"
            "ds_read_b128 %3, %8 offset:3072\n\t"
            "ds_read_b128 %4, %9\n\t"
            "ds_read_b128 %5, %9 offset:32\n\t"
            "ds_read_b128 %6, %9 offset:64\n\t"
            "ds_read_b128 %7, %9 offset:96\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(s0), "=&v"(s1), "=&v"(s2), "=&v"(s3)
            : "v"(fa), "v"(ea)
            : "memory");
        const u32x4 a[4] = {a0, a1, a2, a3};
#pragma unroll
        for (int s = 0; s < 4; ++s) av[s][0] = __builtin_bit_cast(uint4, a[s]);
        sa = 127;
    } else {
        static_assert(Op::kSteps * Op::kAU == 4 && Op::kScaled, "FP8 layout");
        const uint32_t ra = lds_addr(rsc + (lane & 31));
        int r;
        asm volatile(
            "ds_read_b128 %0, %9\n\t"
            "ds_read_b128 %1, %9 offset:1024\n\t"
            "ds_read_b128 %2, %9 offset:2048\n\t"
            "ds_read_b128 %3, %9 offset:3072\n\t"
            "ds_read_b128 %4, %10\n\t"
            "ds_read_b128 %5, %10 offset:32\n\t"
            "ds_read_b128 %6, %10 offset:64\n\t"
            "ds_read_b128 %7, %10 offset:96\n\t"
            "ds_read_b32 %8, %11\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(s0), "=&v"(s1), "=&v"(s2), "=&v"(s3), "=&v"(r)
            : "v"(fa), "v"(ea), "v"(ra)
            : "memory");
        av[0][0] = __builtin_bit_cast(uint4, a0);
        av[0][1] = __builtin_bit_cast(uint4, a1);
        av[1][0] = __builtin_bit_cast(uint4, a2);
        av[1][1] = __builtin_bit_cast(uint4, a3);
        sa = r;
    }
    if constexpr (Op::kQT == 32) {
        const f32x4 sv[4] = {s0, s1, s2, s3};
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int j = 0; j < 4; ++j) sd[4 * g + j] = sv[g][j];
    }
}

#ifndef LNBNN_MFMA_BEFORE_INSERT
#define LNBNN_MFMA_BEFORE_INSERT 1
#endif

// An empty asm that takes the accumulators as inputs: the instructions that
// produce them must issue before it.
template <class Op, int NT>
static __device__ __forceinline__ void pin_acc(const AccArr<Op, NT> &acc)
{
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) asm volatile("" ::"v"(acc[nt]));
#endif
}

// One pipeline step: the MFMA chain of a new tile (into acc_new) and the
// gate of the previous tile (acc_old), scheduled as one block: all LDS reads
// of the new tile first, then MFMAs interleaved with the gate's vector ops.
// Insertions for the previous tile (rare) follow after the block.
template <class Op, int KP, int NT, bool PL, int NL = lists_per_lane<PL, NT>()>
static __device__ __forceinline__ void pipe_step(AccArr<Op, NT> &acc_new, AccArr<Op, NT> &acc_old,
                                                 const uint4 (&bq)[NT][Op::kSteps][Op::kBU], const int (&sb)[NT],
                                                 const uint4 *frag, const float4 *seed, const int32_t *rsc, int lane,
                                                 int h, float (&thr)[NL], typename Op::gate_t (&gt)[NL],
                                                 typename Op::gate_t (&gq)[NT], float (&ld)[NL][KP],
                                                 int (&li)[NL][KP], int row_old, const uint32_t *parity,
                                                 int nb_par = 0)
{
    using acc_t = typename Op::acc_t;
    constexpr int S = Op::kSteps;
    constexpr int AU = Op::kAU;
    typename Op::seed_t sd;
    int sa;
    uint4 av[S][AU];
    tile_reads<Op>(frag, seed, rsc, lane, h, av, sd, sa);
    const acc_t seed_acc = __builtin_bit_cast(acc_t, sd);
    bool any[NT];
    if constexpr (Op::kNbnn)
        nbnn_tile_min<Op, NT>(acc_old, gq, nb_par);
    else
        gate_any<Op, NT, PL>(acc_old, gt, gq, any);
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            acc_new[nt] = Op::mma(av[s], bq[nt][s], s == 0 ? seed_acc : acc_new[nt], sa, sb[nt]);
    }
#pragma unroll
    for (int i = 0; i < S * NT * Op::kMfma; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);     // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);     // up to two vector ops
    }
#if LNBNN_MFMA_BEFORE_INSERT
    // FP8 32x32 blocks: the new tile's accumulators are inputs of an empty
    // asm ahead of the insertion branch, so their MFMAs issue (interleaved
    // with the gate) before it; left to itself the compiler sinks them past
    // the branch, and the next gate then waits for them.  Measured: top-4k
    // lists -1.9 %; the 16-bit and 16x16 FP8 kernels are no faster with it.
    if constexpr (!Op::kNbnn && Op::kScaled && Op::kQT == 32) pin_acc<Op, NT>(acc_new);
#endif
    if constexpr (!Op::kNbnn) gate_insert<Op, KP, NT, PL>(acc_old, any, thr, gt, gq, ld, li, row_old, h, parity);
}

// Calls f(std::integral_constant<int, I>) for I = B .. E-1 (a loop whose
// index must be a compile-time constant in every copy).
template <int B, int E, class F>
static __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

#ifndef LNBNN_GATE_LEAD
#define LNBNN_GATE_LEAD 2
#endif
#ifndef LNBNN_READS_AFTER_LEAD
#define LNBNN_READS_AFTER_LEAD 1
#endif
#ifndef LNBNN_LANDED_AT
#define LNBNN_LANDED_AT (-1)        // -1: the middle of the stage
#endif

// Registers of one reference tile: A fragments, the seeds in the
// accumulator layout (four 16-byte LDS reads: no vector instructions, which
// at the 8-bit rates compete with the MFMAs for issue), row scale.
template <class Op>
struct TileRegs {
    uint4 av[Op::kSteps][Op::kAU];
    typename Op::seed_t sd;
    int sa;
};

// Plain LDS loads of one tile.  With the stage copies invisible to the
// compiler (inline assembly), it schedules these freely: the 8-bit formats
// (4 KB tiles, 5 KB for 160-element INT8 rows) load tile t+1 while the
// MFMAs of tile t run.
template <class Op>
static __device__ __forceinline__ void tile_load(const uint4 *frag, const float4 *seed, const int32_t *rsc, int lane,
                                                 int h, TileRegs<Op> &t)
{
#pragma unroll
    for (int s = 0; s < Op::kSteps; ++s)
#pragma unroll
        for (int u = 0; u < Op::kAU; ++u) t.av[s][u] = frag[frag_off<Op>(s, u, lane)];
#pragma unroll
    for (int g = 0; g < Op::kAccN / 4; ++g) {
        const float4 sv = seed[(Op::kRowStride / 4) * g + h];
        t.sd[4 * g + 0] = sv.x;
        t.sd[4 * g + 1] = sv.y;
        t.sd[4 * g + 2] = sv.z;
        t.sd[4 * g + 3] = sv.w;
    }
    if constexpr (Op::kScaled && Op::kQT == 16)
        t.sa = rsc[lane & 15] | (rsc[16 + (lane & 15)] << 8);
    else
        t.sa = Op::kScaled ? rsc[lane & 31] : 127;
}

// One pipeline step on a tile already in registers: its MFMA chain (into
// acc_new) interleaved with the gate of the previous tile (acc_old); the
// next tile's LDS loads, issued just before by the caller, lead the block.
template <class Op, int KP, int NT, bool PL, int NL = lists_per_lane<PL, NT>()>
static __device__ __forceinline__ void pipe_step_regs(AccArr<Op, NT> &acc_new, AccArr<Op, NT> &acc_old,
                                                      const uint4 (&bq)[NT][Op::kSteps][Op::kBU],
                                                      const int (&sb)[NT], const TileRegs<Op> &cur, int h,
                                                      float (&thr)[NL], typename Op::gate_t (&gt)[NL],
                                                      typename Op::gate_t (&gq)[NT], float (&ld)[NL][KP],
                                                      int (&li)[NL][KP], int row_old, const uint32_t *parity,
                                                      int nb_par = 0)
{
    using acc_t = typename Op::acc_t;
    constexpr int S = Op::kSteps;
    const acc_t seed_acc = __builtin_bit_cast(acc_t, cur.sd);
    bool any[NT];
    if constexpr (Op::kNbnn)
        nbnn_tile_min<Op, NT>(acc_old, gq, nb_par);
    else
        gate_any<Op, NT, PL>(acc_old, gt, gq, any);
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            acc_new[nt] = Op::mma(cur.av[s], bq[nt][s], s == 0 ? seed_acc : acc_new[nt], cur.sa, sb[nt]);
    }
    // The gate reads the previous tile's accumulators, whose last MFMAs were
    // issued just before this block: LEAD MFMAs go first so that those
    // chains have completed when the gate's first vector op issues.
    constexpr int NM = S * NT * Op::kMfma;        // MFMAs of the step
    constexpr int LEAD = LNBNN_GATE_LEAD < NM ? LNBNN_GATE_LEAD : NM;
    constexpr int NREAD = S * Op::kAU + Op::kAccN / 4 + (Op::kScaled ? 32 / Op::kQT : 0);   // next tile's LDS loads
#if LNBNN_READS_AFTER_LEAD
    __builtin_amdgcn_sched_group_barrier(0x008, LEAD, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, NREAD, 0);
#else
    __builtin_amdgcn_sched_group_barrier(0x100, NREAD, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, LEAD, 0);
#endif
#pragma unroll
    for (int i = LEAD; i < NM; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);     // up to three vector ops
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);     // one MFMA
    }
    if constexpr (!Op::kNbnn) gate_insert<Op, KP, NT, PL>(acc_old, any, thr, gt, gq, ld, li, row_old, h, parity);
}

// Two waves per SIMD (256 registers each), except where the lists need one
// wave per SIMD (W = 4) and its full register file: 64-entry lists, and two
// lists per lane longer than 20.
template <int KP, int NL>
constexpr int waves_per_simd() { return (KP > 40 || (NL == 2 && KP > 20)) ? 1 : 2; }

template <class Op, int KP, int NT, int MT, int W, int NB, bool PL = false, int PFM = 0>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * W, 64 * W),
                          amdgpu_waves_per_eu(waves_per_simd<KP, lists_per_lane<PL, NT>()>(),
                                              waves_per_simd<KP, lists_per_lane<PL, NT>()>())))
void k_dist_topk(DistArgs a)
{
    constexpr int S = Op::kSteps;
    constexpr int AU = Op::kAU;
    constexpr int TILE_U4 = S * AU * 64;          // uint4 per 32-row tile
    constexpr int STAGE_U4 = MT * TILE_U4;
    constexpr int QW = Op::kQT * NT;              // queries per wave
    constexpr int NL = lists_per_lane<PL, NT>();  // lists per lane
    static_assert(!PL || NT == Op::kGroups, "shared lists: one query tile per lane group");
    constexpr int QB = W * QW;                    // queries per workgroup
    constexpr int PD = NB - 1;                    // stages in flight ahead of the one computed
    constexpr int LPS = StageLoads<Op, MT, W>::total;   // loads per wave per stage
    // next-tile prefetch: by default where the tiles are 4-5 KB (they leave
    // registers for it); PFM > 0 asks for it, PFM < 0 declines it
    constexpr bool kPrefetch = PFM > 0 || (PFM == 0 && Op::kSteps * Op::kAU <= 5);
    // With 3+ buffers the 8-bit-tile path synchronises per buffer instead of
    // per stage: PF = NB - 2 stages in flight leave one stage of slack, so a
    // wave that inserts delays only itself.
    constexpr bool kCounters = kPrefetch && NB >= 3;
    constexpr int PF = kCounters ? NB - 2 : PD;
    // Tile of stage s at which a wave confirms and announces that its copies
    // of stage s + 1 have landed: later leaves the copies more time, earlier
    // leaves the other waves more slack.  The middle measured best.
    constexpr int kLandedAt = LNBNN_LANDED_AT >= 0 && LNBNN_LANDED_AT < MT - 1 ? LNBNN_LANDED_AT
                              : (MT / 2 < MT - 2 ? MT / 2 : MT - 2);
    constexpr int RSC = Op::kScaled ? MT * kTileRows : 1;
    static_assert(MT % 2 == 0, "tiles are processed in pairs");
    static_assert(!Op::kNbnn || kPrefetch, "per-class minima are built on the 8-bit tile paths");
    static_assert(NB >= 2 && (PD - 1) * LPS < 64, "prefetch depth");
    __shared__ uint4 s_frag[NB][STAGE_U4];
    __shared__ float4 s_seed[NB][MT * 8];
    __shared__ int32_t s_rsc[NB][RSC];
    // [0, NB): waves whose share of the buffer's current stage has landed;
    // [NB, 2NB): waves done reading it (counts accumulate over the item)
    __shared__ uint32_t s_cnt[2 * NB];
    auto cnt_signal = [&](int i) {
        asm volatile("" ::: "memory");
        if ((threadIdx.x & 63) == 0)
            __hip_atomic_fetch_add(&s_cnt[i], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // Bounded wait: after spin_limit sleep rounds the wave stops waiting and
    // the call returns true (see mark_if for how that is reported).
    auto cnt_wait = [&](int i, uint32_t target) -> bool {
        int it = 0;
        for (; it < a.spin_limit; ++it) {
            if (__hip_atomic_load(&s_cnt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= target) break;
            __builtin_amdgcn_s_sleep(1);
        }
        asm volatile("" ::: "memory");
        return it >= a.spin_limit;
    };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane / Op::kQT, col = lane & (Op::kQT - 1);   // lane group, query column
    const int64_t n_q = a.bd->n_q;
    const void *q_src = a.q ? a.q : a.bd->q;
    const int64_t n_qb = (n_q + QB - 1) / QB;
    const int64_t n_items = n_qb * a.n_slices;
    const int n_chunks = (a.tiles_per_slice + a.chunk_tiles - 1) / a.chunk_tiles;

    // Walk: for every chunk of its slice, a workgroup runs all the (query
    // block, slice) items it owns before moving to the next chunk.  With the
    // default chunk (the whole slice) each item is one sweep with its lists in
    // registers; shorter chunks keep the workgroups of an XCD on the same
    // references at the same time, with the lists parked in the partial-list
    // buffer between chunks.
    for (int c = 0; c < n_chunks; ++c) {
        for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
            const int slice = (int)(item / n_qb);
            const int64_t qb = item - (int64_t)slice * n_qb;
            const int64_t ts0 = (int64_t)slice * a.tiles_per_slice;
            const int64_t ts1 = min(ts0 + (int64_t)a.tiles_per_slice, a.n_tiles);
            const int64_t t0 = ts0 + (int64_t)c * a.chunk_tiles;
            if (t0 >= ts1) continue;                  // uniform: this slice has fewer chunks
            const int64_t t1 = min(t0 + (int64_t)a.chunk_tiles, ts1);
            const int n_t = (int)(t1 - t0);           // multiple of 8, so of MT

            uint4 bq[NT][S][Op::kBU];
            int sb[NT];
            int64_t qi[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                qi[nt] = qb * QB + wave * QW + nt * Op::kQT + col;
                Op::load_b(q_src, a.q_scale, qi[nt], qi[nt] < n_q, h, bq[nt], sb[nt]);
            }

            // the query of list l, and its partial list's offset
            auto list_query = [&](int l) -> int64_t {
                return PL ? qb * QB + wave * QW + h * Op::kQT + col : qi[l];
            };
            auto list_base = [&](int l) -> int64_t {
                return PL ? ((int64_t)slice * a.q_cap + list_query(l)) * KP
                          : ((int64_t)(slice * Op::kGroups + h) * a.q_cap + qi[l]) * KP;
            };
            float ld[NL][KP];
            int li[NL][KP];
            float thr[NL];
            typename Op::gate_t gt[NL];
            // shared lists: gate threshold of each query tile's query;
            // original NBNN: each query tile's running minimum key (the
            // lane's share of the rows)
            typename Op::gate_t gq[NT];
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int64_t base = list_base(l);
                const bool load = !Op::kNbnn && c > 0 && list_query(l) < n_q;
#pragma unroll
                for (int p = 0; p < KP; ++p) {
                    ld[l][p] = load ? a.part_d[base + p] : __builtin_inff();
                    li[l][p] = load ? a.part_i[base + p] : -1;
                }
                thr[l] = ld[l][KP - 1];
                gt[l] = Op::gate_thr(thr[l]);
            }
            auto share_gates = [&]() {
                if constexpr (PL) share_gate_thr<Op, NT>(gt[0], gq, col);
            };
            share_gates();
            // A wave whose stage wait gave up marks its first list with a NaN
            // key in the last slot: its threshold turns NaN, so nothing more
            // is inserted, and the kernels that read the lists (merge, FP8
            // candidate merge, the per-class flush below) turn the mark into
            // the call's error.  The mark lives in registers that are live
            // anyway: a flag of its own made the hot loop spill.
            auto mark_if = [&](bool gave_up) {
                const float nan = __builtin_nanf("");
                ld[0][KP - 1] = gave_up ? nan : ld[0][KP - 1];
                thr[0] = gave_up ? nan : thr[0];
            };
            // Original NBNN: the class (and parity) of the running minima, and
            // their flush into the per-class minima: the lanes of a query
            // combine their row shares, one of them takes the atomic minimum.
            // The stage value is 2 x class + parity; the tiles gated in a
            // stage's first step belong to the stage before (p_prev).
            int cur_cls = 0, p_cur = 0, p_prev = 0, enc0 = 0;
            if constexpr (Op::kNbnn) {
                enc0 = a.tile_class[t0];
                cur_cls = enc0 >> 1;
                p_cur = p_prev = enc0 & 1;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) gq[nt] = 0x7fffffff;
            }
            auto nbnn_flush = [&]() {
                if constexpr (Op::kNbnn) {
                    if (__builtin_isnan(ld[0][KP - 1]) && lane == 0) atomicOr(a.status, kStatusWaitGaveUp);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        int key = gq[nt];
#pragma unroll
                        for (int o = Op::kQT; o < 64; o <<= 1) key = min(key, __shfl_xor(key, o));
                        if (h == 0 && qi[nt] < n_q && key < (1 << 29))
                            atomicMin(a.cls_min + (int64_t)cur_cls * a.q_cap + qi[nt], key);
                        gq[nt] = 0x7fffffff;
                    }
                }
            };
            // The queries and lists are in registers before any stage copy
            // is in flight.  (The copies are invisible to the compiler: a
            // wait it placed later for these loads would be a vmcnt(0) that
            // drains the prefetches, e.g. on every insertion.)
            wait_vmcnt<0>();

            // Prologue: the first PF stages in flight, wait for stage 0.
            // Stages past the end of the chunk are not needed; to keep the
            // vmcnt arithmetic uniform they re-load the chunk's first stage
            // (whose values are never used).
            const int n_st = n_t / MT;
            if constexpr (kCounters) {
                if (tid < 2 * NB) s_cnt[tid] = 0u;
                __syncthreads();
            }
#pragma unroll
            for (int p = 0; p < PF; ++p) {
                const int64_t ts = t0 + (int64_t)(p < n_st ? p : 0) * MT;
                stage_copy<Op, MT, W, TILE_U4>(a.frag + ts * TILE_U4, s_frag[p], a.seed + ts * kTileRows,
                                               reinterpret_cast<float *>(s_seed[p]), a.row_scale + ts * kTileRows,
                                               s_rsc[p], wave, lane);
            }
            wait_vmcnt<(PF - 1) * LPS>();
            if constexpr (kCounters) {
                cnt_signal(0);                  // this wave's share of stage 0 has landed
                mark_if(cnt_wait(0, W));
            } else {
                __syncthreads();
            }

            // Software pipeline over pairs of tiles: the MFMA chain of one
            // tile is issued in the same block as the gate of the previous
            // tile, so the matrix cores keep working while the gate's vector
            // ops run.  The "previous tile" of the first step holds no key.
            typename Op::acc_t acc0[NT], acc1[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int r = 0; r < Op::kAccN; ++r) acc1[nt][r] = Op::init();
            int row_prev = 0;
            int buf = 0;
            if constexpr (kCounters) {
                // Stage s lives in buffer s % NB as that buffer's fill s / NB.
                // Before refilling a buffer a wave waits until every wave has
                // finished reading its previous fill (s_cnt[NB + b]); before
                // reading a stage it waits until every wave's share has landed
                // (s_cnt[b]).  Each wave signals "landed" for stage s + 1 in
                // the middle of stage s (its copy was issued at the start of
                // stage s + 1 - PF) and "read" for stage s once its last tile
                // is in registers.
                TileRegs<Op> tr[2];           // tile m lives in tr[m % 2]
                tile_load<Op>(s_frag[0], s_seed[0], s_rsc[0], lane, h, tr[0]);
                // original NBNN: the class and parity of stage st + 1 are
                // loaded during stage st and read after the stage's last LDS
                // wait, so the scalar load never adds a wait of its own
                int st_cls = cur_cls, nx_enc = enc0;
                for (int st = 0; st < n_st; ++st) {
                    int ld_enc = 0;
                    if constexpr (Op::kNbnn) {
                        st_cls = nx_enc >> 1;
                        p_prev = p_cur;
                        p_cur = nx_enc & 1;
                        ld_enc = a.tile_class[t0 + (int64_t)min(st + 1, n_st - 1) * MT];
                    }
                    {
                        const int sn = st + PF;
                        const int nb = sn % NB;
                        mark_if(cnt_wait(NB + nb, (uint32_t)(W * (sn / NB))));
                        const int64_t ts = t0 + (int64_t)(sn < n_st ? sn : 0) * MT;
                        stage_copy<Op, MT, W, TILE_U4>(a.frag + ts * TILE_U4, s_frag[nb], a.seed + ts * kTileRows,
                                                       reinterpret_cast<float *>(s_seed[nb]),
                                                       a.row_scale + ts * kTileRows, s_rsc[nb], wave, lane);
                    }
                    static_for<0, MT>([&](auto M) {
                        constexpr int m = decltype(M)::value;
                        const int row_t = (int)((t0 + (int64_t)st * MT + m) * kTileRows) + (PL ? 0 : 4 * h);
                        if constexpr (m == kLandedAt) {
                            wait_vmcnt<(PF - 1) * LPS>();   // this wave's share of stage st + 1 landed
                            cnt_signal((st + 1) % NB);
                        }
                        if constexpr (m == MT - 1) {
                            __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0): this wave's reads of stage st done
                            if constexpr (Op::kNbnn) nx_enc = ld_enc;
                            cnt_signal(NB + st % NB);
                            const int nb = (st + 1) % NB;
                            mark_if(cnt_wait(nb, (uint32_t)(W * ((st + 1) / NB + 1))));
                            tile_load<Op>(s_frag[nb], s_seed[nb], s_rsc[nb], lane, h, tr[(m + 1) % 2]);
                        } else {
                            tile_load<Op>(s_frag[st % NB] + (m + 1) * TILE_U4, s_seed[st % NB] + (m + 1) * 8,
                                          s_rsc[st % NB] + (Op::kScaled ? (m + 1) * kTileRows : 0), lane, h,
                                          tr[(m + 1) % 2]);
                        }
                        const int nb_par = m == 0 ? p_prev : p_cur;
                        if constexpr (m % 2 == 0)
                            pipe_step_regs<Op, KP, NT, PL>(acc0, acc1, bq, sb, tr[0], h, thr, gt, gq, ld, li, row_prev,
                                                           a.parity, nb_par);
                        else
                            pipe_step_regs<Op, KP, NT, PL>(acc1, acc0, bq, sb, tr[1], h, thr, gt, gq, ld, li, row_prev,
                                                           a.parity, nb_par);
                        // the step of a stage's first tile gated the previous
                        // stage's last tile: a new class starts after it
                        if constexpr (Op::kNbnn && m == 0) {
                            if (st_cls != cur_cls) {
                                nbnn_flush();
                                cur_cls = st_cls;
                            }
                        }
                        row_prev = row_t;
                    });
                }
            } else if constexpr (kPrefetch) {
                // 8-bit tiles: tile t+1's LDS loads overlap tile t's MFMAs.
                // The stage barrier comes before a stage's last tile (whose
                // loads have completed: lgkmcnt 0), so the next stage's first
                // tile can be loaded while that last tile computes.
                TileRegs<Op> tr[2];           // tile m lives in tr[m % 2]
                tile_load<Op>(s_frag[0], s_seed[0], s_rsc[0], lane, h, tr[0]);
                int st_cls = cur_cls, nx_enc = enc0;   // as in the counter path above
                for (int st = 0; st < n_st; ++st) {
                    int ld_enc = 0;
                    if constexpr (Op::kNbnn) {
                        st_cls = nx_enc >> 1;
                        p_prev = p_cur;
                        p_cur = nx_enc & 1;
                        ld_enc = a.tile_class[t0 + (int64_t)min(st + 1, n_st - 1) * MT];
                    }
                    {   // stage st + PD goes into the buffer stage st - 1 used
                        const int sn = st + PD;
                        const int64_t ts = t0 + (int64_t)(sn < n_st ? sn : 0) * MT;
                        const int nb = (buf + PD) % NB;
                        stage_copy<Op, MT, W, TILE_U4>(a.frag + ts * TILE_U4, s_frag[nb], a.seed + ts * kTileRows,
                                                       reinterpret_cast<float *>(s_seed[nb]),
                                                       a.row_scale + ts * kTileRows, s_rsc[nb], wave, lane);
                    }
                    static_for<0, MT>([&](auto M) {
                        constexpr int m = decltype(M)::value;
                        const int row_t = (int)((t0 + (int64_t)st * MT + m) * kTileRows) + (PL ? 0 : 4 * h);
                        if constexpr (m == MT - 1) {
                            wait_vmcnt<(PD - 1) * LPS>();       // stage st + 1 landed (this wave's part)
                            __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0): this wave's reads of stage st done
                            if constexpr (Op::kNbnn) nx_enc = ld_enc;
                            asm volatile("" ::: "memory");
                            __builtin_amdgcn_s_barrier();
                            asm volatile("" ::: "memory");
                            const int nb = (buf + 1) % NB;
                            tile_load<Op>(s_frag[nb], s_seed[nb], s_rsc[nb], lane, h, tr[(m + 1) % 2]);
                        } else {
                            tile_load<Op>(s_frag[buf] + (m + 1) * TILE_U4, s_seed[buf] + (m + 1) * 8,
                                          s_rsc[buf] + (Op::kScaled ? (m + 1) * kTileRows : 0), lane, h,
                                          tr[(m + 1) % 2]);
                        }
                        const int nb_par = m == 0 ? p_prev : p_cur;
                        if constexpr (m % 2 == 0)
                            pipe_step_regs<Op, KP, NT, PL>(acc0, acc1, bq, sb, tr[0], h, thr, gt, gq, ld, li, row_prev,
                                                           a.parity, nb_par);
                        else
                            pipe_step_regs<Op, KP, NT, PL>(acc1, acc0, bq, sb, tr[1], h, thr, gt, gq, ld, li, row_prev,
                                                           a.parity, nb_par);
                        if constexpr (Op::kNbnn && m == 0) {
                            if (st_cls != cur_cls) {
                                nbnn_flush();
                                cur_cls = st_cls;
                            }
                        }
                        row_prev = row_t;
                    });
                    buf = (buf + 1) % NB;
                }
            } else
            for (int st = 0; st < n_st; ++st) {
                {   // stage st + PD goes into the buffer stage st - 1 used
                    const int sn = st + PD;
                    const int64_t ts = t0 + (int64_t)(sn < n_st ? sn : 0) * MT;
                    const int nb = (buf + PD) % NB;
                    stage_copy<Op, MT, W, TILE_U4>(a.frag + ts * TILE_U4, s_frag[nb], a.seed + ts * kTileRows,
                                                   reinterpret_cast<float *>(s_seed[nb]),
                                                   a.row_scale + ts * kTileRows, s_rsc[nb], wave, lane);
                }
#pragma unroll
                for (int m = 0; m < MT; m += 2) {
                    const int row_t = (int)((t0 + (int64_t)st * MT + m) * kTileRows) + (PL ? 0 : 4 * h);
                    pipe_step<Op, KP, NT, PL>(acc0, acc1, bq, sb, s_frag[buf] + m * TILE_U4, s_seed[buf] + m * 8,
                                              s_rsc[buf] + (Op::kScaled ? m * kTileRows : 0), lane, h, thr, gt, gq,
                                              ld, li, row_prev, a.parity);
                    pipe_step<Op, KP, NT, PL>(acc1, acc0, bq, sb, s_frag[buf] + (m + 1) * TILE_U4,
                                              s_seed[buf] + (m + 1) * 8,
                                              s_rsc[buf] + (Op::kScaled ? (m + 1) * kTileRows : 0), lane, h, thr,
                                              gt, gq, ld, li, row_t, a.parity);
                    row_prev = row_t + kTileRows;
                }
                // Stage st + 1 has landed (this wave's part); after the barrier
                // every wave's part has, and stage st has been read by all (the
                // tile reads complete before their MFMAs).  A plain barrier: a
                // workgroup fence here would also wait for the prefetches.
                wait_vmcnt<(PD - 1) * LPS>();
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                buf = (buf + 1) % NB;
            }
            wait_vmcnt<0>();                    // drain the loads past the end of the chunk
            __syncthreads();
            tiles_select<Op, KP, NT, PL>(acc1, thr, gt, gq, ld, li, row_prev, h, a.parity, p_cur);
            if constexpr (Op::kNbnn) {
                nbnn_flush();
                continue;
            }

#pragma unroll
            for (int l = 0; l < NL; ++l) {
                if (list_query(l) < n_q) {
                    const int64_t base = list_base(l);
#pragma unroll
                    for (int p = 0; p < KP; ++p) {
                        a.part_d[base + p] = ld[l][p];
                        a.part_i[base + p] = li[l][p];
                    }
                }
            }
        }
    }
}

template <class Op, int KP, int NT, int MT, int W, int NB, bool PL = false, int PFM = 0>
static void *kernel_ptr()
{
    return reinterpret_cast<void *>(&k_dist_topk<Op, KP, NT, MT, W, NB, PL, PFM>);
}

template <class Op, int KP>
static void *pick_variant(int v)
{
    if constexpr (Op::kFmt == FMT_I8L) {
        // 5 KB tiles: a stage of MT tiles splits into 1 KB copies evenly
        // over the waves only for MT * 5 a multiple of W, and four 8-tile
        // buffers would not fit in LDS
        if constexpr (KP <= 16) {
            switch (v) {
            case 2: return kernel_ptr<Op, KP, 2, 4, 4, 2>();
            case 7: return kernel_ptr<Op, KP, 2, 4, 4, 3>();
            case 10: return kernel_ptr<Op, KP, 2, 8, 8, 3>();
            }
        }
        if (v == 11) return kernel_ptr<Op, KP, 1, 8, 8, 3>();
        // shared lists (one list per query): two query tiles at every list length
        if constexpr (KP <= 33)
            if (v == 19) return kernel_ptr<Op, KP, 2, 8, 8, 3, true>();
        return nullptr;
    } else {
        // shared lists (one list per query, half the list registers): two
        // query tiles per wave up to 40-entry lists; one wave per SIMD (the
        // whole register file) for the 40- and 64-entry FP8 candidate lists
        if constexpr (Op::kSteps * Op::kAU == 4 && KP <= 40)
            if (v == 16) return kernel_ptr<Op, KP, 2, 8, 8, 4, true>();
        // 4 KB tiles without the next-tile prefetch: its registers go to the
        // lists' insertion path (the FP8 candidate lists insert often)
        if constexpr (Op::kSteps * Op::kAU == 4 && !Op::kNbnn) {
            if constexpr (KP <= 40)
                if (v == 21) return kernel_ptr<Op, KP, 2, 8, 8, 4, true, -1>();
            if constexpr (KP <= 20)
                if (v == 22) return kernel_ptr<Op, KP, 2, 8, 8, 4, false, -1>();
        }
        if constexpr (Op::kSteps * Op::kAU == 8 && KP <= 33) {
            if (v == 17) return kernel_ptr<Op, KP, 2, 4, 8, 4, true>();
            // the same with next-tile prefetch (its 8 KB tiles fit the
            // registers shared lists free; the insertion path spills)
            if constexpr (KP <= 16)
                if (v == 20) return kernel_ptr<Op, KP, 2, 4, 8, 4, true, 1>();
            // other stage shapes: 8-tile stages (half the stage barriers) in
            // two buffers, and 4-tile stages three deep
            if (v == 23) return kernel_ptr<Op, KP, 2, 8, 8, 2, true>();
            if (v == 24) return kernel_ptr<Op, KP, 2, 4, 8, 3, true>();
        }
        if constexpr (Op::kFmt == FMT_FP8 && KP > 20)
            if (v == 18) return kernel_ptr<Op, KP, 2, 8, 4, 3, true>();
        if (v == 0) return kernel_ptr<Op, KP, 1, 2, 4, 4>();
        if constexpr (KP <= 40)
            if (v == 6) return kernel_ptr<Op, KP, 1, 4, 8, 4>();
        // 8-tile stages for one query tile per wave (the longer lists): 4 KB tiles
        if constexpr (KP <= 40 && Op::kSteps * Op::kAU == 4)
            if (v == 11) return kernel_ptr<Op, KP, 1, 8, 8, 3>();
        // 16x16 output blocks, in the formats that have that form: four
        // lists per query, so shorter ones
        using Q16 = typename Square16<Op>::type;
        // 16x16 blocks with shared lists: four query tiles, one list per query
        if constexpr (!std::is_void<Q16>::value && !Op::kNbnn && KP <= 33) {
            if constexpr (Op::kSteps * Op::kAU == 4) {
                if (v == 25) return kernel_ptr<Q16, KP, 4, 8, 8, 4, true>();
            } else {
                if (v == 26) return kernel_ptr<Q16, KP, 4, 4, 8, 4, true>();
            }
        }
        // the FP8 top-4k candidate lists on 16x16 blocks (40 entries at
        // k = 10), with and without the next-tile prefetch
        if constexpr (Op::kFmt == FMT_FP8 && KP > 33 && KP <= 40)
            if (v == 25) return kernel_ptr<Q16, KP, 4, 8, 8, 4, true>();
        if constexpr (Op::kFmt == FMT_FP8 && KP <= 40)
            if (v == 27) return kernel_ptr<Q16, KP, 4, 8, 8, 4, true, -1>();
        if constexpr (!std::is_void<Q16>::value && Op::kFmt != FMT_FP8 && KP <= 16) {
            if constexpr (Op::kSteps * Op::kAU == 4) {      // 4 KB tiles
                if (v == 13) return kernel_ptr<Q16, KP, 2, 8, 8, 4>();
                if constexpr (KP <= 6)
                    if (v == 15) return kernel_ptr<Q16, KP, 4, 8, 8, 4>();
            } else {
                if (v == 14) return kernel_ptr<Q16, KP, 2, 4, 8, 4>();
            }
        }
        // two query tiles of 64-entry lists, one wave per SIMD: FP8 candidate
        // lists (at 40 entries this shape spills heavily)
        if constexpr (Op::kFmt == FMT_FP8 && KP > 40)
            if (v == 12) return kernel_ptr<Op, KP, 2, 8, 4, 3>();
        if constexpr (Op::kFmt == FMT_FP8) {
            if constexpr (KP <= 20) {
                switch (v) {
                case 1: return kernel_ptr<Op, KP, 2, 2, 4, 4>();
                case 4: return kernel_ptr<Op, KP, 2, 4, 8, 4>();
                case 5: return kernel_ptr<Op, KP, 2, 2, 8, 8>();
                case 8: return kernel_ptr<Op, KP, 2, 8, 8, 4>();
                case 9: return kernel_ptr<Op, KP, 2, 4, 8, 8>();
                }
            }
        } else if constexpr (KP <= 16) {
            switch (v) {
            case 1: return kernel_ptr<Op, KP, 2, 2, 4, 4>();
            case 2: return kernel_ptr<Op, KP, 2, 4, 4, 2>();
            case 3: return kernel_ptr<Op, KP, 2, 2, 4, 2>();
            case 4: return kernel_ptr<Op, KP, 2, 4, 8, 4>();
            case 5: return kernel_ptr<Op, KP, 2, 2, 8, 8>();
            case 7: return kernel_ptr<Op, KP, 2, 4, 4, 3>();
            }
            if constexpr (Op::kSteps * Op::kAU == 4) {      // 4 KB tiles
                switch (v) {
                case 8: return kernel_ptr<Op, KP, 2, 8, 8, 4>();
                case 9: return kernel_ptr<Op, KP, 2, 4, 8, 8>();
                }
            }
        }
        return nullptr;
    }
}

}  // namespace lnbnn
