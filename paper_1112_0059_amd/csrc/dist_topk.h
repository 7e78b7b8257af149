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

namespace lnbnn {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

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
struct OpF16 {
    static constexpr int kFmt = FMT_F16;
    static constexpr int kSteps = 8;
    static constexpr int kAU = 1;          // uint4 per lane per step
    static constexpr bool kScaled = false;
    static __device__ __forceinline__ uint4 cvt8(uint2 raw, float mul)
    {
        f16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (_Float16)(mul * (float)byte_at(raw, e));
        return __builtin_bit_cast(uint4, v);
    }
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kAU], int &sb)
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
    static __device__ __forceinline__ f32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kAU], f32x16 c, int, int)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a[0]),
                                                      __builtin_bit_cast(f16x8, b[0]), c, 0, 0, 0);
    }
};

struct OpBF16 {
    static constexpr int kFmt = FMT_BF16;
    static constexpr int kSteps = 8;
    static constexpr int kAU = 1;
    static constexpr bool kScaled = false;
    static __device__ __forceinline__ uint4 cvt8(uint2 raw, float mul)
    {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)(mul * (float)byte_at(raw, e));
        return __builtin_bit_cast(uint4, v);
    }
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kAU], int &sb)
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
    static __device__ __forceinline__ f32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kAU], f32x16 c, int, int)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                       __builtin_bit_cast(bf16x8, b[0]), c, 0, 0, 0);
    }
};

struct OpFP8 {
    static constexpr int kFmt = FMT_FP8;
    static constexpr int kSteps = 2;
    static constexpr int kAU = 2;
    static constexpr bool kScaled = true;
    // queries: FP8 codes [n_q][128] in natural K order, E8M0 scale per query
    static __device__ __forceinline__ void load_b(const void *q, const int32_t *qsc, int64_t qi, bool ok, int h,
                                                  uint4 (&b)[kSteps][kAU], int &sb)
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(q) + (ok ? qi : 0) * kDim);
#pragma unroll
        for (int s = 0; s < kSteps; ++s)
#pragma unroll
            for (int u = 0; u < kAU; ++u) b[s][u] = ok ? qrow[4 * s + 2 * h + u] : make_uint4(0u, 0u, 0u, 0u);
        sb = ok ? qsc[qi] : 127;
    }
    static __device__ __forceinline__ f32x16 mma(const uint4 (&a)[kAU], const uint4 (&b)[kAU], f32x16 c, int sa,
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

// ---------------------------------------------------------------------------
// K1: distances + top-(k+1).
//
// Work item = (query block of W * 32 * NT queries, reference slice).
// Each wave keeps 32*NT queries' operand fragments in registers; the
// workgroup streams 32-row reference tiles through NB LDS stages of MT
// tiles.  With references as the MFMA M dimension and queries as N, lane l's
// 16 accumulator registers are 16 references of one query (column l & 31):
// register r is row 8*(r/4) + 4*(l/32) + r%4.
//
// Selection.  Each lane keeps a sorted register list of the KP best
// (d', index) pairs of its query among the rows it has seen (lanes l and
// l+32 each see half of every tile and keep separate lists).  A tile is
// gated by the minimum of the lane's 16 values: only when some lane of the
// wave beats its current KP-th value does the wave walk the 16 registers and
// insert.  Rows reach a lane in increasing index order, so "strictly less
// than" on d' alone realises the (distance, index) order.
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

static __device__ __forceinline__ float min16(const f32x16 &acc)
{
    const float m0 = __builtin_fminf(__builtin_fminf(acc[0], acc[1]), acc[2]);
    const float m1 = __builtin_fminf(__builtin_fminf(acc[3], acc[4]), acc[5]);
    const float m2 = __builtin_fminf(__builtin_fminf(acc[6], acc[7]), acc[8]);
    const float m3 = __builtin_fminf(__builtin_fminf(acc[9], acc[10]), acc[11]);
    const float m4 = __builtin_fminf(__builtin_fminf(acc[12], acc[13]), acc[14]);
    float mn = __builtin_fminf(__builtin_fminf(m0, m1), __builtin_fminf(m2, m3));
    return __builtin_fminf(__builtin_fminf(mn, m4), acc[15]);
}

// Insert every value of one tile that beats the list's current KP-th value.
template <int KP>
static __device__ __forceinline__ void tile_insert(const f32x16 &acc, float &thr, float (&ld)[KP], int (&li)[KP],
                                                   int row0)
{
    // the row base is made opaque here so the 16 index computations stay on
    // this (rarely taken) path instead of being hoisted into the gate
    int base = row0;
    asm volatile("" : "+v"(base));
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float v = acc[r];
        const bool take = v < thr;
        if (__builtin_amdgcn_ballot_w64(take) != 0) {
            if (take) list_insert<KP>(v, base + 8 * (r >> 2) + (r & 3), ld, li, thr);
        }
    }
}

// Gate + insert for the NT query tiles of one reference tile.  All gates
// are computed before any branch so they can overlap the next MFMA chain.
template <int KP, int NT>
static __device__ __forceinline__ void tiles_select(const f32x16 (&acc)[NT], float (&thr)[NT], float (&ld)[NT][KP],
                                                    int (&li)[NT][KP], int row0)
{
    bool any[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) any[nt] = __builtin_amdgcn_ballot_w64(min16(acc[nt]) < thr[nt]) != 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
        if (any[nt]) tile_insert<KP>(acc[nt], thr[nt], ld[nt], li[nt], row0);
}

typedef __attribute__((address_space(1))) const void *gmem_ptr;
typedef __attribute__((address_space(3))) void *lds_ptr;

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

template <class Op, int MT, int W, int TILE_U4>
static __device__ __forceinline__ void stage_copy(const uint4 *src, uint4 *dst, const float *seed_src, float *seed_dst,
                                                  const int32_t *rsc_src, int32_t *rsc_dst, int wave, int lane)
{
    using SL = StageLoads<Op, MT, W>;
#pragma unroll
    for (int c = 0; c < SL::frag; ++c) {
        const int chunk = c * W + wave;
        __builtin_amdgcn_global_load_lds((gmem_ptr)(src + chunk * 64 + lane), (lds_ptr)(dst + chunk * 64), 16, 0, 0);
    }
    const int s0 = wave * SL::seeds_per_wave;
    if (lane < SL::seeds_per_wave)
        __builtin_amdgcn_global_load_lds((gmem_ptr)(seed_src + s0 + lane), (lds_ptr)(seed_dst + s0), 4, 0, 0);
    if constexpr (Op::kScaled) {
        if (lane < SL::seeds_per_wave)
            __builtin_amdgcn_global_load_lds((gmem_ptr)(rsc_src + s0 + lane), (lds_ptr)(rsc_dst + s0), 4, 0, 0);
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

// One pipeline step: the MFMA chain of a new tile (into acc_new) and the
// gate of the previous tile (acc_old), scheduled as one block: all LDS reads
// of the new tile first, then MFMAs interleaved with the gate's vector ops.
// Insertions for the previous tile (rare) follow after the block.
template <class Op, int KP, int NT>
static __device__ __forceinline__ void pipe_step(f32x16 (&acc_new)[NT], const f32x16 (&acc_old)[NT],
                                                 const uint4 (&bq)[NT][Op::kSteps][Op::kAU], const int (&sb)[NT],
                                                 const uint4 *frag, const float4 *seed, const int32_t *rsc, int lane,
                                                 int h, float (&thr)[NT], float (&ld)[NT][KP], int (&li)[NT][KP],
                                                 int row_old)
{
    constexpr int S = Op::kSteps;
    constexpr int AU = Op::kAU;
    f32x16 sd;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 sv = seed[2 * g + h];
        sd[4 * g + 0] = sv.x;
        sd[4 * g + 1] = sv.y;
        sd[4 * g + 2] = sv.z;
        sd[4 * g + 3] = sv.w;
    }
    int sa = 127;
    if constexpr (Op::kScaled) sa = rsc[lane & 31];
    uint4 av[S][AU];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int u = 0; u < AU; ++u) av[s][u] = frag[(s * AU + u) * 64 + lane];
    bool any[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) any[nt] = __builtin_amdgcn_ballot_w64(min16(acc_old[nt]) < thr[nt]) != 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc_new[nt] = Op::mma(av[s], bq[nt][s], s == 0 ? sd : acc_new[nt], sa, sb[nt]);
    }
    __builtin_amdgcn_sched_group_barrier(0x100, S * AU + 4 + (Op::kScaled ? 1 : 0), 0);   // LDS reads
#pragma unroll
    for (int i = 0; i < S * NT; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);     // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);     // up to two vector ops
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
        if (any[nt]) tile_insert<KP>(acc_old[nt], thr[nt], ld[nt], li[nt], row_old);
}

template <class Op, int KP, int NT, int MT, int W, int NB>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * W, 64 * W), amdgpu_waves_per_eu(2, 2)))
void k_dist_topk(DistArgs a)
{
    constexpr int S = Op::kSteps;
    constexpr int AU = Op::kAU;
    constexpr int TILE_U4 = S * AU * 64;          // uint4 per 32-row tile
    constexpr int STAGE_U4 = MT * TILE_U4;
    constexpr int QW = 32 * NT;                   // queries per wave
    constexpr int QB = W * QW;                    // queries per workgroup
    constexpr int PD = NB - 1;                    // stages in flight ahead of the one computed
    constexpr int LPS = StageLoads<Op, MT, W>::total;   // loads per wave per stage
    constexpr int RSC = Op::kScaled ? MT * kTileRows : 1;
    static_assert(MT % 2 == 0, "tiles are processed in pairs");
    static_assert(NB >= 2 && (PD - 1) * LPS < 64, "prefetch depth");
    __shared__ uint4 s_frag[NB][STAGE_U4];
    __shared__ float4 s_seed[NB][MT * 8];
    __shared__ int32_t s_rsc[NB][RSC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, col = lane & 31;
    const int64_t n_q = a.bd->n_q;
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

            uint4 bq[NT][S][AU];
            int sb[NT];
            int64_t qi[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                qi[nt] = qb * QB + wave * QW + nt * 32 + col;
                Op::load_b(a.q, a.q_scale, qi[nt], qi[nt] < n_q, h, bq[nt], sb[nt]);
            }

            float ld[NT][KP];
            int li[NT][KP];
            float thr[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int64_t base = ((int64_t)(slice * 2 + h) * a.q_cap + qi[nt]) * KP;
                const bool load = c > 0 && qi[nt] < n_q;
#pragma unroll
                for (int p = 0; p < KP; ++p) {
                    ld[nt][p] = load ? a.part_d[base + p] : __builtin_inff();
                    li[nt][p] = load ? a.part_i[base + p] : -1;
                }
                thr[nt] = ld[nt][KP - 1];
            }

            // Prologue: stages 0..PD-1 in flight, wait for stage 0.  Stages
            // past the end of the chunk are not needed; to keep the vmcnt
            // arithmetic uniform they re-load the chunk's first stage into a
            // buffer that is never read.
            const int n_st = n_t / MT;
#pragma unroll
            for (int p = 0; p < PD; ++p) {
                const int64_t ts = t0 + (int64_t)(p < n_st ? p : 0) * MT;
                stage_copy<Op, MT, W, TILE_U4>(a.frag + ts * TILE_U4, s_frag[p], a.seed + ts * kTileRows,
                                               reinterpret_cast<float *>(s_seed[p]), a.row_scale + ts * kTileRows,
                                               s_rsc[p], wave, lane);
            }
            wait_vmcnt<(PD - 1) * LPS>();
            __syncthreads();

            // Software pipeline over pairs of tiles: the MFMA chain of one
            // tile is issued in the same block as the gate of the previous
            // tile, so the matrix cores keep working while the gate's vector
            // ops run.  The "previous tile" of the first step is all +inf.
            f32x16 acc0[NT], acc1[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc1[nt][r] = __builtin_inff();
            int row_prev = 0;
            int buf = 0;
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
                    const int row_t = (int)((t0 + (int64_t)st * MT + m) * kTileRows) + 4 * h;
                    pipe_step<Op, KP, NT>(acc0, acc1, bq, sb, s_frag[buf] + m * TILE_U4, s_seed[buf] + m * 8,
                                          s_rsc[buf] + (Op::kScaled ? m * kTileRows : 0), lane, h, thr, ld, li,
                                          row_prev);
                    pipe_step<Op, KP, NT>(acc1, acc0, bq, sb, s_frag[buf] + (m + 1) * TILE_U4,
                                          s_seed[buf] + (m + 1) * 8,
                                          s_rsc[buf] + (Op::kScaled ? (m + 1) * kTileRows : 0), lane, h, thr, ld,
                                          li, row_t);
                    row_prev = row_t + kTileRows;
                }
                wait_vmcnt<(PD - 1) * LPS>();   // stage st + 1 has landed (this wave's part)
                __syncthreads();                // ... every wave's part; stage st is consumed
                buf = (buf + 1) % NB;
            }
            wait_vmcnt<0>();                    // drain the loads past the end of the chunk
            __syncthreads();
            tiles_select<KP, NT>(acc1, thr, ld, li, row_prev);

#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (qi[nt] < n_q) {
                    const int64_t base = ((int64_t)(slice * 2 + h) * a.q_cap + qi[nt]) * KP;
#pragma unroll
                    for (int p = 0; p < KP; ++p) {
                        a.part_d[base + p] = ld[nt][p];
                        a.part_i[base + p] = li[nt][p];
                    }
                }
            }
        }
    }
}

template <class Op, int KP, int NT, int MT, int W, int NB>
static void *kernel_ptr()
{
    return reinterpret_cast<void *>(&k_dist_topk<Op, KP, NT, MT, W, NB>);
}

template <class Op, int KP>
static void *pick_variant(int v)
{
    switch (v) {
    case 0: return kernel_ptr<Op, KP, 1, 2, 4, 4>();
    case 6: return kernel_ptr<Op, KP, 1, 4, 8, 4>();
    }
    if constexpr (Op::kFmt == FMT_FP8) {
        if constexpr (KP <= 20) {
            switch (v) {
            case 1: return kernel_ptr<Op, KP, 2, 2, 4, 4>();
            case 4: return kernel_ptr<Op, KP, 2, 4, 8, 4>();
            case 5: return kernel_ptr<Op, KP, 2, 2, 8, 8>();
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
    }
    return nullptr;
}

}  // namespace lnbnn
