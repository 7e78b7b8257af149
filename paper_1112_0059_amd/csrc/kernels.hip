// HIP kernels of the local NBNN hot path for gfx950 (MI355X), apart from
// the distance kernel itself (dist_topk.h, instantiated by dist_inst.hip):
//
// K0  pack        references -> MFMA A-fragment tiles + accumulator seeds
// K2  finish      merge of the per-slice lists, background distance,
//                 per-class update of the image totals (Algorithm 2 body)
// K3  argmin      per-image decision (Algorithm 2, return line)
// plus the variant table and the dispatch to the K1 instances.  (The FP8
// packing, candidate merge, exact re-rank and per-image reduction live in
// rerank.hip.)
#include <algorithm>

#include "dist_topk.h"

namespace lnbnn {

// ---------------------------------------------------------------------------
// K0: packing of u8 references ([n_refs, Op::kRow] bytes).  Fragment
// u = (tile * kSteps + s) * 64 + lane holds the K elements lane `lane`
// supplies at step s for row 32*tile + (lane & 31) (eight FP16/BF16 values,
// or sixteen int8 values).  With `perm`, packed row r holds reference
// perm[r] (padding where perm[r] < 0): the class-sorted copy of the index.
// ---------------------------------------------------------------------------
static __device__ __forceinline__ int64_t source_row(const int32_t *perm, int64_t row, int64_t n_refs)
{
    if (perm) return perm[row];
    return row < n_refs ? row : -1;
}

template <class Op>
__global__ void k_pack_u8(const uint8_t *__restrict__ refs, int64_t n_refs, int64_t n_frag,
                          uint4 *__restrict__ frag, const int32_t *__restrict__ perm)
{
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n_frag;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(u & 63);
        const int s = (int)((u >> 6) % Op::kSteps);
        const int64_t tile = (u >> 6) / Op::kSteps;
        const int64_t src = source_row(perm, tile * kTileRows + (lane & 31), n_refs);
        const bool ok = src >= 0;
        frag[u] = Op::pack_frag(refs + (ok ? src : 0) * Op::kRow, ok, s, lane >> 5);
    }
}

// INT8 seeds of [n_refs, dim] references: floor(||s||^2 / 2) + sum(s) with
// s = r - 128 (stored as the int32 bit pattern), 2^30 on padding rows; and
// per 32-row tile the mask of the rows' ||s||^2 parities (= parity of sum(r)).
__global__ void k_seed_i8(const uint8_t *__restrict__ refs, int64_t n_refs, int64_t n_pad, int dim,
                          int32_t *__restrict__ seed, uint32_t *__restrict__ parity,
                          const int32_t *__restrict__ perm)
{
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n_pad;
         row += (int64_t)gridDim.x * blockDim.x) {
        int32_t sq = 0, sum = 0;
        const int64_t src = source_row(perm, row, n_refs);
        const bool real = src >= 0;
        if (real) {
            const uint4 *p = reinterpret_cast<const uint4 *>(refs + src * dim);
            for (int c = 0; c < dim / 16; ++c) {
                const uint4 v = p[c];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
                for (int i = 0; i < 4; ++i)
                    for (int b = 0; b < 4; ++b) {
                        const int32_t x = (int32_t)((w[i] >> (8 * b)) & 0xffu) - 128;
                        sq += x * x;
                        sum += x;
                    }
            }
        }
        seed[row] = real ? (sq >> 1) + sum : OpI8::kPadSeed;
        // one 32-row tile per wave half: bit (row & 31) of its mask
        const uint64_t bits = __builtin_amdgcn_ballot_w64(real && (sq & 1));
        const int lane = threadIdx.x & 63;
        if ((lane & 31) == 0) parity[row >> 5] = (uint32_t)(bits >> (lane & 32));
    }
}

// Parity of ||r - 128||^2 per reference row: the same as the parity of the
// row's byte sum, since x^2 and x have the same parity and 128 is even.
__global__ void k_row_parity(const uint8_t *__restrict__ refs, int64_t n_refs, int dim, uint8_t *__restrict__ out)
{
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n_refs;
         row += (int64_t)gridDim.x * blockDim.x) {
        const uint4 *p = reinterpret_cast<const uint4 *>(refs + row * dim);
        uint32_t x = 0;
        for (int c = 0; c < dim / 16; ++c) {
            const uint4 v = p[c];
            x ^= v.x ^ v.y ^ v.z ^ v.w;
        }
        // the parity of the byte sum is the xor of the bytes' low bits
        x ^= x >> 16;
        x ^= x >> 8;
        out[row] = (uint8_t)(x & 1u);
    }
}

// Accumulator seed ||r||^2 (an exact integer in FP32), +inf on padding rows
// so they never enter a neighbour list.
__global__ void k_seed_u8(const uint8_t *__restrict__ refs, int64_t n_refs, int64_t n_pad,
                          float *__restrict__ seed)
{
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n_pad;
         row += (int64_t)gridDim.x * blockDim.x) {
        if (row >= n_refs) {
            seed[row] = __builtin_inff();
            continue;
        }
        const uint4 *p = reinterpret_cast<const uint4 *>(refs + row * kDim);
        uint32_t acc = 0;
#pragma unroll
        for (int c = 0; c < kDim / 16; ++c) {
            uint4 v = p[c];
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    uint32_t x = (w[i] >> (8 * b)) & 0xffu;
                    acc += x * x;
                }
        }
        seed[row] = (float)acc;
    }
}

// ---------------------------------------------------------------------------
// K2: finish.  One thread per query: merge the n_lists sorted partial
// lists into the k+1 best (d', index) pairs, then apply Algorithm 2's update:
// dist_B is the (k+1)-th distance, and each class met among the first k
// neighbours, at its first (= nearest) occurrence, adds dist_C - dist_B to
// the image total.  Exact modes add exact integers with 64-bit atomics, so
// totals do not depend on the order of the atomics.
// ---------------------------------------------------------------------------
static __device__ __forceinline__ bool pair_less(float d0, int i0, float d1, int i1)
{
    return d0 < d1 || (d0 == d1 && (uint32_t)i0 < (uint32_t)i1);
}

__global__ __launch_bounds__(256) void k_finish(FinishArgs a)
{
    const int64_t n_q = a.bd->n_q;
    const int64_t n_img = a.bd->n_img;
    const int kp = a.k + 1;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n_q;
         q += (int64_t)gridDim.x * blockDim.x) {
        int heads[kMaxLists];
        bool marked = false;            // a list's last key is NaN: its stage wait gave up
        for (int l = 0; l < a.n_lists; ++l) {
            heads[l] = 0;
            const float last = a.part_d[((int64_t)l * a.q_cap + q) * a.kp_stride + a.kp_stride - 1];
            marked = marked || __builtin_isnan(last);
        }
        if (marked) atomicOr(a.status, kStatusWaitGaveUp);
        float dd[kMaxKP];
        int ii[kMaxKP];
        for (int p = 0; p < kp; ++p) {
            float bd = __builtin_inff();
            int bi = -1, bl = 0;
            for (int l = 0; l < a.n_lists; ++l) {
                if (heads[l] >= kp) continue;
                const int64_t o = ((int64_t)l * a.q_cap + q) * a.kp_stride + heads[l];
                const float d = a.part_d[o];
                const int i = a.part_i[o];
                if (pair_less(d, i, bd, bi)) {
                    bd = d;
                    bi = i;
                    bl = l;
                }
            }
            heads[bl] += 1;
            dd[p] = bd;
            ii[p] = bi;
        }
        // ||q - shift||^2 turns the key back into the squared distance
        const uint4 *qr = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(a.bd->q) + q * a.dim);
        uint32_t qq = 0;
        for (int c = 0; c < a.dim / 16; ++c) {
            const uint4 v = qr[c];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            for (int i = 0; i < 4; ++i)
                for (int b = 0; b < 4; ++b) {
                    const int32_t x = (int32_t)((w[i] >> (8 * b)) & 0xffu) - a.q_shift;
                    qq += (uint32_t)(x * x);
                }
        }
        // image of query q: last m with offsets[m] <= q
        int64_t lo = 0, hi = n_img - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.offsets[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int64_t img = lo;
        const int db = (int)dd[a.k];
        int lab[kMaxKP];
        for (int j = 0; j < a.k; ++j) {
            // an index outside the reference set cannot occur; the guard keeps
            // a defect visible as a wrong answer instead of a wild read
            const int c = (ii[j] >= 0 && ii[j] < a.n_refs) ? a.labels[ii[j]] : 0;
            lab[j] = c;
            bool first = true;
            for (int jj = 0; jj < j; ++jj) first = first && (lab[jj] != c);
            if (first) {
                const long long delta = (long long)((int)dd[j] - db);
                atomicAdd(a.totals + img * a.n_classes + c, (unsigned long long)delta);
            }
        }
        int32_t *nbr_idx = a.bd->nbr_idx;
        float *nbr_dist = a.bd->nbr_dist;
        if (nbr_idx) {
            for (int p = 0; p < kp; ++p) {
                nbr_idx[q * kp + p] = ii[p];
                nbr_dist[q * kp + p] = dd[p] + (float)qq;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K3: argmin over classes, lowest class on ties.  One wave per image.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_argmin(const unsigned long long *__restrict__ totals,
                                                const BatchDesc *bd, int32_t n_classes)
{
    int32_t *out_class = bd->cls;
    const int lane = threadIdx.x & 63;
    const int64_t n_img = bd->n_img;
    for (int64_t img = blockIdx.x * 4 + (threadIdx.x >> 6); img < n_img; img += (int64_t)gridDim.x * 4) {
        const long long *t = reinterpret_cast<const long long *>(totals) + img * n_classes;
        long long best = 0x7fffffffffffffffLL;
        int bc = 0x7fffffff;
        for (int c = lane; c < n_classes; c += 64) {
            const long long v = t[c];
            if (v < best) {
                best = v;
                bc = c;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const long long ov = __shfl_xor(best, off);
            const int oc = __shfl_xor(bc, off);
            if (ov < best || (ov == best && oc < bc)) {
                best = ov;
                bc = oc;
            }
        }
        if (lane == 0) out_class[img] = bc;
    }
}

__global__ void k_set_i32(int32_t *p, int32_t v)
{
    if (threadIdx.x == 0) *p = v;
}

// [rows][stride] array: entries [r][0, bd->n_q) set to v.
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t stride, int64_t rows, const BatchDesc *bd)
{
    const int64_t n = bd->n_q;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            p[r * stride + i] = v;
}

// ---------------------------------------------------------------------------
// Original NBNN totals (Algorithm 1): totals[img][C] = sum over the image's
// descriptors d of ||d - NN_C(d)||^2.  cls_min holds the smallest INT8 key
// of every (class, query); the squared distance is that key plus
// ||q - 128||^2.  One workgroup per image: each wave takes every 4th class
// and sums its keys over the image's queries (lanes over queries, 64-bit
// sums, exact); the norms are summed once per image.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nbnn_totals(NbnnArgs a)
{
    __shared__ long long s_nrm[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n_img = a.bd->n_img;
    const uint8_t *qb = static_cast<const uint8_t *>(a.bd->q);
    for (int64_t img = blockIdx.x; img < n_img; img += gridDim.x) {
        const int64_t q0 = a.offsets[img], q1 = a.offsets[img + 1];
        long long nrm = 0;
        for (int64_t q = q0 + tid; q < q1; q += 256) {
            const uint4 *qr = reinterpret_cast<const uint4 *>(qb + q * kDim);
            for (int c = 0; c < kDim / 16; ++c) {
                const uint4 v = qr[c];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
                for (int i = 0; i < 4; ++i)
                    for (int b = 0; b < 4; ++b) {
                        const int32_t x = (int32_t)((w[i] >> (8 * b)) & 0xffu) - 128;
                        nrm += x * x;
                    }
            }
        }
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off);
        if (lane == 0) s_nrm[wave] = nrm;
        __syncthreads();
        nrm = s_nrm[0] + s_nrm[1] + s_nrm[2] + s_nrm[3];
        for (int c = wave; c < a.n_classes; c += 4) {
            const int32_t *m = a.cls_min + (int64_t)c * a.q_cap;
            long long sum = 0;
            for (int64_t q = q0 + lane; q < q1; q += 64) sum += m[q];
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            if (lane == 0) a.totals[img * a.n_classes + c] = (unsigned long long)(sum + nrm);
        }
        __syncthreads();
    }
}

__global__ void k_fill_u64(unsigned long long *p, const BatchDesc *bd, int32_t n_classes, int64_t cap)
{
    int64_t n = bd->n_img * (int64_t)n_classes;
    if (n > cap) n = cap;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Variant table and dispatch
// ---------------------------------------------------------------------------
static const Variant kVariants[] = {
    // nt, mt, waves, buffers, qt, pl
    {1, 2, 4, 4, 32, 0},   // 0
    {2, 2, 4, 4, 32, 0},   // 1
    {2, 4, 4, 2, 32, 0},   // 2
    {2, 2, 4, 2, 32, 0},   // 3
    {2, 4, 8, 4, 32, 0},   // 4
    {2, 2, 8, 8, 32, 0},   // 5
    {1, 4, 8, 4, 32, 0},   // 6
    {2, 4, 4, 3, 32, 0},   // 7
    {2, 8, 8, 4, 32, 0},   // 8  (4 KB tiles only: INT8, FP8)
    {2, 4, 8, 8, 32, 0},   // 9  (4 KB tiles only: INT8, FP8)
    {2, 8, 8, 3, 32, 0},   // 10 (160-element INT8 rows only)
    {1, 8, 8, 3, 32, 0},   // 11 (8-bit formats: INT8 rows of 128 or 160, FP8 lists up to 40)
    {2, 8, 4, 3, 32, 0},   // 12 (FP8 lists of 64: one wave per SIMD)
    {2, 8, 8, 4, 16, 0},   // 13 (16x16 blocks, INT8 rows of 128)
    {2, 4, 8, 4, 16, 0},   // 14 (16x16 blocks, FP16 / BF16)
    {4, 8, 8, 4, 16, 0},   // 15 (16x16 blocks, INT8 rows of 128, lists up to 6)
    {2, 8, 8, 4, 32, 1},   // 16 (pair lists, 4 KB tiles: INT8, FP8 lists up to 40)
    {2, 4, 8, 4, 32, 1},   // 17 (pair lists, FP16 / BF16)
    {2, 8, 4, 3, 32, 1},   // 18 (pair lists, FP8 lists of 40 and 64: one wave per SIMD)
    {2, 8, 8, 3, 32, 1},   // 19 (pair lists, 160-element INT8 rows)
    {2, 4, 8, 4, 32, 1},   // 20 (pair lists + next-tile prefetch, FP16 / BF16)
    {2, 8, 8, 4, 32, 1},   // 21 (pair lists without next-tile prefetch: INT8, FP8)
    {2, 8, 8, 4, 32, 0},   // 22 (w8_nt2_mt8_nb4 without next-tile prefetch: INT8, FP8)
    {2, 8, 8, 2, 32, 1},   // 23 (pair lists, FP16 / BF16, 8-tile stages in two buffers)
    {2, 4, 8, 3, 32, 1},   // 24 (pair lists, FP16 / BF16, 4-tile stages three deep)
    {4, 8, 8, 4, 16, 1},   // 25 (16x16 blocks, shared lists: INT8 rows of 128, FP8 lists up to 40)
    {4, 4, 8, 4, 16, 1},   // 26 (16x16 blocks, shared lists: FP16 / BF16)
    {4, 8, 8, 4, 16, 1},   // 27 (25 without next-tile prefetch: FP8)
};
static const char *kVariantNames[] = {"w4_nt1_mt2_nb4", "w4_nt2_mt2_nb4", "w4_nt2_mt4_nb2", "w4_nt2_mt2_nb2",
                                      "w8_nt2_mt4_nb4", "w8_nt2_mt2_nb8", "w8_nt1_mt4_nb4", "w4_nt2_mt4_nb3",
                                      "w8_nt2_mt8_nb4", "w8_nt2_mt4_nb8", "w8_nt2_mt8_nb3", "w8_nt1_mt8_nb3",
                                      "w4_nt2_mt8_nb3", "q16_w8_nt2_mt8_nb4", "q16_w8_nt2_mt4_nb4",
                                      "q16_w8_nt4_mt8_nb4", "pl_w8_nt2_mt8_nb4", "pl_w8_nt2_mt4_nb4",
                                      "pl_w4_nt2_mt8_nb3", "pl_w8_nt2_mt8_nb3", "plpf_w8_nt2_mt4_nb4",
                                      "plnp_w8_nt2_mt8_nb4", "np_w8_nt2_mt8_nb4", "pl_w8_nt2_mt8_nb2",
                                      "pl_w8_nt2_mt4_nb3", "plq16_w8_nt4_mt8_nb4", "plq16_w8_nt4_mt4_nb4",
                                      "plq16np_w8_nt4_mt8_nb4"};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int num_variants() { return kNumVariants; }
Variant variant(int v) { return kVariants[v]; }
const char *variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariantNames[v] : "?"; }

int kp_bucket(int kp, int fmt)
{
    if (fmt == FMT_I8N) return kp == 1 ? 1 : 0;   // one running minimum per class
    if (fmt == FMT_F16 || fmt == FMT_BF16 || fmt == FMT_I8 || fmt == FMT_I8L) {
        static const int b[] = {2, 6, 11, 16, 21, 33};
        for (int x : b)
            if (kp <= x) return x;
    } else if (fmt == FMT_FP8) {
        static const int b[] = {4, 8, 20, 40, 64};   // per-half candidate lists (>= 2k)
        for (int x : b)
            if (kp <= x) return x;
    }
    return 0;
}

bool variant_supports(int v, int fmt, int kp)
{
    if (v < 0 || v >= kNumVariants) return false;
    const int b = kp_bucket(kp, fmt);
    if (b == 0) return false;
    // 5 KB tiles (160-element INT8 rows) split evenly over the waves only
    // in these stage shapes
    if (fmt == FMT_I8L) return v == 11 || ((v == 2 || v == 7 || v == 10) && b <= 16) || (v == 19 && b <= 33);
    if (v == 10 || v == 19) return false;
    // pair lists: one list per query
    if (v == 16) return (fmt == FMT_I8 || fmt == FMT_I8N || fmt == FMT_FP8) && b <= 40;
    if (v == 17) return (fmt == FMT_F16 || fmt == FMT_BF16) && b <= 33;
    if (v == 20) return (fmt == FMT_F16 || fmt == FMT_BF16) && b <= 16;
    if (v == 21) return (fmt == FMT_FP8 && b <= 40) || fmt == FMT_I8;
    if (v == 22) return (fmt == FMT_FP8 && b <= 20) || (fmt == FMT_I8 && b <= 16);
    if (v == 23 || v == 24) return (fmt == FMT_F16 || fmt == FMT_BF16) && b <= 33;
    if (v == 25) return (fmt == FMT_I8 && b <= 33) || (fmt == FMT_FP8 && b <= 40);
    if (v == 27) return fmt == FMT_FP8 && b <= 40;
    if (v == 26) return (fmt == FMT_F16 || fmt == FMT_BF16) && b <= 33;
    if (v == 18) return fmt == FMT_FP8 && b > 20;
    // 16x16 output blocks: INT8 (128-element rows) and the 16-bit formats
    if (v == 13) return (fmt == FMT_I8 || fmt == FMT_I8N) && b <= 16;
    if (v == 14) return (fmt == FMT_F16 || fmt == FMT_BF16) && b <= 16;
    if (v == 15) return (fmt == FMT_I8 || fmt == FMT_I8N) && b <= 6;
    if (v == 12) return fmt == FMT_FP8 && b > 40;
    // one query tile per wave with 8-tile stages: the 4 KB-tile formats
    if (v == 11) return fmt == FMT_I8 || fmt == FMT_I8N || (fmt == FMT_FP8 && b <= 40);
    // the deep stage variants need the 4 KB tiles of the 8-bit formats
    if ((v == 8 || v == 9) && (fmt == FMT_F16 || fmt == FMT_BF16)) return false;
    // 64-entry lists take a SIMD's whole register file: one wave per SIMD
    if (fmt == FMT_FP8 && b > 40) return v == 0;
    if (fmt == FMT_FP8) return v == 0 || v == 6 || ((v == 1 || v == 4 || v == 5 || v >= 8) && b <= 20);
    return kVariants[v].nt == 1 || b <= 16;
}

// Every compiled K1 instance set: dist_kernel_<tag>_<kp>(v) returns the
// kernel of variant v, or nullptr when v is not built for that list length.
#define LNBNN_DECLARE_INSTANCE(tag, op, fmt, kp) void *dist_kernel_##tag##_##kp(int v);
LNBNN_DIST_INSTANCES(LNBNN_DECLARE_INSTANCE)
#undef LNBNN_DECLARE_INSTANCE

static void *dist_kernel(int v, int fmt, int kp)
{
    if (!variant_supports(v, fmt, kp)) return nullptr;
    const int b = kp_bucket(kp, fmt);
#define LNBNN_PICK_INSTANCE(tag, op, f, k) \
    if (fmt == f && b == k) return dist_kernel_##tag##_##k(v);
    LNBNN_DIST_INSTANCES(LNBNN_PICK_INSTANCE)
#undef LNBNN_PICK_INSTANCE
    return nullptr;
}

hipError_t launch_dist_topk(int v, int fmt, int kp, const DistArgs &a, int grid, hipStream_t s)
{
    void *fn = dist_kernel(v, fmt, kp);
    if (!fn) return hipErrorInvalidValue;
    DistArgs args = a;
    void *params[] = {&args};
    return hipLaunchKernel(fn, dim3(grid), dim3(kVariants[v].waves * 64), params, 0, s);
}

int dist_topk_blocks_per_cu(int v, int fmt, int kp)
{
    void *fn = dist_kernel(v, fmt, kp);
    if (!fn) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kVariants[v].waves * 64, 0) != hipSuccess) return 0;
    return n;
}

// ---------------------------------------------------------------------------
// Host launchers of the small kernels
// ---------------------------------------------------------------------------
int grid_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_pack_u8(const uint8_t *refs, int64_t n_refs, int64_t n_pad, int fmt, uint4 *frag,
                          float *seed, hipStream_t s)
{
    const int64_t n_tiles = n_pad / kTileRows;
    if (fmt == FMT_F16) {
        const int64_t n_frag = n_tiles * OpF16::kSteps * 64;
        k_pack_u8<OpF16><<<grid_for(n_frag, 256, 65536), 256, 0, s>>>(refs, n_refs, n_frag, frag, nullptr);
    } else if (fmt == FMT_BF16) {
        const int64_t n_frag = n_tiles * OpBF16::kSteps * 64;
        k_pack_u8<OpBF16><<<grid_for(n_frag, 256, 65536), 256, 0, s>>>(refs, n_refs, n_frag, frag, nullptr);
    } else {
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (seed) {
        k_seed_u8<<<grid_for(n_pad, 256, 65536), 256, 0, s>>>(refs, n_refs, n_pad, seed);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_pack_i8(const uint8_t *refs, int64_t n_refs, int64_t n_pad, int dim, uint4 *frag,
                          int32_t *seed, uint32_t *parity, hipStream_t s, const int32_t *perm)
{
    if (dim == kDim) {
        const int64_t n_frag = (n_pad / kTileRows) * OpI8::kSteps * 64;
        k_pack_u8<OpI8><<<grid_for(n_frag, 256, 65536), 256, 0, s>>>(refs, n_refs, n_frag, frag, perm);
    } else if (dim == kDimLoc) {
        const int64_t n_frag = (n_pad / kTileRows) * OpI8L::kSteps * 64;
        k_pack_u8<OpI8L><<<grid_for(n_frag, 256, 65536), 256, 0, s>>>(refs, n_refs, n_frag, frag, perm);
    } else {
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // whole waves over whole tiles: n_pad is a multiple of 256, as is the
    // grid stride
    k_seed_i8<<<grid_for(n_pad, 256, 65536), 256, 0, s>>>(refs, n_refs, n_pad, dim, seed, parity, perm);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t cap, const BatchDesc *bd, int32_t n_classes,
                           hipStream_t s)
{
    k_fill_u64<<<grid_for(cap, 256, 4096), 256, 0, s>>>(p, bd, n_classes, cap);
    return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs &a, int64_t q_cap, hipStream_t s)
{
    k_finish<<<grid_for(q_cap, 256, 16384), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_argmin(const unsigned long long *totals, const BatchDesc *bd, int64_t img_cap,
                         int32_t n_classes, hipStream_t s)
{
    k_argmin<<<grid_for(img_cap, 4, 16384), 256, 0, s>>>(totals, bd, n_classes);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, int64_t stride, int64_t rows, const BatchDesc *bd,
                           hipStream_t s)
{
    dim3 grid(grid_for(n, 256, 1024), (unsigned)std::min<int64_t>(std::max<int64_t>(rows, 1), 1024));
    k_fill_i32<<<grid, 256, 0, s>>>(p, v, stride, rows, bd);
    return hipGetLastError();
}

hipError_t launch_nbnn_totals(const NbnnArgs &a, int64_t img_cap, hipStream_t s)
{
    k_nbnn_totals<<<grid_for(img_cap, 1, 16384), 256, 0, s>>>(a);
    return hipGetLastError();
}

// A one-word store as a kernel (a fill node, not a memset node, when the
// sequence is captured in a graph).
hipError_t launch_row_parity(const uint8_t *refs, int64_t n_refs, int dim, uint8_t *out, hipStream_t s)
{
    k_row_parity<<<grid_for(n_refs, 256, 65536), 256, 0, s>>>(refs, n_refs, dim, out);
    return hipGetLastError();
}

hipError_t launch_set_i32(int32_t *p, int32_t v, hipStream_t s)
{
    k_set_i32<<<1, 64, 0, s>>>(p, v);
    return hipGetLastError();
}

}  // namespace lnbnn
