// FP8 candidate pass support and exact re-rank (float descriptors).
//
//   k_fp8_rowprep   per reference: power-of-two scale, E8M0 exponent, seed
//   k_fp8_pack      references -> FP8 A-fragment tiles
//   k_fp8_qprep     queries -> FP8 codes of -q * 2^e_q and E8M0 2^(1-e_q)
//   k_cand_merge    per query: 4k best candidates over the half/slice lists
//   k_rerank        per query (one wave): exact FP32 squared distances of the
//                   candidates, the k+1 nearest by (distance, index), and
//                   Algorithm 2's per-class updates dist_C - dist_B
//   k_img_reduce    per image: per-class sums of the updates in descriptor
//                   order, then neighbour order (FP64), and the argmin
//
// Every step depends only on the image's own descriptors, so an image's
// result is the same whatever batch it is classified in.
#include "internal.h"

namespace lnbnn {

// Largest e with m * 2^e <= 448 (OCP e4m3 maximum), for m > 0; 0 for m == 0.
// Clamped so that the E8M0 exponents built from it stay inside 1..254.
static __device__ __forceinline__ int fp8_exponent(float m)
{
    if (!(m > 0.0f)) return 0;
    int ex;
    (void)frexpf(m, &ex);                 // m < 2^ex
    int e = 8 - ex;                       // m * 2^e < 256 <= 448
    if (ldexpf(m, e + 1) <= 448.0f) e += 1;
    return max(-120, min(120, e));
}

// pack two floats into two OCP e4m3 codes (round to nearest even)
static __device__ __forceinline__ uint32_t fp8x2(float a, float b)
{
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

__global__ void k_fp8_rowprep(const float *__restrict__ refs, int64_t n_refs, int64_t n_pad,
                              int32_t *__restrict__ rsc, float *__restrict__ seed)
{
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n_pad;
         row += (int64_t)gridDim.x * blockDim.x) {
        if (row >= n_refs) {
            rsc[row] = 127;
            seed[row] = __builtin_inff();
            continue;
        }
        const float4 *p = reinterpret_cast<const float4 *>(refs + row * kDim);
        float m = 0.0f;
        for (int c = 0; c < kDim / 4; ++c) {
            const float4 v = p[c];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        const int e = fp8_exponent(m);
        // ||r~||^2 of the dequantised values r~ = fp8(r * 2^e) * 2^-e
        float s = 0.0f;
        for (int c = 0; c < kDim / 4; ++c) {
            const float4 v = p[c];
            const uint32_t lo = fp8x2(ldexpf(v.x, e), ldexpf(v.y, e));
            const uint32_t hi = fp8x2(ldexpf(v.z, e), ldexpf(v.w, e));
            const int w = (int)(lo | (hi << 16));
            const float r0 = ldexpf(__builtin_amdgcn_cvt_f32_fp8(w, 0), -e);
            const float r1 = ldexpf(__builtin_amdgcn_cvt_f32_fp8(w, 1), -e);
            const float r2 = ldexpf(__builtin_amdgcn_cvt_f32_fp8(w, 2), -e);
            const float r3 = ldexpf(__builtin_amdgcn_cvt_f32_fp8(w, 3), -e);
            s = fmaf(r0, r0, s);
            s = fmaf(r1, r1, s);
            s = fmaf(r2, r2, s);
            s = fmaf(r3, r3, s);
        }
        rsc[row] = 127 - e;
        seed[row] = s;
    }
}

// Fragment u = ((tile * 2 + s) * 2 + half) * 64 + lane: 16 codes of row
// 32*tile + (lane & 31), K elements 64*s + 32*(lane >> 5) + 16*half + 0..15.
__global__ void k_fp8_pack(const float *__restrict__ refs, int64_t n_refs, int64_t n_frag,
                           const int32_t *__restrict__ rsc, uint4 *__restrict__ frag)
{
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n_frag;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(u & 63);
        const int half = (int)((u >> 6) & 1);
        const int s = (int)((u >> 7) & 1);
        const int64_t tile = u >> 8;
        const int64_t row = tile * kTileRows + (lane & 31);
        uint4 out = make_uint4(0u, 0u, 0u, 0u);
        if (row < n_refs) {
            const int e = 127 - rsc[row];
            const float4 *p = reinterpret_cast<const float4 *>(refs + row * kDim + 64 * s + 32 * (lane >> 5) + 16 * half);
            uint32_t w[4];
            for (int c = 0; c < 4; ++c) {
                const float4 v = p[c];
                w[c] = fp8x2(ldexpf(v.x, e), ldexpf(v.y, e)) | (fp8x2(ldexpf(v.z, e), ldexpf(v.w, e)) << 16);
            }
            out = make_uint4(w[0], w[1], w[2], w[3]);
        }
        frag[u] = out;
    }
}

// Queries: codes of -q * 2^e_q in natural K order and the E8M0 exponent of
// 2^(1 - e_q), so the candidate pass accumulates -2 q~.r~.
__global__ void k_fp8_qprep(const BatchDesc *bd, uint4 *__restrict__ q8, int32_t *__restrict__ qsc)
{
    const int64_t n_q = bd->n_q;
    const float *q = static_cast<const float *>(bd->q);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_q; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 *p = reinterpret_cast<const float4 *>(q + i * kDim);
        float m = 0.0f;
        for (int c = 0; c < kDim / 4; ++c) {
            const float4 v = p[c];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        const int e = fp8_exponent(m);
        for (int c = 0; c < kDim / 16; ++c) {
            uint32_t w[4];
            for (int j = 0; j < 4; ++j) {
                const float4 v = p[4 * c + j];
                w[j] = fp8x2(-ldexpf(v.x, e), -ldexpf(v.y, e)) | (fp8x2(-ldexpf(v.z, e), -ldexpf(v.w, e)) << 16);
            }
            q8[i * (kDim / 16) + c] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        qsc[i] = 128 - e;
    }
}

static __device__ __forceinline__ bool pair_less(float d0, int i0, float d1, int i1)
{
    return d0 < d1 || (d0 == d1 && (uint32_t)i0 < (uint32_t)i1);
}

// One thread per query: the n_cand best (key, index) pairs over the
// n_lists sorted candidate lists of kp_stride entries each (together at
// least n_cand; entries past a list's real rows carry +inf keys and lose).
__global__ __launch_bounds__(256) void k_cand_merge(RerankArgs a)
{
    const int64_t n_q = a.bd->n_q;
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
        for (int p = 0; p < a.n_cand; ++p) {
            float bd = __builtin_inff();
            int bi = -1, bl = 0;
            for (int l = 0; l < a.n_lists; ++l) {
                if (heads[l] >= a.kp_stride) continue;
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
            a.cand[q * a.n_cand + p] = bi;
        }
    }
}

// One wave per query.  Lane j holds candidates j and j + 64 (n_cand <= 128)
// and computes each one's squared distance in FP32, directly as
// sum_t (q_t - r_t)^2 in dimension order; the candidates are ranked by
// (distance, index); the k+1 smallest are the neighbours.  The holder of
// rank j < k emits Algorithm 2's update for its class if no lower rank has
// that class: dist_C - dist_B, formed in FP64 from the two FP32 distances
// (exactly).
__global__ __launch_bounds__(256) void k_rerank(RerankArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t n_q = a.bd->n_q;
    const int k = a.k;
    const int nc = a.n_cand > 64 ? 2 : 1;       // candidate slots per lane
    const float *qf32 = static_cast<const float *>(a.bd->q);
    int32_t *nbr_idx = a.bd->nbr_idx;
    float *nbr_dist = a.bd->nbr_dist;
    for (int64_t q = blockIdx.x * 4 + (threadIdx.x >> 6); q < n_q; q += (int64_t)gridDim.x * 4) {
        float d[2];
        int idx[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int j = lane + 64 * c;
            d[c] = __builtin_inff();
            idx[c] = 0x7fffffff;
            if (j >= a.n_cand) continue;
            const int r = a.cand[q * a.n_cand + j];
            if (r < 0 || r >= a.n_refs) continue;
            const float4 *qr = reinterpret_cast<const float4 *>(qf32 + q * kDim);
            const float4 *rr = reinterpret_cast<const float4 *>(a.ref_f32 + (int64_t)r * kDim);
            float s = 0.0f;
            for (int t = 0; t < kDim / 4; ++t) {
                const float4 x = qr[t], y = rr[t];
                float e = x.x - y.x;
                s = fmaf(e, e, s);
                e = x.y - y.y;
                s = fmaf(e, e, s);
                e = x.z - y.z;
                s = fmaf(e, e, s);
                e = x.w - y.w;
                s = fmaf(e, e, s);
            }
            d[c] = s;
            idx[c] = r;
        }
        int rank[2] = {0, 0};
        for (int c2 = 0; c2 < nc; ++c2) {
            for (int i = 0; i < 64; ++i) {
                const float di = __shfl(d[c2], i);
                const int ii = __shfl(idx[c2], i);
#pragma unroll
                for (int c = 0; c < 2; ++c) rank[c] += pair_less(di, ii, d[c], idx[c]) ? 1 : 0;
            }
        }
        const unsigned long long m0 = __builtin_amdgcn_ballot_w64(rank[0] == k);
        const unsigned long long m1 = __builtin_amdgcn_ballot_w64(nc > 1 && rank[1] == k);
        // the holder of rank k (always one with valid lists; lane 0 otherwise)
        const int src = m0 ? (int)__builtin_ctzll(m0) : m1 ? (int)__builtin_ctzll(m1) : 0;
        const float db = m0 ? __shfl(d[0], src) : __shfl(d[1], src);
        int cls[2];
        bool first[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // a slot without a real candidate (only possible when the lists
            // are invalid, e.g. after a stage wait gave up) never reads a label
            const bool real = idx[c] >= 0 && idx[c] < a.n_refs;
            first[c] = c < nc && rank[c] < k && real;
            cls[c] = first[c] ? a.labels[idx[c]] : -1;
        }
        for (int c2 = 0; c2 < nc; ++c2) {
            for (int i = 0; i < 64; ++i) {
                const int ri = __shfl(rank[c2], i);
                const int ci = __shfl(cls[c2], i);
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (ri < rank[c] && ci == cls[c]) first[c] = false;
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c >= nc) break;
            if (rank[c] < k) {
                a.upd_cls[q * k + rank[c]] = first[c] ? cls[c] : -1;
                a.upd_delta[q * k + rank[c]] = (double)d[c] - (double)db;
            }
            if (nbr_idx && rank[c] <= k) {
                nbr_idx[q * (k + 1) + rank[c]] = idx[c];
                nbr_dist[q * (k + 1) + rank[c]] = d[c];
            }
        }
    }
}

// One workgroup per image: totals[c] = sum over the image's descriptors (in
// order), then over ranks, of the updates of class c; argmin with the lowest
// class on ties.  Classes with no update stay 0.
__global__ __launch_bounds__(256) void k_img_reduce(RerankArgs a)
{
    constexpr int CHUNK = 1024;
    __shared__ int s_cls[CHUNK];
    __shared__ double s_del[CHUNK];
    __shared__ double s_bv[256];
    __shared__ int s_bc[256];
    const int tid = threadIdx.x;
    const int64_t n_img = a.bd->n_img;
    const int k = a.k;
    for (int64_t img = blockIdx.x; img < n_img; img += gridDim.x) {
        const int64_t r0 = a.offsets[img] * k, r1 = a.offsets[img + 1] * k;
        double best = __builtin_inf();
        int bc = 0x7fffffff;
        for (int c0 = 0; c0 < a.n_classes; c0 += 256) {
            const int c = c0 + tid;
            double sum = 0.0;
            for (int64_t base = r0; base < r1; base += CHUNK) {
                const int n = (int)min((int64_t)CHUNK, r1 - base);
                __syncthreads();
                for (int i = tid; i < n; i += 256) {
                    s_cls[i] = a.upd_cls[base + i];
                    s_del[i] = a.upd_delta[base + i];
                }
                __syncthreads();
                for (int i = 0; i < n; ++i)
                    if (s_cls[i] == c) sum += s_del[i];
            }
            if (c < a.n_classes) {
                a.totals_f64[img * a.n_classes + c] = sum;
                if (sum < best) {
                    best = sum;
                    bc = c;
                }
            }
        }
        s_bv[tid] = best;
        s_bc[tid] = bc;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (tid < off) {
                const double ov = s_bv[tid + off];
                const int oc = s_bc[tid + off];
                if (ov < s_bv[tid] || (ov == s_bv[tid] && oc < s_bc[tid])) {
                    s_bv[tid] = ov;
                    s_bc[tid] = oc;
                }
            }
            __syncthreads();
        }
        if (tid == 0) a.bd->cls[img] = s_bc[0] == 0x7fffffff ? 0 : s_bc[0];
        __syncthreads();
    }
}

hipError_t launch_fp8_index(const float *refs, int64_t n_refs, int64_t n_pad, uint4 *frag, float *seed,
                            int32_t *rsc, hipStream_t s)
{
    k_fp8_rowprep<<<grid_for(n_pad, 256, 65536), 256, 0, s>>>(refs, n_refs, n_pad, rsc, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_frag = (n_pad / kTileRows) * 4 * 64;
    k_fp8_pack<<<grid_for(n_frag, 256, 65536), 256, 0, s>>>(refs, n_refs, n_frag, rsc, frag);
    return hipGetLastError();
}

hipError_t launch_fp8_qprep(const BatchDesc *bd, int64_t q_cap, uint4 *q8, int32_t *qsc, hipStream_t s)
{
    k_fp8_qprep<<<grid_for(q_cap, 256, 16384), 256, 0, s>>>(bd, q8, qsc);
    return hipGetLastError();
}

hipError_t launch_rerank(const RerankArgs &a, int64_t q_cap, int64_t img_cap, hipStream_t s)
{
    k_cand_merge<<<grid_for(q_cap, 256, 16384), 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_rerank<<<grid_for(q_cap, 4, 65536), 256, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_img_reduce<<<grid_for(img_cap, 1, 16384), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace lnbnn
