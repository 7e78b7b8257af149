// lnbnn_classify_noalloc: the batched classification of lnbnn_classify for
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid allocation).  Every buffer the
// launch sequence needs beyond the caller's inputs and outputs (batch
// descriptor, image offsets, partial neighbour lists, per-image totals when
// the caller does not want them, the FP8 mode's codes, candidates and
// updates, the status word) is carved out of one file-scope device array.
//
// The array lives once per GPU for the life of the process; its device
// address is looked up once per device (hipGetSymbolAddress) and only that
// address is handed to kernels and copies.  Every call on a GPU shares that
// GPU's array: calls that overlap on one GPU (two host threads, or two
// streams without ordering between them) race on it.  Each call clears what
// must start at zero (the totals, the status word) with kernels of its own
// sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "runtime.h"

namespace lnbnn {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, uint8_t *> g_scratch_addr;   // device -> its copy of `scratch`

// Device address of this GPU's `scratch` (the current device must be
// `device`); looked up on the first call on each device.
static int scratch_base(int device, uint8_t **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return LNBNN_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)");
    g_scratch_addr[device] = static_cast<uint8_t *>(p);
    *out = static_cast<uint8_t *>(p);
    return LNBNN_OK;
}

// Bump allocation of 256-byte aligned pieces of the scratch array (sizes
// only while `base` is null: the first pass measures, the second carves).
struct Carve {
    uint8_t *base;
    size_t used = 0;
    template <class T>
    T *take(int64_t n)
    {
        const size_t off = used;
        used += ((size_t)std::max<int64_t>(n, 1) * sizeof(T) + 255) / 256 * 256;
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

}  // namespace lnbnn

using namespace lnbnn;

extern "C" int lnbnn_classify_noalloc(lnbnn_index *ix, const void *queries_dev, int dtype,
                                      const int64_t *img_offsets, int32_t n_images, int32_t k, int mode,
                                      int32_t *out_class_dev, void *out_totals_dev, int32_t *out_nbr_idx_dev,
                                      float *out_nbr_dist_dev, int32_t *out_status_dev, void *stream)
{
    int rc = validate_classify(ix, queries_dev, dtype, img_offsets, n_images, k, mode, LNBNN_DEVICE_PTRS,
                               out_class_dev != nullptr, out_nbr_idx_dev, out_nbr_dist_dev);
    if (rc) return rc;
    LN_HIP(hipSetDevice(ix->device));
    uint8_t *base = nullptr;
    if ((rc = scratch_base(ix->device, &base))) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : ix->own_stream;
    if (n_images == 0) return LNBNN_OK;
    const bool fp8 = is_fp8_mode(mode);
    const int64_t n_q = img_offsets[n_images];
    const int64_t nc = ix->n_classes;
    const int64_t q_cap = std::max<int64_t>(1, n_q);
    Plan plan;
    if ((rc = make_plan(ix, mode, dist_list_len(mode, k), q_cap, -1, &plan))) return rc;
    const int64_t part = work_elems(ix, plan, q_cap);
    const int n_cand = fp8_candidates(k);

    // measure, then carve
    Workspace ws;   // a view of the scratch array: owns nothing
    BatchIO io;
    for (int pass = 0; pass < 2; ++pass) {
        Carve c{pass ? base : nullptr};
        BatchDesc *bd = c.take<BatchDesc>(1);
        int64_t *offsets = c.take<int64_t>(n_images + 1);
        int32_t *status = out_status_dev ? out_status_dev : c.take<int32_t>(1);
        unsigned long long *totals = nullptr;
        double *totals_f64 = nullptr;
        if (fp8)
            totals_f64 = out_totals_dev ? static_cast<double *>(out_totals_dev) : c.take<double>(n_images * nc);
        else
            totals = out_totals_dev ? static_cast<unsigned long long *>(out_totals_dev)
                                    : c.take<unsigned long long>(n_images * nc);
        float *part_d = c.take<float>(part);
        int32_t *part_i = c.take<int32_t>(part);
        uint4 *q8 = fp8 ? c.take<uint4>(q_cap * (kDim / 16)) : nullptr;
        int32_t *qsc = fp8 ? c.take<int32_t>(q_cap) : nullptr;
        int32_t *cand = fp8 ? c.take<int32_t>(q_cap * n_cand) : nullptr;
        int32_t *upd_cls = fp8 ? c.take<int32_t>(q_cap * k) : nullptr;
        double *upd_delta = fp8 ? c.take<double>(q_cap * k) : nullptr;
        if (pass == 0) {
            if (c.used > kScratchBytes)
                return set_err(LNBNN_ENOMEM,
                               "this batch (%lld descriptors, %d images, k = %d) needs %zu bytes of scratch; "
                               "the library holds %zu per GPU",
                               (long long)n_q, n_images, k, c.used, kScratchBytes);
            continue;
        }
        ws.q_cap = ws.q8_cap = q_cap;
        ws.img_cap = n_images;
        ws.part_cap = part;
        ws.cand_cap = q_cap * n_cand;
        ws.upd_cap = q_cap * k;
        ws.status = status;
        io.ws = &ws;
        io.offsets = offsets;
        io.bd = bd;
        io.q_cap = q_cap;
        io.img_cap = n_images;
        io.k = k;
        io.mode = mode;
        io.totals = totals;
        io.totals_f64 = totals_f64;
        io.part_d = part_d;
        io.part_i = part_i;
        io.q8 = q8;
        io.qsc = qsc;
        io.cand = cand;
        io.upd_cls = upd_cls;
        io.upd_delta = upd_delta;
    }
    const BatchDesc hb{n_q, n_images, queries_dev, out_class_dev, out_nbr_idx_dev, out_nbr_dist_dev};
    int result = LNBNN_OK;
    hipError_t e = hipMemcpyAsync(const_cast<BatchDesc *>(io.bd), &hb, sizeof hb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<int64_t *>(io.offsets), img_offsets, (size_t)(n_images + 1) * 8,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_set_i32(ws.status, 0, s);
    if (e != hipSuccess) result = hip_err(e, "classify_noalloc setup");
    if (!result) result = enqueue_batch(ix, plan, io, s, nullptr);
    // the view must not free the scratch array
    ws.status = nullptr;
    return result;
}
