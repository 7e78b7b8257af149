// C ABI of the local NBNN library: index residency, batch planning, the
// launch sequence (direct or replayed from a hipGraph), timing and the
// project autotuner.  See include/lnbnn.h for the contract of every entry
// point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "runtime.h"

using namespace lnbnn;

namespace lnbnn {

static thread_local std::string g_err;

int set_err(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_err(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return set_err(LNBNN_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return set_err(LNBNN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// LNBNN_FAULT=alloc|launch makes the named site fail with LNBNN_EDEVICE, so
// error paths can be exercised without breaking the device.
bool fault_injected(const char *site)
{
    const char *f = getenv("LNBNN_FAULT");
    return f && strcmp(f, site) == 0;
}

// LNBNN_LOG=1: one line on stderr per notable event.
bool log_enabled()
{
    const char *e = getenv("LNBNN_LOG");
    return e && *e && strcmp(e, "0") != 0;
}

void log_line(const char *fmt, ...)
{
    if (!log_enabled()) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[lnbnn] %s\n", buf);
}

// LNBNN_HBM_BUDGET: bytes, with an optional K / M / G suffix; 0 when unset
// or malformed.
static int64_t env_budget()
{
    const char *e = getenv("LNBNN_HBM_BUDGET");
    if (!e || !*e) return 0;
    char *end = nullptr;
    const double v = strtod(e, &end);
    if (end == e || !(v > 0)) return 0;
    double mul = 1;
    if (*end == 'K' || *end == 'k') mul = 1024.0;
    else if (*end == 'M' || *end == 'm') mul = 1024.0 * 1024;
    else if (*end == 'G' || *end == 'g') mul = 1024.0 * 1024 * 1024;
    else if (*end) return 0;
    return (int64_t)(v * mul);
}

static hipError_t dmalloc(void **p, size_t bytes)
{
    if (fault_injected("alloc")) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

int64_t row_bytes(int dtype, int dim) { return dtype == LNBNN_U8 ? dim : (int64_t)dim * 4; }

int mode_fmt(int mode)
{
    switch (mode) {
    case LNBNN_EXACT_F16: return FMT_F16;
    case LNBNN_EXACT_BF16: return FMT_BF16;
    case LNBNN_FP8_RERANK: return FMT_FP8;
    case LNBNN_EXACT_I8: return FMT_I8;
    case LNBNN_FP8_RERANK_2K: return FMT_FP8;
    case LNBNN_NBNN_I8: return FMT_I8N;
    }
    return -1;
}

bool is_fp8_mode(int mode) { return mode == LNBNN_FP8_RERANK || mode == LNBNN_FP8_RERANK_2K; }

int index_fmt(const lnbnn_index *ix, int mode)
{
    const int f = mode_fmt(mode);
    return f == FMT_I8 && ix->dim == kDimLoc ? FMT_I8L : f;
}

Workspace::~Workspace()
{
    void *ps[] = {q, offsets, bd, part_d, part_i, totals, totals_f64, cls, nbr_idx, nbr_dist,
                  q8, qsc, cand, upd_cls, upd_delta, status};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    if (h_status) (void)hipHostFree(h_status);
}

int64_t Workspace::bytes() const
{
    return qbytes_cap + (2 * img_cap + 2) * 8 + img_cap * (int64_t)sizeof(BatchDesc) + part_cap * 8 +
           nbr_cap * 8 + img_cap * 4 + q8_cap * (kDim + 4) + cand_cap * 4 + upd_cap * 12;
}

// The FP8 modes re-rank 4k candidates per query (at least k + 1), the best
// 4k FP8 keys of the union of the distance kernel's lists; lanes l and l+32
// see disjoint halves of every reference tile and keep separate lists.
// LNBNN_FP8_RERANK keeps 4k keys per half (up to the 64-entry lists, k <=
// 16), so the union holds the FP8 top 4k and the candidates are exactly
// them, whatever the launch plan.  LNBNN_FP8_RERANK_2K keeps 2k per half:
// faster (shorter lists), and the union still holds the FP8 top 2k.
// The original NBNN mode keeps one running minimum per class.
int fp8_candidates(int k) { return 4 * k; }
int dist_list_len(int mode, int k)
{
    if (mode == LNBNN_FP8_RERANK) return std::min(4 * k, 64);
    if (mode == LNBNN_FP8_RERANK_2K) return 2 * k;
    if (mode == LNBNN_NBNN_I8) return 1;
    return k + 1;
}

// (Re)allocate *p for `need` elements.  A buffer being replaced goes to the
// index's retired list instead of hipFree, which would synchronise the
// whole device (and break a graph being captured on another thread); the
// retired buffers are freed with the index.
static int grow(lnbnn_index *ix, void **p, int64_t need, size_t elem)
{
    if (*p) {
        std::lock_guard<std::mutex> lock(ix->retired_mu);
        ix->retired.push_back(*p);
        *p = nullptr;
    }
    LN_HIP(dmalloc(p, (size_t)std::max<int64_t>(need, 1) * elem));
    return LNBNN_OK;
}

int64_t cap_bucket(int64_t n, int64_t lo)
{
    int64_t b = lo;
    while (b < n) b *= 2;
    return b;
}

int32_t wait_spin_limit()
{
    const char *e = getenv("LNBNN_WAIT_SPINS");
    if (!e || !*e) return 1 << 20;
    const long v = strtol(e, nullptr, 10);
    return (int32_t)std::max(0L, std::min(v, (long)(1 << 30)));
}

int status_begin(Workspace &ws, hipStream_t s)
{
    if (ws.status_dirty) {
        LN_HIP(launch_set_i32(ws.status, 0, s));
        ws.status_dirty = false;
    }
    return LNBNN_OK;
}

int status_end(Workspace &ws, hipStream_t s)
{
    LN_HIP(hipMemcpyAsync(ws.h_status, ws.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    return LNBNN_OK;
}

int status_check(Workspace &ws, hipStream_t s)
{
    const int32_t st = *ws.h_status;
    if (!(st & kStatusWaitGaveUp)) return LNBNN_OK;
    // the word accumulates until a failure is reported; clear it now
    LN_HIP(launch_set_i32(ws.status, 0, s));
    LN_HIP(hipStreamSynchronize(s));
    *ws.h_status = 0;
    return set_err(LNBNN_EDEVICE,
                   "the distance kernel gave up a bounded wait for an LDS stage (results of the call are invalid)");
}

void drop_graphs(std::map<std::string, GraphEntry> &graphs)
{
    for (auto &kv : graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
}

static void drop_graphs(lnbnn_index *ix) { drop_graphs(ix->graphs); }

// Wait for the work that may still use a workspace before its buffers are
// replaced: the index's own workspace is last used by the work before the
// ws_free event; a serving slot's grows only when the slot is created, with
// no work on it yet.  (No device-wide synchronisation: another thread may be
// capturing a graph on a serving stream, and that call is refused then.)
static int quiesce_ws(lnbnn_index *ix, const Workspace &ws)
{
    if (&ws == &ix->ws && ix->ws_used) LN_HIP(hipEventSynchronize(ix->ws_free));
    return LNBNN_OK;
}

int ensure_ws(lnbnn_index *ix, Workspace &ws, int64_t q_cap, int64_t img_cap, int64_t part, int64_t nbr,
              int64_t qbytes, bool need_f64)
{
    const bool ok = q_cap <= ws.q_cap && img_cap <= ws.img_cap && part <= ws.part_cap &&
                    nbr <= ws.nbr_cap && qbytes <= ws.qbytes_cap && (!need_f64 || ws.totals_f64);
    if (ok && ws.bd) return LNBNN_OK;
    // buffers may be in use by earlier asynchronous work
    int rc;
    if ((rc = quiesce_ws(ix, ws))) return rc;
    if (&ws == &ix->ws) drop_graphs(ix);
    const int64_t nc = ix->n_classes;
    img_cap = std::max(img_cap, ws.img_cap);
    if (img_cap > ws.img_cap || !ws.bd) {
        if ((rc = grow(ix, (void **)&ws.offsets, 2 * img_cap + 2, 8))) return rc;
        if ((rc = grow(ix, (void **)&ws.bd, img_cap + 1, sizeof(BatchDesc)))) return rc;
        if ((rc = grow(ix, (void **)&ws.totals, img_cap * nc, 8))) return rc;
        if ((rc = grow(ix, (void **)&ws.cls, img_cap, 4))) return rc;
        if (ws.totals_f64 || need_f64)
            if ((rc = grow(ix, (void **)&ws.totals_f64, img_cap * nc, 8))) return rc;
        ws.img_cap = img_cap;
    }
    if (need_f64 && !ws.totals_f64)
        if ((rc = grow(ix, (void **)&ws.totals_f64, ws.img_cap * nc, 8))) return rc;
    if (part > ws.part_cap) {
        if ((rc = grow(ix, (void **)&ws.part_d, part, 4))) return rc;
        if ((rc = grow(ix, (void **)&ws.part_i, part, 4))) return rc;
        ws.part_cap = part;
    }
    if (nbr > ws.nbr_cap) {
        if ((rc = grow(ix, (void **)&ws.nbr_idx, nbr, 4))) return rc;
        if ((rc = grow(ix, (void **)&ws.nbr_dist, nbr, 4))) return rc;
        ws.nbr_cap = nbr;
    }
    if (qbytes > ws.qbytes_cap) {
        if ((rc = grow(ix, &ws.q, qbytes, 1))) return rc;
        ws.qbytes_cap = qbytes;
    }
    if (!ws.status) {
        if ((rc = grow(ix, (void **)&ws.status, 1, 4))) return rc;
        LN_HIP(hipHostMalloc((void **)&ws.h_status, sizeof(int32_t), hipHostMallocDefault));
        *ws.h_status = 0;
        ws.status_dirty = true;
    }
    ws.q_cap = std::max(ws.q_cap, q_cap);
    return LNBNN_OK;
}

int ensure_fp8_ws(lnbnn_index *ix, Workspace &ws, int64_t q_cap, int n_cand, int k)
{
    const int64_t cand = q_cap * n_cand, upd = q_cap * k;
    if (q_cap <= ws.q8_cap && cand <= ws.cand_cap && upd <= ws.upd_cap && ws.q8) return LNBNN_OK;
    int rc;
    if ((rc = quiesce_ws(ix, ws))) return rc;
    if (&ws == &ix->ws) drop_graphs(ix);
    if (q_cap > ws.q8_cap || !ws.q8) {
        if ((rc = grow(ix, (void **)&ws.q8, q_cap * (kDim / 16), 16))) return rc;
        if ((rc = grow(ix, (void **)&ws.qsc, q_cap, 4))) return rc;
        ws.q8_cap = q_cap;
    }
    if (cand > ws.cand_cap || !ws.cand) {
        if ((rc = grow(ix, (void **)&ws.cand, cand, 4))) return rc;
        ws.cand_cap = cand;
    }
    if (upd > ws.upd_cap || !ws.upd_cls) {
        if ((rc = grow(ix, (void **)&ws.upd_cls, upd, 4))) return rc;
        if ((rc = grow(ix, (void **)&ws.upd_delta, upd, 8))) return rc;
        ws.upd_cap = upd;
    }
    return LNBNN_OK;
}

static int blocks_per_cu(lnbnn_index *ix, int v, int fmt, int kpb)
{
    auto key = std::make_tuple(v, fmt, kpb);
    {
        std::lock_guard<std::mutex> lock(ix->plan_mu);
        auto it = ix->occupancy.find(key);
        if (it != ix->occupancy.end()) return it->second;
    }
    int n = dist_topk_blocks_per_cu(v, fmt, kpb);
    if (n < 1) n = 1;
    std::lock_guard<std::mutex> lock(ix->plan_mu);
    ix->occupancy[key] = n;
    return n;
}

// A variant that can run the mode's format and list length, and keeps the
// mode's candidate rule: the union-of-halves FP8 rule is defined on one list
// per row half, so pair-list variants do not serve it.
static bool variant_serves(int v, int mode, int fmt, int kp)
{
    if (!variant_supports(v, fmt, kp)) return false;
    return !(variant(v).pl && mode == LNBNN_FP8_RERANK_2K);
}

static int default_variant(int mode, int fmt, int kp)
{
    // the shapes the tuner picked on the 15.36M-reference workloads: pair
    // lists (one list per query) with 8 waves x 64 queries, 8-tile stages
    // for the 4-5 KB tiles; the FP8 top-4k candidate lists without the
    // next-tile prefetch; the union-of-halves FP8 rule on per-half lists
    if (fmt == FMT_I8 || fmt == FMT_I8N) return 16;
    if (fmt == FMT_I8L) return 19;
    if (fmt == FMT_F16 || fmt == FMT_BF16) return 17;
    const int b = kp_bucket(kp, fmt);
    if (mode == LNBNN_FP8_RERANK_2K) return b <= 20 ? 8 : b <= 40 ? 11 : 0;
    return b <= 20 ? 16 : b <= 40 ? 21 : 0;
}

int make_plan(lnbnn_index *ix, int mode, int kp, int64_t q_cap, int forced_variant, Plan *out)
{
    const int fmt = index_fmt(ix, mode);
    const int kpb = kp_bucket(kp, fmt);
    if (kpb == 0) return set_err(LNBNN_EINVAL, "k + 1 = %d is not supported by mode %d", kp, mode);
    lnbnn_tuning tu{-1, 0, 0};
    {
        std::lock_guard<std::mutex> lock(ix->plan_mu);
        auto it = ix->pinned.find({mode, kpb});
        if (it != ix->pinned.end() && q_cap >= it->second.min_q) tu = it->second.t;
    }
    int v = forced_variant >= 0 ? forced_variant : tu.variant;
    if (v < 0) v = default_variant(mode, fmt, kp);
    if (!variant_serves(v, mode, fmt, kp))
        return set_err(LNBNN_EINVAL, "variant %d cannot serve mode %d with k + 1 = %d", v, mode, kp);
    const Variant var = variant(v);
    const int64_t qb = (int64_t)var.waves * var.qt * var.nt;
    const int groups = var.pl ? 1 : 64 / var.qt;  // lists per query and slice
    const int64_t n_qb = std::max<int64_t>(1, (q_cap + qb - 1) / qb);
    const int64_t n_tiles = ix->rows[fmt] / kTileRows;
    const int bpc = blocks_per_cu(ix, v, fmt, kpb);
    int64_t resident = (int64_t)ix->cu_count * bpc;
    if (tu.max_workgroups > 0) resident = std::min<int64_t>(resident, tu.max_workgroups);
    // Split the reference set only when the query blocks alone cannot keep
    // every workgroup slot busy twice over; each split costs one more
    // partial list per lane group (the merge takes at most kMaxLists lists
    // per query).  The split is the one whose (query block, slice) items
    // fill the resident workgroups most evenly: estimated time = rounds of
    // items x (tiles per slice + a start-up cost per item), fewest slices on
    // a tie.
    auto slice_tiles = [&](int64_t s) {
        const int64_t t = (n_tiles + s - 1) / s;
        return std::max<int64_t>(8, (t + 7) / 8 * 8);
    };
    int64_t tps = slice_tiles(1);
    if (n_qb < 2 * resident) {
        constexpr int64_t kItemStartTiles = 32;
        double best = 1e300;
        for (int64_t s = 1; s <= kMaxLists / groups; ++s) {
            const int64_t t = slice_tiles(s);
            if ((n_tiles + t - 1) / t != s) continue;          // the same split as a smaller s
            const int64_t rounds = (n_qb * s + resident - 1) / resident;
            const double cost = (double)rounds * (double)(t + kItemStartTiles);
            if (cost < best) {
                best = cost;
                tps = t;
            }
        }
    }
    const int64_t S = (n_tiles + tps - 1) / tps;
    out->variant = v;
    out->fmt = fmt;
    out->kpb = kpb;
    out->n_slices = (int)S;
    out->n_lists = (int)S * groups;
    out->tiles_per_slice = (int)tps;
    out->grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_qb * S, resident));
    // By default an item sweeps its whole slice with its lists in registers;
    // a tuned chunk length makes workgroups that own several items walk the
    // slice chunk by chunk instead (lists saved between chunks), which keeps
    // the workgroups of an XCD on the same references at the same time.
    out->chunk_tiles = tu.chunk_tiles > 0 ? (int)std::min<int64_t>(tu.chunk_tiles, tps) : (int)tps;
    out->q_cap = q_cap;
    return LNBNN_OK;
}

int64_t part_elems(const Plan &p, int64_t q_cap) { return (int64_t)p.n_lists * q_cap * p.kpb; }

int64_t work_elems(const lnbnn_index *ix, const Plan &p, int64_t q_cap)
{
    // the original NBNN mode keeps its per-class minima in part_i
    if (p.fmt == FMT_I8N) return std::max(part_elems(p, q_cap), (int64_t)ix->n_classes * q_cap);
    return part_elems(p, q_cap);
}

int enqueue_batch(lnbnn_index *ix, const Plan &p, const BatchIO &io, hipStream_t s, hipEvent_t *kev)
{
    if (fault_injected("launch")) return set_err(LNBNN_EDEVICE, "injected launch failure");
    const bool fp8 = p.fmt == FMT_FP8;
    // every buffer the launches write must hold what this plan writes
    const Workspace *w = io.ws;
    const bool nbnn = p.fmt == FMT_I8N;
    if (!w || io.q_cap > w->q_cap || io.img_cap > w->img_cap || work_elems(ix, p, io.q_cap) > w->part_cap ||
        !w->status)
        return set_err(LNBNN_EINVAL, "internal: workspace smaller than the plan");
    if (fp8 && (io.q_cap > w->q8_cap || io.q_cap * fp8_candidates(io.k) > w->cand_cap ||
                io.q_cap * io.k > w->upd_cap))
        return set_err(LNBNN_EINVAL, "internal: FP8 workspace smaller than the plan");
    if (fp8)
        LN_HIP(launch_fp8_qprep(io.bd, io.q_cap, io.q8, io.qsc, s));
    else if (nbnn)
        LN_HIP(launch_fill_i32(io.part_i, 0x7fffffff, io.q_cap, io.q_cap, ix->n_classes, io.bd, s));
    else
        LN_HIP(launch_fill_u64(io.totals, io.img_cap * ix->n_classes, io.bd, ix->n_classes, s));
    DistArgs a{};
    a.q = fp8 ? static_cast<const void *>(io.q8) : nullptr;
    a.q_scale = io.qsc;
    a.bd = io.bd;
    a.frag = ix->frag[p.fmt];
    a.seed = ix->seed[p.fmt];
    // never read by the unscaled formats; any valid address keeps the
    // kernel's pointer arithmetic defined
    a.row_scale = ix->row_scale ? ix->row_scale : reinterpret_cast<const int32_t *>(a.seed);
    a.parity = nbnn ? ix->parity_n : ix->parity;
    if (!a.parity) a.parity = reinterpret_cast<const uint32_t *>(a.seed);
    a.n_tiles = ix->rows[p.fmt] / kTileRows;
    a.tiles_per_slice = p.tiles_per_slice;
    a.n_slices = p.n_slices;
    a.chunk_tiles = p.chunk_tiles;
    a.q_cap = io.q_cap;
    a.part_d = io.part_d;
    a.part_i = io.part_i;
    a.status = w->status;
    a.spin_limit = wait_spin_limit();
    a.tile_class = nbnn ? ix->tile_class : nullptr;
    a.cls_min = nbnn ? io.part_i : nullptr;
    if (kev) LN_HIP(hipEventRecord(kev[0], s));
    LN_HIP(launch_dist_topk(p.variant, p.fmt, p.kpb, a, p.grid, s));
    if (kev) LN_HIP(hipEventRecord(kev[1], s));
    if (fp8) {
        RerankArgs r{};
        r.bd = io.bd;
        r.offsets = io.offsets;
        r.ref_f32 = ix->ref_f32;
        r.labels = ix->labels;
        r.n_refs = ix->n_refs;
        r.n_lists = p.n_lists;
        r.kp_stride = p.kpb;
        r.n_cand = fp8_candidates(io.k);
        r.k = io.k;
        r.n_classes = ix->n_classes;
        r.q_cap = io.q_cap;
        r.part_d = io.part_d;
        r.part_i = io.part_i;
        r.cand = io.cand;
        r.upd_cls = io.upd_cls;
        r.upd_delta = io.upd_delta;
        r.totals_f64 = io.totals_f64;
        r.status = w->status;
        LN_HIP(launch_rerank(r, io.q_cap, io.img_cap, s));
    } else if (nbnn) {
        NbnnArgs n{};
        n.bd = io.bd;
        n.offsets = io.offsets;
        n.cls_min = io.part_i;
        n.q_cap = io.q_cap;
        n.n_classes = ix->n_classes;
        n.totals = io.totals;
        LN_HIP(launch_nbnn_totals(n, io.img_cap, s));
        LN_HIP(launch_argmin(io.totals, io.bd, io.img_cap, ix->n_classes, s));
    } else {
        FinishArgs f{};
        f.q_shift = p.fmt == FMT_I8 || p.fmt == FMT_I8L ? 128 : 0;
        f.dim = ix->dim;
        f.bd = io.bd;
        f.offsets = io.offsets;
        f.labels = ix->labels;
        f.n_refs = ix->n_refs;
        f.n_lists = p.n_lists;
        f.kp_stride = p.kpb;
        f.k = io.k;
        f.n_classes = ix->n_classes;
        f.q_cap = io.q_cap;
        f.part_d = io.part_d;
        f.part_i = io.part_i;
        f.totals = io.totals;
        f.status = w->status;
        LN_HIP(launch_finish(f, io.q_cap, s));
        LN_HIP(launch_argmin(io.totals, io.bd, io.img_cap, ix->n_classes, s));
    }
    return LNBNN_OK;
}

}  // namespace lnbnn

// ===========================================================================
// index
// ===========================================================================
static int free_index_buffers(lnbnn_index *ix)
{
    for (int f = 0; f < kNumFmt; ++f) {
        if (ix->frag[f]) (void)hipFree(ix->frag[f]);
        ix->frag[f] = nullptr;
    }
    // seeds of the two exact 16-bit formats share one buffer
    if (ix->seed[FMT_F16]) (void)hipFree(ix->seed[FMT_F16]);
    else if (ix->seed[FMT_BF16]) (void)hipFree(ix->seed[FMT_BF16]);
    if (ix->seed[FMT_FP8]) (void)hipFree(ix->seed[FMT_FP8]);
    if (ix->seed[FMT_I8]) (void)hipFree(ix->seed[FMT_I8]);
    if (ix->seed[FMT_I8L]) (void)hipFree(ix->seed[FMT_I8L]);
    if (ix->seed[FMT_I8N]) (void)hipFree(ix->seed[FMT_I8N]);
    for (int f = 0; f < kNumFmt; ++f) ix->seed[f] = nullptr;
    if (ix->parity) (void)hipFree(ix->parity);
    ix->parity = nullptr;
    if (ix->parity_n) (void)hipFree(ix->parity_n);
    ix->parity_n = nullptr;
    if (ix->tile_class) (void)hipFree(ix->tile_class);
    ix->tile_class = nullptr;
    if (ix->labels) (void)hipFree(ix->labels);
    if (ix->ref_f32) (void)hipFree(ix->ref_f32);
    if (ix->row_scale) (void)hipFree(ix->row_scale);
    ix->labels = nullptr;
    ix->ref_f32 = nullptr;
    ix->row_scale = nullptr;
    std::lock_guard<std::mutex> lock(ix->retired_mu);
    for (void *p : ix->retired) (void)hipFree(p);
    ix->retired.clear();
    return LNBNN_OK;
}

// The class-sorted INT8 copy of the index for the original NBNN rule
// (Algorithm 1 needs every class's nearest reference): references sorted by
// class (stable), every class padded to a multiple of 256 rows so that a
// class never shares a 32-row tile or an 8-tile stage with another, and
// the class of every tile.  Every class must own a reference.
struct NbnnHost {
    std::vector<int32_t> perm, tile_class;
};

static int build_nbnn_layout(lnbnn_index *ix, const uint8_t *d_refs, const int32_t *hlab, hipStream_t s,
                             NbnnHost &h, int64_t *bytes)
{
    if (ix->dim != kDim) return set_err(LNBNN_EINVAL, "the original NBNN mode takes %d-byte descriptors", kDim);
    const int32_t nc = ix->n_classes;
    // Rows sorted by (class, parity of ||r - 128||^2), each (class, parity)
    // group padded to whole stages: every stage then holds one class and one
    // parity, so the kernel knows a tile's exact smallest key from its
    // smallest accumulator value (key = 2 D + parity).
    std::vector<uint8_t> par(ix->n_refs);
    {
        uint8_t *d_par = nullptr;
        LN_HIP(hipMallocAsync((void **)&d_par, std::max<int64_t>(1, ix->n_refs), s));
        hipError_t e = launch_row_parity(d_refs, ix->n_refs, kDim, d_par, s);
        if (e == hipSuccess) e = hipMemcpyAsync(par.data(), d_par, ix->n_refs, hipMemcpyDeviceToHost, s);
        (void)hipFreeAsync(d_par, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(e, "row parity");
    }
    std::vector<int64_t> cnt(2 * (size_t)nc, 0), start(2 * (size_t)nc + 1, 0);
    for (int64_t j = 0; j < ix->n_refs; ++j) cnt[2 * (size_t)hlab[j] + par[j]] += 1;
    for (int32_t c = 0; c < nc; ++c)
        if (cnt[2 * c] + cnt[2 * c + 1] == 0)
            return set_err(LNBNN_EINVAL, "the original NBNN mode needs every class to own a reference (class %d has none)",
                           c);
    for (int32_t g = 0; g < 2 * nc; ++g) start[g + 1] = start[g] + (cnt[g] + kPadRows - 1) / kPadRows * kPadRows;
    const int64_t n_nb = start[2 * nc];
    if (n_nb >= (int64_t)0x7fffffff) return set_err(LNBNN_EINVAL, "class-sorted index too large");
    h.perm.assign(n_nb, -1);
    std::vector<int64_t> next(start.begin(), start.end() - 1);
    for (int64_t j = 0; j < ix->n_refs; ++j) h.perm[next[2 * (size_t)hlab[j] + par[j]]++] = (int32_t)j;
    // per tile: 2 * class + parity
    h.tile_class.resize(n_nb / kTileRows);
    for (int32_t g = 0; g < 2 * nc; ++g)
        for (int64_t t = start[g] / kTileRows; t < start[g + 1] / kTileRows; ++t) h.tile_class[t] = g;
    int rc;
    int32_t *d_perm = nullptr, *iseed = nullptr;
    if ((rc = grow(ix, (void **)&ix->tile_class, n_nb / kTileRows, 4))) return rc;
    if ((rc = grow(ix, (void **)&ix->frag[FMT_I8N], n_nb * kDim, 1))) return rc;
    if ((rc = grow(ix, (void **)&iseed, n_nb, 4))) return rc;
    ix->seed[FMT_I8N] = reinterpret_cast<float *>(iseed);
    if ((rc = grow(ix, (void **)&ix->parity_n, n_nb / kTileRows, 4))) return rc;
    *bytes = n_nb * (kDim + 4) + n_nb / kTileRows * 8;
    LN_HIP(hipMallocAsync((void **)&d_perm, n_nb * 4, s));
    hipError_t e = hipMemcpyAsync(d_perm, h.perm.data(), n_nb * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ix->tile_class, h.tile_class.data(), h.tile_class.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_pack_i8(d_refs, ix->n_refs, n_nb, kDim, ix->frag[FMT_I8N], iseed, ix->parity_n, s, d_perm);
    (void)hipFreeAsync(d_perm, s);
    if (e != hipSuccess) return hip_err(e, "class-sorted pack");
    ix->rows[FMT_I8N] = n_nb;
    return LNBNN_OK;
}

extern "C" int lnbnn_build_index(const void *refs, int dtype, int64_t n_refs, int32_t dim,
                                 const int32_t *labels, int32_t n_classes, uint32_t mode_mask,
                                 int64_t hbm_budget_bytes, uint32_t flags, void *stream,
                                 lnbnn_index **out)
{
    if (!out || !refs || !labels) return set_err(LNBNN_EINVAL, "NULL argument");
    if (dim != LNBNN_DIM && dim != LNBNN_DIM_LOC)
        return set_err(LNBNN_EINVAL, "dim must be %d or %d (got %d)", LNBNN_DIM, LNBNN_DIM_LOC, dim);
    if (dim == LNBNN_DIM_LOC && (dtype != LNBNN_U8 || mode_mask != LNBNN_MODE_BIT(LNBNN_EXACT_I8)))
        return set_err(LNBNN_EINVAL, "dim %d (location-augmented) needs u8 data and the INT8 mode alone",
                       LNBNN_DIM_LOC);
    if (n_refs < 1 || n_refs >= (int64_t)0x7fffffff - kPadRows)
        return set_err(LNBNN_EINVAL, "n_refs out of range: %lld", (long long)n_refs);
    if (n_classes < 1) return set_err(LNBNN_EINVAL, "n_classes must be >= 1");
    if (dtype != LNBNN_U8 && dtype != LNBNN_F32) return set_err(LNBNN_EINVAL, "bad dtype %d", dtype);
    if (hbm_budget_bytes < 0) return set_err(LNBNN_EINVAL, "negative HBM budget");
    const uint32_t exact = LNBNN_MODE_BIT(LNBNN_EXACT_F16) | LNBNN_MODE_BIT(LNBNN_EXACT_BF16) |
                           LNBNN_MODE_BIT(LNBNN_EXACT_I8) | LNBNN_MODE_BIT(LNBNN_NBNN_I8);
    const uint32_t fp8m = LNBNN_MODE_BIT(LNBNN_FP8_RERANK) | LNBNN_MODE_BIT(LNBNN_FP8_RERANK_2K);
    if (mode_mask == 0) return set_err(LNBNN_EINVAL, "empty mode mask");
    if (dtype == LNBNN_U8 && (mode_mask & ~exact))
        return set_err(LNBNN_EINVAL, "mode mask 0x%x: u8 data builds only the exact modes", mode_mask);
    if (dtype == LNBNN_F32 && (mode_mask & ~fp8m))
        return set_err(LNBNN_EINVAL, "mode mask 0x%x: float data builds only the FP8 re-rank modes", mode_mask);
    if (flags & ~(uint32_t)LNBNN_DEVICE_PTRS) return set_err(LNBNN_EINVAL, "unknown flags 0x%x", flags);
    const bool dev_in = flags & LNBNN_DEVICE_PTRS;
    if (!dev_in) {
        for (int64_t j = 0; j < n_refs; ++j)
            if (labels[j] < 0 || labels[j] >= n_classes)
                return set_err(LNBNN_EINVAL, "label[%lld] = %d outside [0, %d)", (long long)j, labels[j],
                               n_classes);
    }

    int dev = 0;
    LN_HIP(hipGetDevice(&dev));
    std::unique_ptr<lnbnn_index> ix(new lnbnn_index());
    ix->device = dev;
    ix->dtype = dtype;
    ix->dim = dim;
    ix->n_refs = n_refs;
    ix->n_pad = (n_refs + kPadRows - 1) / kPadRows * kPadRows;
    ix->n_classes = n_classes;
    ix->modes = mode_mask;
    ix->ws.device = dev;
    LN_HIP(hipDeviceGetAttribute(&ix->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
    // a blocking stream stays ordered after work on the NULL stream
    LN_HIP(hipStreamCreate(&ix->own_stream));
    for (auto &e : ix->tev) LN_HIP(hipEventCreate(&e));
    LN_HIP(hipEventCreateWithFlags(&ix->ws_free, hipEventDisableTiming));
    hipStream_t s = stream ? (hipStream_t)stream : ix->own_stream;
    lnbnn_index *ixp = ix.get();

    auto fail = [&](int rc) {
        (void)hipStreamSynchronize(s);
        free_index_buffers(ix.get());
        return rc;
    };

    // labels: device copy (and validation when they came as device memory)
    int rc;
    if ((rc = grow(ixp, (void **)&ix->labels, n_refs, 4))) return fail(rc);
    std::vector<int32_t> hl;           // host copy of device labels
    if (dev_in) {
        hl.resize(n_refs);
        hipError_t e = hipMemcpy(hl.data(), labels, n_refs * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(hip_err(e, "hipMemcpy(labels)"));
        for (int64_t j = 0; j < n_refs; ++j)
            if (hl[j] < 0 || hl[j] >= n_classes)
                return fail(set_err(LNBNN_EINVAL, "label[%lld] = %d outside [0, %d)", (long long)j, hl[j],
                                    n_classes));
        e = hipMemcpyAsync(ix->labels, labels, n_refs * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(hip_err(e, "hipMemcpyAsync(labels)"));
    } else {
        hipError_t e = hipMemcpyAsync(ix->labels, labels, n_refs * 4, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail(hip_err(e, "hipMemcpyAsync(labels)"));
    }

    // references: stage the rows on the device, then pack per mode
    const int64_t rbytes = n_refs * row_bytes(dtype, dim);
    const void *d_refs = refs;
    void *staged = nullptr;
    if (dtype == LNBNN_F32) {
        // the FP32 rows stay resident for the exact re-rank
        if ((rc = grow(ixp, (void **)&ix->ref_f32, n_refs * kDim, 4))) return fail(rc);
        hipError_t e = hipMemcpyAsync(ix->ref_f32, refs, (size_t)rbytes,
                                      dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail(hip_err(e, "hipMemcpyAsync(refs)"));
        d_refs = ix->ref_f32;
    } else if (!dev_in) {
        // stream-ordered staging: freeing it does not synchronise the device
        hipError_t e = fault_injected("alloc") ? hipErrorOutOfMemory : hipMallocAsync(&staged, (size_t)rbytes, s);
        if (e != hipSuccess) return fail(hip_err(e, "hipMallocAsync(staging)"));
        e = hipMemcpyAsync(staged, refs, (size_t)rbytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            (void)hipFreeAsync(staged, s);
            return fail(hip_err(e, "hipMemcpyAsync(refs)"));
        }
        d_refs = staged;
    }
    float *seed = nullptr;
    int64_t bytes = n_refs * 4 + (dtype == LNBNN_F32 ? rbytes : 0);
    rc = grow(ixp, (void **)&seed, ix->n_pad, 4);
    if (!rc) bytes += ix->n_pad * 4;
    bool seeded = false;
    if (dtype == LNBNN_F32) {
        if (!rc) rc = grow(ixp, (void **)&ix->row_scale, ix->n_pad, 4);
        if (!rc) rc = grow(ixp, (void **)&ix->frag[FMT_FP8], ix->n_pad * kDim, 1);
        if (!rc) {
            bytes += ix->n_pad * (4 + kDim);
            hipError_t e = launch_fp8_index(static_cast<const float *>(d_refs), n_refs, ix->n_pad,
                                            ix->frag[FMT_FP8], seed, ix->row_scale, s);
            if (e != hipSuccess) rc = hip_err(e, "fp8 pack");
            seeded = true;
            ix->seed[FMT_FP8] = seed;
        }
    }
    for (int mode : {LNBNN_EXACT_F16, LNBNN_EXACT_BF16}) {
        if (rc || dtype != LNBNN_U8 || !(mode_mask & LNBNN_MODE_BIT(mode))) continue;
        const int fmt = mode_fmt(mode);
        if ((rc = grow(ixp, (void **)&ix->frag[fmt], ix->n_pad * kDim * 2, 1))) break;
        bytes += ix->n_pad * kDim * 2;
        hipError_t e = launch_pack_u8(static_cast<const uint8_t *>(d_refs), n_refs, ix->n_pad, fmt, ix->frag[fmt],
                                      seeded ? nullptr : seed, s);
        if (e != hipSuccess) {
            rc = hip_err(e, "pack");
            break;
        }
        seeded = true;
        ix->seed[fmt] = seed;
    }
    if (!rc && dtype == LNBNN_U8 && (mode_mask & LNBNN_MODE_BIT(LNBNN_EXACT_I8))) {
        // INT8 mode: its own fragments, seeds and parity masks
        const int f8 = index_fmt(ix.get(), LNBNN_EXACT_I8);
        int32_t *iseed = nullptr;
        rc = grow(ixp, (void **)&ix->frag[f8], ix->n_pad * dim, 1);
        if (!rc) rc = grow(ixp, (void **)&iseed, ix->n_pad, 4);
        if (!rc) ix->seed[f8] = reinterpret_cast<float *>(iseed);
        if (!rc) rc = grow(ixp, (void **)&ix->parity, ix->n_pad / kTileRows, 4);
        if (!rc) {
            bytes += ix->n_pad * (dim + 4) + ix->n_pad / kTileRows * 4;
            hipError_t e = launch_pack_i8(static_cast<const uint8_t *>(d_refs), n_refs, ix->n_pad, dim, ix->frag[f8],
                                          iseed, ix->parity, s);
            if (e != hipSuccess) rc = hip_err(e, "pack i8");
        }
    }
    for (int f = 0; f < kNumFmt; ++f) ix->rows[f] = ix->n_pad;
    NbnnHost nbh;   // host arrays of the class-sorted copy: alive until the sync below
    if (!rc && (mode_mask & LNBNN_MODE_BIT(LNBNN_NBNN_I8))) {
        int64_t nb_bytes = 0;
        rc = build_nbnn_layout(ixp, static_cast<const uint8_t *>(d_refs), dev_in ? hl.data() : labels, s, nbh,
                               &nb_bytes);
        bytes += nb_bytes;
    }
    if (staged) (void)hipFreeAsync(staged, s);
    hipError_t e = hipStreamSynchronize(s);
    if (rc) {
        if (seed && !seeded) (void)hipFree(seed);
        return fail(rc);
    }
    if (e != hipSuccess) return fail(hip_err(e, "build_index sync"));
    if (seed && !seeded) {   // no mode used the shared seed buffer
        (void)hipFree(seed);
        bytes -= ix->n_pad * 4;
    }
    ix->device_bytes = bytes;
    size_t free_b = 0, total_b = 0;
    LN_HIP(hipMemGetInfo(&free_b, &total_b));
    const int64_t env_b = env_budget();
    ix->hbm_budget = hbm_budget_bytes ? hbm_budget_bytes : env_b ? env_b : (int64_t)(free_b / 4);
    log_line("index built: %lld references, dim %d, %d classes, modes 0x%x, %lld device bytes, serving budget %lld bytes",
             (long long)ix->n_refs, ix->dim, ix->n_classes, ix->modes, (long long)ix->device_bytes,
             (long long)ix->hbm_budget);
    *out = ix.release();
    return LNBNN_OK;
}

extern "C" int lnbnn_index_free(lnbnn_index *ix)
{
    if (!ix) return LNBNN_OK;
    if (server_pending(ix)) return set_err(LNBNN_EBUSY, "index has pending tickets");
    server_stop(ix);                       // joins the serving threads after their streams drain
    (void)hipSetDevice(ix->device);
    // the index's own work: classify calls (up to the ws_free event) and
    // its stream
    if (ix->ws_used) (void)hipEventSynchronize(ix->ws_free);
    if (ix->own_stream) (void)hipStreamSynchronize(ix->own_stream);
    drop_graphs(ix);
    free_index_buffers(ix);
    for (auto &e : ix->tev)
        if (e) (void)hipEventDestroy(e);
    if (ix->ws_free) (void)hipEventDestroy(ix->ws_free);
    if (ix->own_stream) (void)hipStreamDestroy(ix->own_stream);
    delete ix;
    return LNBNN_OK;
}

extern "C" int lnbnn_index_info(const lnbnn_index *ix, int64_t *n_refs, int32_t *n_classes,
                                uint32_t *mode_mask, int64_t *device_bytes)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    if (n_refs) *n_refs = ix->n_refs;
    if (n_classes) *n_classes = ix->n_classes;
    if (mode_mask) *mode_mask = ix->modes;
    if (device_bytes) *device_bytes = ix->device_bytes;
    return LNBNN_OK;
}

// ===========================================================================
// classify
// ===========================================================================
int lnbnn::validate_classify(const lnbnn_index *ix, const void *queries, int dtype, const int64_t *off,
                             int32_t n_images, int32_t k, int mode, uint32_t flags, bool has_out_class,
                             const int32_t *nbr_idx, const float *nbr_dist)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    if (!off || !has_out_class) return set_err(LNBNN_EINVAL, "NULL img_offsets or out_class");
    if (n_images < 0) return set_err(LNBNN_EINVAL, "n_images < 0");
    if (flags & ~(uint32_t)(LNBNN_DEVICE_PTRS | LNBNN_PER_IMAGE_LAUNCH | LNBNN_NO_GRAPH | LNBNN_TIMING))
        return set_err(LNBNN_EINVAL, "unknown flags 0x%x", flags);
    if (mode < 0 || mode >= kNumModes || !(ix->modes & LNBNN_MODE_BIT(mode)))
        return set_err(LNBNN_EINVAL, "mode %d is not materialised in this index", mode);
    const int want = is_fp8_mode(mode) ? LNBNN_F32 : LNBNN_U8;
    if (dtype != want) return set_err(LNBNN_EINVAL, "dtype %d does not match mode %d", dtype, mode);
    if (k < 1 || k > LNBNN_MAX_K) return set_err(LNBNN_EINVAL, "k = %d outside [1, %d]", k, LNBNN_MAX_K);
    if ((int64_t)k + 1 > ix->n_refs) return set_err(LNBNN_EINVAL, "k + 1 > n_refs");
    if (mode == LNBNN_NBNN_I8 && (nbr_idx || nbr_dist))
        return set_err(LNBNN_EINVAL, "the original NBNN mode returns no neighbour lists");
    if (is_fp8_mode(mode)) {
        if (k > kMaxFp8K) return set_err(LNBNN_EINVAL, "FP8 re-rank mode needs k <= %d", kMaxFp8K);
        if ((int64_t)fp8_candidates(k) > ix->n_refs) return set_err(LNBNN_EINVAL, "4k > n_refs");
    }
    if ((nbr_idx == nullptr) != (nbr_dist == nullptr))
        return set_err(LNBNN_EINVAL, "out_nbr_idx and out_nbr_dist must both be set or both NULL");
    if (off[0] != 0) return set_err(LNBNN_EINVAL, "img_offsets[0] must be 0");
    for (int32_t m = 0; m < n_images; ++m)
        if (off[m + 1] < off[m]) return set_err(LNBNN_EINVAL, "img_offsets decrease at %d", m);
    if (off[n_images] > 0 && !queries) return set_err(LNBNN_EINVAL, "NULL queries");
    return LNBNN_OK;
}

std::string lnbnn::graph_key(const Plan &p, const BatchIO &io)
{
    // the plan, the capacities, the workspace buffers and the stage-wait
    // bound (all kernel arguments frozen into the graph); the caller's
    // queries and outputs travel in the batch descriptor
    std::ostringstream o;
    o << wait_spin_limit() << '/' << p.variant << '/' << p.fmt << '/' << p.kpb << '/' << p.n_slices << '/' << p.tiles_per_slice << '/' << p.chunk_tiles << '/'
      << p.grid << '/' << io.q_cap << '/' << io.img_cap << '/' << io.k << '/' << io.mode << '/' << io.offsets << '/'
      << io.bd << '/' << io.totals << '/' << io.totals_f64 << '/' << io.part_d << '/' << io.part_i << '/' << io.q8
      << '/' << io.cand;
    return o.str();
}

// Replay (capturing on first use) the launch sequence of a batch.  The
// caller has made sure that no earlier replay of these graphs is still in
// flight when an entry is evicted (the workspace's work is ordered on one
// fence, and eviction waits for it).
int lnbnn::launch_graph(std::map<std::string, GraphEntry> &graphs, uint64_t &clock, lnbnn_index *ix, const Plan &p,
                        const BatchIO &io, hipStream_t s)
{
    const std::string key = graph_key(p, io);
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        if (graphs.size() >= kMaxGraphs) {
            auto lru = graphs.begin();
            for (auto g = graphs.begin(); g != graphs.end(); ++g)
                if (g->second.last_use < lru->second.last_use) lru = g;
            if (lru->second.exec) LN_HIP(hipGraphExecDestroy(lru->second.exec));
            graphs.erase(lru);
        }
        GraphEntry g;
        LN_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_batch(ix, p, io, s, nullptr);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_err(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_err(e, "hipGraphInstantiate");
        log_line("graph captured: mode %d, k %d, %s, %d slices, chunk %d tiles, grid %d, capacity %lld descriptors / "
                 "%lld images (%zu cached)", io.mode, io.k, variant_name(p.variant), p.n_slices, p.chunk_tiles, p.grid,
                 (long long)io.q_cap, (long long)io.img_cap, graphs.size() + 1);
        it = graphs.emplace(key, g).first;
    }
    it->second.last_use = ++clock;
    LN_HIP(hipGraphLaunch(it->second.exec, s));
    return LNBNN_OK;
}

// The plain per-image form: one launch sequence per image, each planned for
// that image alone (no graph).  With `kev`, the distance-kernel time of every
// launch is summed.
static int classify_per_image(lnbnn_index *ix, const void *dq, const int64_t *off, int32_t n_images,
                              int32_t k, int mode, int32_t *cls, int32_t *nbr_idx, float *nbr_dist, hipStream_t s,
                              hipEvent_t *kev)
{
    Workspace &ws = ix->ws;
    const int kp = k + 1;
    const int list_len = dist_list_len(mode, k);
    std::vector<Plan> plans(n_images);
    for (int32_t m = 0; m < n_images; ++m) {
        int rc = make_plan(ix, mode, list_len, std::max<int64_t>(1, off[m + 1] - off[m]), -1, &plans[m]);
        if (rc) return rc;
    }
    const int64_t rb = row_bytes(ix->dtype, ix->dim);
    std::vector<BatchDesc> bds(n_images);
    std::vector<int64_t> offs(2 * (size_t)n_images);
    for (int32_t m = 0; m < n_images; ++m) {
        bds[m].n_q = off[m + 1] - off[m];
        bds[m].n_img = 1;
        bds[m].q = static_cast<const uint8_t *>(dq) + off[m] * rb;
        bds[m].cls = cls + m;
        bds[m].nbr_idx = nbr_idx ? nbr_idx + off[m] * kp : nullptr;
        bds[m].nbr_dist = nbr_dist ? nbr_dist + off[m] * kp : nullptr;
        offs[2 * m] = 0;
        offs[2 * m + 1] = bds[m].n_q;
    }
    LN_HIP(hipMemcpyAsync(ws.bd, bds.data(), n_images * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
    LN_HIP(hipMemcpyAsync(ws.offsets, offs.data(), offs.size() * 8, hipMemcpyHostToDevice, s));
    double kms = 0;
    for (int32_t m = 0; m < n_images; ++m) {
        BatchIO io;
        io.offsets = ws.offsets + 2 * m;
        io.bd = ws.bd + m;
        io.q_cap = plans[m].q_cap;
        io.img_cap = 1;
        io.k = k;
        io.mode = mode;
        io.totals = ws.totals + (int64_t)m * ix->n_classes;
        io.ws = &ws;
        io.part_d = ws.part_d;
        io.part_i = ws.part_i;
        io.totals_f64 = ws.totals_f64 ? ws.totals_f64 + (int64_t)m * ix->n_classes : nullptr;
        io.q8 = ws.q8;
        io.qsc = ws.qsc;
        io.cand = ws.cand;
        io.upd_cls = ws.upd_cls;
        io.upd_delta = ws.upd_delta;
        int rc = enqueue_batch(ix, plans[m], io, s, kev);
        if (rc) return rc;
        if (kev) {
            LN_HIP(hipEventSynchronize(kev[1]));
            float ms = 0;
            LN_HIP(hipEventElapsedTime(&ms, kev[0], kev[1]));
            kms += ms;
        }
    }
    if (kev) {
        ix->last_timing.dist_kernel_ms = kms;
        ix->last_timing.dist_launches = n_images;
    }
    return LNBNN_OK;
}

extern "C" int lnbnn_classify(lnbnn_index *ix, const void *queries, int dtype, const int64_t *img_offsets,
                              int32_t n_images, int32_t k, int mode, uint32_t flags, int32_t *out_class,
                              void *out_totals, int32_t *out_nbr_idx, float *out_nbr_dist, void *stream)
{
    int rc = validate_classify(ix, queries, dtype, img_offsets, n_images, k, mode, flags, out_class != nullptr,
                               out_nbr_idx, out_nbr_dist);
    if (rc) return rc;
    if (n_images == 0) return LNBNN_OK;
    std::lock_guard<std::mutex> lock(ix->mu);
    LN_HIP(hipSetDevice(ix->device));
    hipStream_t s = stream ? (hipStream_t)stream : ix->own_stream;
    const bool dev = flags & LNBNN_DEVICE_PTRS;
    const bool per_image = flags & LNBNN_PER_IMAGE_LAUNCH;
    const bool timed = flags & LNBNN_TIMING;
    const bool direct = (flags & LNBNN_NO_GRAPH) || timed;   // events inside a graph cannot be read back
    const int kp = k + 1;
    const bool fp8 = is_fp8_mode(mode);
    const int list_len = dist_list_len(mode, k);   // what the distance kernel keeps
    const int64_t n_q = img_offsets[n_images];
    const int64_t rb = row_bytes(dtype, ix->dim);
    const int64_t nc = ix->n_classes;

    // Capacities: a batched call is planned for power-of-two buckets of its
    // descriptor and image counts, so one captured graph serves every batch
    // up to the bucket (the data pointers travel in the batch descriptor).
    Plan plan;
    int64_t part = 0, q_max = 1, q_cap = 1, img_cap = n_images;
    if (per_image) {
        for (int32_t m = 0; m < n_images; ++m) {
            Plan pm;
            const int64_t nm = std::max<int64_t>(1, img_offsets[m + 1] - img_offsets[m]);
            if ((rc = make_plan(ix, mode, list_len, nm, -1, &pm))) return rc;
            part = std::max(part, work_elems(ix, pm, pm.q_cap));
            q_max = std::max(q_max, nm);
        }
        q_cap = std::max<int64_t>(1, n_q);
    } else {
        q_cap = cap_bucket(n_q, 1024);
        img_cap = cap_bucket(n_images, 8);
        if ((rc = make_plan(ix, mode, list_len, q_cap, -1, &plan))) return rc;
        part = work_elems(ix, plan, plan.q_cap);
        q_max = plan.q_cap;
    }
    const bool want_nbr = out_nbr_idx != nullptr;
    if ((rc = ensure_ws(ix, ix->ws, q_cap, img_cap, part, (want_nbr && !dev) ? n_q * kp : 0, dev ? 0 : n_q * rb,
                        fp8)))
        return rc;
    if (fp8 && (rc = ensure_fp8_ws(ix, ix->ws, q_max, fp8_candidates(k), k))) return rc;
    Workspace &ws = ix->ws;

    // the shared workspace may still be read by a call on another stream
    if (ix->ws_used) LN_HIP(hipStreamWaitEvent(s, ix->ws_free, 0));
    // from here on, every exit (errors included) marks the end of this
    // call's use of the workspace on `s`
    struct WsFence {
        lnbnn_index *ix;
        hipStream_t s;
        bool armed;
        ~WsFence()
        {
            if (!armed) return;
            (void)hipEventRecord(ix->ws_free, s);
            ix->ws_used = true;
        }
    } fence{ix, s, true};
    const void *dq = queries;
    if (!dev && n_q > 0) {
        LN_HIP(hipMemcpyAsync(ws.q, queries, (size_t)(n_q * rb), hipMemcpyHostToDevice, s));
        dq = ws.q;
    }
    int32_t *d_cls = dev ? out_class : ws.cls;
    int32_t *d_nbr_i = want_nbr ? (dev ? out_nbr_idx : ws.nbr_idx) : nullptr;
    float *d_nbr_d = want_nbr ? (dev ? out_nbr_dist : ws.nbr_dist) : nullptr;

    hipEvent_t *kev = timed ? ix->tev : nullptr;
    if (timed) LN_HIP(hipEventRecord(ix->tev[2], s));
    if ((rc = status_begin(ws, s))) return rc;
    if (per_image) {
        rc = classify_per_image(ix, dq, img_offsets, n_images, k, mode, d_cls, d_nbr_i, d_nbr_d, s, kev);
        if (rc) return rc;
    } else {
        BatchDesc hb{n_q, n_images, dq, d_cls, d_nbr_i, d_nbr_d};
        LN_HIP(hipMemcpyAsync(ws.bd, &hb, sizeof hb, hipMemcpyHostToDevice, s));
        LN_HIP(hipMemcpyAsync(ws.offsets, img_offsets, (size_t)(n_images + 1) * 8, hipMemcpyHostToDevice, s));
        BatchIO io;
        io.offsets = ws.offsets;
        io.bd = ws.bd;
        io.q_cap = plan.q_cap;
        io.img_cap = img_cap;
        io.k = k;
        io.mode = mode;
        io.totals = ws.totals;
        io.ws = &ws;
        io.part_d = ws.part_d;
        io.part_i = ws.part_i;
        io.totals_f64 = ws.totals_f64;
        io.q8 = ws.q8;
        io.qsc = ws.qsc;
        io.cand = ws.cand;
        io.upd_cls = ws.upd_cls;
        io.upd_delta = ws.upd_delta;
        if (direct) {
            if ((rc = enqueue_batch(ix, plan, io, s, kev))) return rc;
        } else {
            if (ix->graphs.size() >= kMaxGraphs && !ix->graphs.count(graph_key(plan, io)) && ix->ws_used)
                LN_HIP(hipEventSynchronize(ix->ws_free));   // an eviction: no replay in flight
            if ((rc = launch_graph(ix->graphs, ix->graph_clock, ix, plan, io, s))) return rc;
        }
    }
    if ((rc = status_end(ws, s))) return rc;
    if (timed) LN_HIP(hipEventRecord(ix->tev[3], s));

    // outputs
    if (out_totals)
        LN_HIP(hipMemcpyAsync(out_totals, fp8 ? (const void *)ws.totals_f64 : (const void *)ws.totals,
                              (size_t)(n_images * nc * 8), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!dev) {
        LN_HIP(hipMemcpyAsync(out_class, ws.cls, (size_t)n_images * 4, hipMemcpyDeviceToHost, s));
        if (want_nbr) {
            LN_HIP(hipMemcpyAsync(out_nbr_idx, ws.nbr_idx, (size_t)(n_q * kp * 4), hipMemcpyDeviceToHost, s));
            LN_HIP(hipMemcpyAsync(out_nbr_dist, ws.nbr_dist, (size_t)(n_q * kp * 4), hipMemcpyDeviceToHost, s));
        }
    }
    fence.armed = false;
    LN_HIP(hipEventRecord(ix->ws_free, s));
    ix->ws_used = true;
    if (!dev) LN_HIP(hipStreamSynchronize(s));
    if (timed) {
        LN_HIP(hipEventSynchronize(ix->tev[3]));
        float ms = 0;
        if (!per_image) {
            LN_HIP(hipEventElapsedTime(&ms, ix->tev[0], ix->tev[1]));
            ix->last_timing.dist_kernel_ms = ms;
            ix->last_timing.dist_launches = 1;
        }
        LN_HIP(hipEventElapsedTime(&ms, ix->tev[2], ix->tev[3]));
        ix->last_timing.total_ms = ms;
        ix->last_timing.slices = per_image ? 0 : plan.n_slices;
        ix->last_timing.tile_variant = per_image ? -1 : plan.variant;
        ix->has_timing = true;
    }
    // a completed sequence (host pointers, or a timed call) reports a
    // bounded wait that gave up
    if (!dev || timed) return status_check(ws, s);
    return LNBNN_OK;
}

extern "C" int lnbnn_sync_status(lnbnn_index *ix)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    std::lock_guard<std::mutex> lock(ix->mu);
    LN_HIP(hipSetDevice(ix->device));
    if (!ix->ws_used || !ix->ws.h_status) return LNBNN_OK;
    LN_HIP(hipEventSynchronize(ix->ws_free));
    return status_check(ix->ws, ix->own_stream);
}

extern "C" int lnbnn_last_timing(const lnbnn_index *ix, lnbnn_timing *out)
{
    if (!ix || !out) return set_err(LNBNN_EINVAL, "NULL argument");
    if (!ix->has_timing) return set_err(LNBNN_EINVAL, "no timed classify has run on this index");
    *out = ix->last_timing;
    return LNBNN_OK;
}

// ===========================================================================
// variants and autotuner
// ===========================================================================
extern "C" int32_t lnbnn_num_variants(void) { return num_variants(); }
extern "C" const char *lnbnn_variant_name(int32_t v) { return variant_name(v); }

extern "C" int lnbnn_set_tuning(lnbnn_index *ix, int mode, int32_t k, const lnbnn_tuning *t)
{
    if (!ix || !t) return set_err(LNBNN_EINVAL, "NULL argument");
    if (mode < 0 || mode >= kNumModes || !(ix->modes & LNBNN_MODE_BIT(mode))) return set_err(LNBNN_EINVAL, "bad mode");
    if (k < 1 || k > LNBNN_MAX_K) return set_err(LNBNN_EINVAL, "bad k");
    if (t->chunk_tiles < 0 || t->chunk_tiles % 8 != 0) return set_err(LNBNN_EINVAL, "chunk_tiles must be a multiple of 8");
    if (t->max_workgroups < 0) return set_err(LNBNN_EINVAL, "negative max_workgroups");
    const int fmt = index_fmt(ix, mode);
    const int list_len = dist_list_len(mode, k);
    const int kpb = kp_bucket(list_len, fmt);
    if (kpb == 0) return set_err(LNBNN_EINVAL, "k = %d is not supported by mode %d", k, mode);
    if (t->variant >= 0 && !variant_serves(t->variant, mode, fmt, list_len))
        return set_err(LNBNN_EINVAL, "variant %d cannot serve k = %d", t->variant, k);
    std::lock_guard<std::mutex> lock(ix->plan_mu);
    if (t->variant < 0 && t->chunk_tiles == 0 && t->max_workgroups == 0)
        ix->pinned.erase({mode, kpb});
    else
        ix->pinned[{mode, kpb}] = lnbnn_index::Pin{*t, 0};
    return LNBNN_OK;
}

extern "C" int lnbnn_set_variant(lnbnn_index *ix, int mode, int32_t k, int32_t v)
{
    lnbnn_tuning t{v < 0 ? -1 : v, 0, 0};
    return lnbnn_set_tuning(ix, mode, k, &t);
}

// Flat JSON object of string -> integer, the tuning cache format.
static std::map<std::string, int> read_cache(const char *path)
{
    std::map<std::string, int> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t c = s.find(':', j);
        if (c == std::string::npos) break;
        m[key] = atoi(s.c_str() + c + 1);
        i = s.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
    return m;
}

static void write_cache(const char *path, const std::map<std::string, int> &m)
{
    const std::string tmp = std::string(path) + ".tmp";
    std::ofstream f(tmp);
    f << "{\n";
    size_t n = 0;
    for (auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++n < m.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    std::rename(tmp.c_str(), path);
}

extern "C" int lnbnn_autotune(lnbnn_index *ix, const void *queries_dev, int dtype, const int64_t *img_offsets,
                              int32_t n_images, int32_t k, int mode, const char *cache_path,
                              int32_t *best_variant, void *stream)
{
    int rc = validate_classify(ix, queries_dev, dtype, img_offsets, n_images, k, mode, LNBNN_DEVICE_PTRS, true,
                               nullptr, nullptr);
    if (rc) return rc;
    if (!cache_path) {
        const char *e = getenv("LNBNN_TUNE_CACHE");
        if (e && *e) cache_path = e;
    }
    const int fmt = index_fmt(ix, mode);
    const int kpb = kp_bucket(dist_list_len(mode, k), fmt);
    // the setting holds for plans within 8x of this batch's capacity bucket:
    // the fastest shape for a full batch is not the fastest for serving-size
    // batches, which keep the defaults
    const int64_t min_q = cap_bucket(std::max<int64_t>(img_offsets[n_images], 1), 1024) / 8;
    char arch[64] = "gfx";
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ix->device) == hipSuccess) snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    }
    std::ostringstream key;
    key << "arch=" << arch << ",n_refs=" << ix->n_refs << ",dim=" << ix->dim << ",kp=" << kpb << ",mode=" << mode;
    if (cache_path) {
        auto m = read_cache(cache_path);
        auto it = m.find(key.str());
        // cache value: variant | chunk_tiles << 8 (chunk 0 = whole slice)
        const int cv = it != m.end() ? it->second & 0xff : -1;
        const int cc = it != m.end() ? it->second >> 8 : 0;
        if (it != m.end() && variant_serves(cv, mode, fmt, dist_list_len(mode, k)) && cc >= 0 && cc % 8 == 0) {
            {
                std::lock_guard<std::mutex> lock(ix->plan_mu);
                ix->pinned[{mode, kpb}] = lnbnn_index::Pin{lnbnn_tuning{cv, cc, 0}, min_q};
            }
            if (best_variant) *best_variant = cv;
            log_line("tuner: cache hit %s -> %s, chunk %d", key.str().c_str(), variant_name(cv), cc);
            return LNBNN_OK;
        }
    }
    hipStream_t ts = stream ? (hipStream_t)stream : ix->own_stream;
    int32_t *d_cls = nullptr;
    // stream-ordered: freeing it does not synchronise the device
    LN_HIP(hipMallocAsync((void **)&d_cls, std::max<int32_t>(1, n_images) * 4, ts));
    // distance-kernel time of one (variant, chunk) setting: mean of two runs
    // after one warm-up run
    auto time_setting = [&](int v, int chunk, double *ms) {
        lnbnn_tuning t{v, chunk, 0};
        int r = lnbnn_set_tuning(ix, mode, k, &t);
        double tot = 0;
        for (int rep = 0; rep < 3 && !r; ++rep) {
            r = lnbnn_classify(ix, queries_dev, dtype, img_offsets, n_images, k, mode,
                               LNBNN_DEVICE_PTRS | LNBNN_NO_GRAPH | LNBNN_TIMING, d_cls, nullptr, nullptr, nullptr,
                               stream);
            if (!r && rep > 0) tot += ix->last_timing.dist_kernel_ms;
        }
        *ms = tot / 2;
        if (!r) log_line("tuner: mode %d, k %d: %s, chunk %d: %.2f ms", mode, k, variant_name(v), chunk, *ms);
        return r;
    };
    // every variant with whole-slice sweeps, then chunk lengths (chunk-major
    // walk: the workgroups of an XCD sweep the same references together) for
    // the two fastest variants
    std::vector<std::pair<double, int>> by_variant;
    const int list_len = dist_list_len(mode, k);
    for (int v = 0; v < num_variants() && !rc; ++v) {
        if (!variant_serves(v, mode, fmt, list_len)) continue;
        double ms = 0;
        if (!(rc = time_setting(v, 0, &ms))) by_variant.push_back({ms, v});
    }
    std::sort(by_variant.begin(), by_variant.end());
    int best = by_variant.empty() ? -1 : by_variant[0].second, best_chunk = 0;
    double best_ms = by_variant.empty() ? 1e30 : by_variant[0].first;
    for (size_t i = 0; i < by_variant.size() && i < 2 && !rc; ++i) {
        for (int chunk : {2048, 4096, 8192}) {
            double ms = 0;
            if ((rc = time_setting(by_variant[i].second, chunk, &ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = by_variant[i].second;
                best_chunk = chunk;
            }
        }
    }
    (void)hipFreeAsync(d_cls, ts);
    if (rc || best < 0) {
        lnbnn_set_variant(ix, mode, k, -1);
        return rc ? rc : set_err(LNBNN_EINVAL, "no variant can serve mode %d with k = %d", mode, k);
    }
    {
        std::lock_guard<std::mutex> lock(ix->plan_mu);
        ix->pinned[{mode, kpb}] = lnbnn_index::Pin{lnbnn_tuning{best, best_chunk, 0}, min_q};
    }
    if (best_variant) *best_variant = best;
    log_line("tuner: %s -> %s, chunk %d (%.2f ms; %zu variants timed)", key.str().c_str(), variant_name(best),
             best_chunk, best_ms, by_variant.size());
    if (cache_path) {
        auto m = read_cache(cache_path);
        m[key.str()] = best | (best_chunk << 8);
        write_cache(cache_path, m);
    }
    return LNBNN_OK;
}

extern "C" const char *lnbnn_last_error(void) { return g_err.c_str(); }
