// Serving loop: continuous batching of query images over the resident index.
//
// lnbnn_submit copies a request into library memory and queues it.  A
// scheduler thread forms batches in arrival order (requests of one
// (k, mode) per batch; others wait for a later batch) as long as the batch
// fits a slot's capacity, and launches each batch on one of up to four
// slots; a slot owns a stream, a device workspace sized for its capacity
// and pinned staging.  Several slots in flight let the next batch's
// uploads and launches overlap the current batch on the device.  A
// completion thread waits for slots in launch order and publishes results;
// lnbnn_poll hands them out.
//
// Memory admission: every slot's workspace is sized once, from the index's
// HBM budget, for max_batch_desc descriptors; a request larger than that can
// never run and is refused at submit with LNBNN_ENOMEM.
//
// Results do not depend on the batch a request lands in: exact modes add
// exact integers; the FP8 mode reduces each image on its own in a fixed
// order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <ctime>

#include "runtime.h"

using namespace lnbnn;

namespace lnbnn {

static int64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

struct Request {
    uint64_t ticket = 0;
    std::vector<uint8_t> data;     // the query rows, copied at submit
    int64_t n_desc = 0;
    int32_t k = 0;
    int mode = 0;
    int status = LNBNN_EAGAIN;     // LNBNN_EAGAIN until done
    std::string error;
    int32_t cls = 0;
    std::vector<uint8_t> totals;   // n_classes * 8 bytes (int64 or double)
    lnbnn_req_stats st{};
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Workspace ws;
    uint8_t *h_q = nullptr;        // pinned staging
    int64_t *h_off = nullptr;
    BatchDesc *h_bd = nullptr;
    int32_t *h_cls = nullptr;
    uint8_t *h_tot = nullptr;
    std::vector<Request *> batch;
    int64_t batch_desc = 0;        // descriptors of the batch it holds
    int status = LNBNN_OK;
    std::string error;
    bool busy = false;
    std::map<std::string, GraphEntry> graphs;
    uint64_t graph_clock = 0;
};

struct Server {
    lnbnn_index *ix = nullptr;
    int64_t max_batch_desc = 0;
    int32_t max_images = 0;
    int32_t n_slots = 2;
    bool started = false;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv;           // scheduler: queue / free slot / stop
    std::condition_variable cv_done;      // completion: a slot was launched / stop
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    std::deque<Slot *> inflight;
    std::vector<Slot *> slots;
    std::thread sched, compl_thr;
    uint64_t next_ticket = 1;
    int64_t next_batch = 0;
    int64_t pending = 0;                  // tickets not yet consumed
    // memory accounting: the device bytes the slots hold (measured after
    // they are set up, never more than the index's HBM budget), descriptors
    // queued and on the device, and the largest batch / in-flight load so far
    int64_t device_bytes = 0;
    int64_t queued_desc = 0;
    int64_t inflight_desc = 0;
    int64_t peak_batch_desc = 0;
    int64_t peak_inflight_desc = 0;
};

static int64_t row_bytes_for_mode(const lnbnn_index *ix, int mode)
{
    return row_bytes(is_fp8_mode(mode) ? LNBNN_F32 : LNBNN_U8, ix->dim);
}

// Device bytes of one slot for `cap` descriptors and `img_cap` images.
static int64_t slot_bytes(lnbnn_index *ix, int64_t cap, int64_t img_cap)
{
    const bool fp8 = ix->dtype == LNBNN_F32;
    // worst case over the k a request may ask for: the longest lists
    const int kmax = fp8 ? kMaxFp8K : LNBNN_MAX_K;
    int list = 0;
    for (int mode = 0; mode < kNumModes; ++mode)
        if (ix->modes & LNBNN_MODE_BIT(mode)) list = std::max(list, kp_bucket(dist_list_len(mode, kmax), index_fmt(ix, mode)));
    int64_t b = cap * row_bytes_for_mode(ix, fp8 ? LNBNN_FP8_RERANK : 0);
    // partial lists: a plan splits into at most kMaxLists lists per query
    b += std::max((int64_t)kMaxLists * cap * (int64_t)list, (int64_t)ix->n_classes * cap) * 8;
    b += img_cap * (16 + 8 + ix->n_classes * 16 + 4) + 16;
    if (fp8) b += cap * (kDim + 4) + cap * (int64_t)fp8_candidates(kmax) * 4 + cap * kmax * 12;
    return b;
}

static int setup_slot(Server *sv, Slot *sl)
{
    lnbnn_index *ix = sv->ix;
    const bool fp8 = ix->dtype == LNBNN_F32;
    const int64_t cap = sv->max_batch_desc, img = sv->max_images;
    LN_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
    LN_HIP(hipEventCreateWithFlags(&sl->done, hipEventDisableTiming));
    sl->ws.device = ix->device;
    const int kmax = fp8 ? kMaxFp8K : LNBNN_MAX_K;
    // partial lists: the largest layout any (mode, k, batch bucket) plans
    int64_t part = 0;
    for (int mode = 0; mode < kNumModes; ++mode) {
        if (!(ix->modes & LNBNN_MODE_BIT(mode))) continue;
        for (int k = 1; k <= kmax; ++k) {
            const int len = dist_list_len(mode, k);
            for (int64_t q = 1024; ; q = std::min(cap, q * 2)) {
                Plan p;
                if (make_plan(ix, mode, len, std::min(q, cap), -1, &p) == LNBNN_OK)
                    part = std::max(part, work_elems(ix, p, cap));
                if (q >= cap) break;
            }
        }
    }
    const int64_t rb = row_bytes_for_mode(ix, fp8 ? LNBNN_FP8_RERANK : 0);
    int rc = ensure_ws(ix, sl->ws, cap, img, part, 0, cap * rb, fp8);
    if (rc) return rc;
    if (fp8 && (rc = ensure_fp8_ws(ix, sl->ws, cap, fp8_candidates(kmax), kmax))) return rc;
    LN_HIP(hipHostMalloc((void **)&sl->h_q, std::max<int64_t>(1, cap * rb), hipHostMallocDefault));
    LN_HIP(hipHostMalloc((void **)&sl->h_off, (img + 1) * 8, hipHostMallocDefault));
    LN_HIP(hipHostMalloc((void **)&sl->h_bd, sizeof(BatchDesc), hipHostMallocDefault));
    LN_HIP(hipHostMalloc((void **)&sl->h_cls, img * 4, hipHostMallocDefault));
    LN_HIP(hipHostMalloc((void **)&sl->h_tot, img * (int64_t)ix->n_classes * 8, hipHostMallocDefault));
    return LNBNN_OK;
}

static void free_slot(Slot *sl)
{
    drop_graphs(sl->graphs);
    if (sl->h_q) (void)hipHostFree(sl->h_q);
    if (sl->h_off) (void)hipHostFree(sl->h_off);
    if (sl->h_bd) (void)hipHostFree(sl->h_bd);
    if (sl->h_cls) (void)hipHostFree(sl->h_cls);
    if (sl->h_tot) (void)hipHostFree(sl->h_tot);
    if (sl->done) (void)hipEventDestroy(sl->done);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
}

// Enqueue one batch on a slot (the slot's requests are in sl->batch).
static int launch_slot(Server *sv, Slot *sl)
{
    lnbnn_index *ix = sv->ix;
    const int mode = sl->batch[0]->mode;
    const int k = sl->batch[0]->k;
    const bool fp8 = is_fp8_mode(mode);
    const int64_t rb = row_bytes_for_mode(ix, mode);
    int64_t n_q = 0;
    sl->h_off[0] = 0;
    for (size_t i = 0; i < sl->batch.size(); ++i) {
        Request *r = sl->batch[i];
        if (r->n_desc) std::memcpy(sl->h_q + n_q * rb, r->data.data(), (size_t)(r->n_desc * rb));
        n_q += r->n_desc;
        sl->h_off[i + 1] = n_q;
    }
    const int64_t n_img = (int64_t)sl->batch.size();
    Workspace &ws = sl->ws;
    *sl->h_bd = BatchDesc{n_q, n_img, ws.q, ws.cls, nullptr, nullptr};
    LN_HIP(hipMemcpyAsync(ws.q, sl->h_q, (size_t)std::max<int64_t>(rb, n_q * rb), hipMemcpyHostToDevice, sl->stream));
    LN_HIP(hipMemcpyAsync(ws.offsets, sl->h_off, (size_t)(n_img + 1) * 8, hipMemcpyHostToDevice, sl->stream));
    LN_HIP(hipMemcpyAsync(ws.bd, sl->h_bd, sizeof(BatchDesc), hipMemcpyHostToDevice, sl->stream));
    // one captured sequence per power-of-two batch size, so small batches
    // get a plan (reference split) that still fills the GPU
    int64_t bucket = 1024;
    while (bucket < n_q) bucket *= 2;
    bucket = std::min(bucket, sv->max_batch_desc);
    Plan plan;
    int rc = make_plan(ix, mode, dist_list_len(mode, k), std::max<int64_t>(1, bucket), -1, &plan);
    if (rc) return rc;
    BatchIO io;
    io.offsets = ws.offsets;
    io.bd = ws.bd;
    io.q_cap = sv->max_batch_desc;
    io.img_cap = sv->max_images;
    io.k = k;
    io.mode = mode;
    io.totals = ws.totals;
    io.totals_f64 = ws.totals_f64;
    io.ws = &ws;
    io.part_d = ws.part_d;
    io.part_i = ws.part_i;
    io.q8 = ws.q8;
    io.qsc = ws.qsc;
    io.cand = ws.cand;
    io.upd_cls = ws.upd_cls;
    io.upd_delta = ws.upd_delta;
    // part buffers are laid out for the slot capacity; the plan for the
    // bucket only chooses the split and the grid
    plan.q_cap = sv->max_batch_desc;
    if (work_elems(ix, plan, plan.q_cap) > ws.part_cap)
        return set_err(LNBNN_EINVAL, "launch tuning changed after the serving loop sized its buffers");
    // each batch starts from a clear status word (checked by the completer)
    LN_HIP(launch_set_i32(ws.status, 0, sl->stream));
    ws.status_dirty = false;
    if ((rc = launch_graph(sl->graphs, sl->graph_clock, ix, plan, io, sl->stream))) return rc;
    if ((rc = status_end(ws, sl->stream))) return rc;
    LN_HIP(hipMemcpyAsync(sl->h_cls, ws.cls, (size_t)n_img * 4, hipMemcpyDeviceToHost, sl->stream));
    LN_HIP(hipMemcpyAsync(sl->h_tot, fp8 ? (const void *)ws.totals_f64 : (const void *)ws.totals,
                          (size_t)(n_img * ix->n_classes * 8), hipMemcpyDeviceToHost, sl->stream));
    LN_HIP(hipEventRecord(sl->done, sl->stream));
    return LNBNN_OK;
}

static void scheduler(Server *sv)
{
    (void)hipSetDevice(sv->ix->device);
    std::unique_lock<std::mutex> lock(sv->mu);
    for (;;) {
        Slot *free_slot_p = nullptr;
        sv->cv.wait(lock, [&] {
            if (sv->stop) return true;
            if (sv->queue.empty()) return false;
            for (Slot *s : sv->slots)
                if (!s->busy) return true;
            return false;
        });
        if (sv->stop) break;
        for (Slot *s : sv->slots)
            if (!s->busy) {
                free_slot_p = s;
                break;
            }
        // batch: requests of the head's (k, mode), in arrival order
        Slot *sl = free_slot_p;
        sl->batch.clear();
        const int32_t k = sv->queue.front()->k;
        const int mode = sv->queue.front()->mode;
        int64_t sum = 0;
        const int64_t t_admit = now_ns();
        for (auto it = sv->queue.begin(); it != sv->queue.end();) {
            Request *r = *it;
            if (r->k != k || r->mode != mode) {
                ++it;
                continue;
            }
            if (sum + r->n_desc > sv->max_batch_desc || (int32_t)sl->batch.size() >= sv->max_images) break;
            sum += r->n_desc;
            r->st.t_admit_ns = t_admit;
            sl->batch.push_back(r);
            it = sv->queue.erase(it);
        }
        sl->batch_desc = sum;
        sv->queued_desc -= sum;
        sv->inflight_desc += sum;
        sv->peak_batch_desc = std::max(sv->peak_batch_desc, sum);
        sv->peak_inflight_desc = std::max(sv->peak_inflight_desc, sv->inflight_desc);
        sl->busy = true;
        const int64_t bid = sv->next_batch++;
        lock.unlock();
        const int64_t t_start = now_ns();
        sl->status = launch_slot(sv, sl);
        if (sl->status != LNBNN_OK) sl->error = lnbnn_last_error();
        lock.lock();
        for (Request *r : sl->batch) {
            r->st.t_start_ns = t_start;
            r->st.batch_id = bid;
            r->st.batch_images = (int32_t)sl->batch.size();
        }
        sv->inflight.push_back(sl);
        sv->cv_done.notify_all();
    }
}

static void completer(Server *sv)
{
    (void)hipSetDevice(sv->ix->device);
    const int64_t nc = sv->ix->n_classes;
    std::unique_lock<std::mutex> lock(sv->mu);
    for (;;) {
        sv->cv_done.wait(lock, [&] { return !sv->inflight.empty() || sv->stop; });
        if (sv->inflight.empty() && sv->stop) break;
        Slot *sl = sv->inflight.front();
        lock.unlock();
        int status = sl->status;
        std::string error = sl->error;
        if (status == LNBNN_OK) {
            hipError_t e = hipEventSynchronize(sl->done);
            if (e != hipSuccess) {
                status = LNBNN_EDEVICE;
                error = std::string("batch failed: ") + hipGetErrorString(e);
            } else if (*sl->ws.h_status & kStatusWaitGaveUp) {
                status = LNBNN_EDEVICE;
                error = "batch failed: the distance kernel gave up a bounded wait for an LDS stage";
            }
        }
        const int64_t t_done = now_ns();
        lock.lock();
        for (size_t i = 0; i < sl->batch.size(); ++i) {
            Request *r = sl->batch[i];
            r->status = status;
            r->error = error;
            if (status == LNBNN_OK) {
                r->cls = sl->h_cls[i];
                r->totals.assign(sl->h_tot + i * nc * 8, sl->h_tot + (i + 1) * nc * 8);
            }
            r->data.clear();
            r->data.shrink_to_fit();
            r->st.t_done_ns = t_done;
        }
        sl->batch.clear();
        sv->inflight_desc -= sl->batch_desc;
        sl->batch_desc = 0;
        sl->busy = false;
        sv->inflight.pop_front();
        sv->cv.notify_all();
    }
}

static int server_start(lnbnn_index *ix)
{
    Server *sv = ix->server;
    if (sv->started) return LNBNN_OK;
    LN_HIP(hipSetDevice(ix->device));
    if (sv->max_images <= 0) sv->max_images = 1024;
    const bool auto_cap = sv->max_batch_desc <= 0;
    if (auto_cap) {
        // the largest capacity whose slots fit the budget, at most 2^17
        int64_t cap = 1 << 17;
        while (cap > 1024 && sv->n_slots * slot_bytes(ix, cap, sv->max_images) > ix->hbm_budget) cap /= 2;
        sv->max_batch_desc = cap;
    }
    if (sv->n_slots * slot_bytes(ix, sv->max_batch_desc, sv->max_images) > ix->hbm_budget)
        return set_err(LNBNN_ENOMEM, "serving slots (%lld descriptors) exceed the HBM budget",
                       (long long)sv->max_batch_desc);
    for (int i = 0; i < sv->n_slots; ++i) {
        Slot *sl = new Slot();
        sv->slots.push_back(sl);
        int rc = setup_slot(sv, sl);
        if (rc) {
            // undo everything: a later submit starts from scratch
            const std::string msg = lnbnn_last_error();
            for (Slot *d : sv->slots) {
                free_slot(d);
                delete d;
            }
            sv->slots.clear();
            if (auto_cap) sv->max_batch_desc = 0;
            return set_err(rc, "%s", msg.c_str());
        }
    }
    // the budget holds for what was actually allocated, not only for the
    // estimate that chose the capacity
    int64_t held = 0;
    for (Slot *sl : sv->slots) held += sl->ws.bytes();
    if (held > ix->hbm_budget) {
        for (Slot *d : sv->slots) {
            free_slot(d);
            delete d;
        }
        sv->slots.clear();
        if (auto_cap) sv->max_batch_desc = 0;
        return set_err(LNBNN_ENOMEM, "serving slots hold %lld bytes, above the HBM budget of %lld",
                       (long long)held, (long long)ix->hbm_budget);
    }
    sv->device_bytes = held;
    log_line("serving started: %d slots of %lld descriptors / %d images, %lld device bytes of a %lld-byte budget",
             sv->n_slots, (long long)sv->max_batch_desc, sv->max_images, (long long)held, (long long)ix->hbm_budget);
    sv->sched = std::thread(scheduler, sv);
    sv->compl_thr = std::thread(completer, sv);
    sv->started = true;
    return LNBNN_OK;
}

void server_stop(lnbnn_index *ix)
{
    Server *sv = ix->server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    sv->cv_done.notify_all();
    if (sv->sched.joinable()) sv->sched.join();
    if (sv->compl_thr.joinable()) sv->compl_thr.join();
    for (Slot *sl : sv->slots) {
        if (sl->stream) (void)hipStreamSynchronize(sl->stream);
        free_slot(sl);
        delete sl;
    }
    for (auto &kv : sv->reqs) delete kv.second;
    for (Request *r : sv->queue)
        if (!sv->reqs.count(r->ticket)) delete r;
    delete sv;
    ix->server = nullptr;
}

bool server_pending(lnbnn_index *ix)
{
    std::lock_guard<std::mutex> lock(ix->server_mu);
    Server *sv = ix->server;
    if (!sv) return false;
    std::lock_guard<std::mutex> l2(sv->mu);
    return sv->pending > 0;
}

}  // namespace lnbnn

extern "C" int lnbnn_serve_config(lnbnn_index *ix, int64_t max_batch_desc, int32_t max_inflight)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    if (max_batch_desc < 0 || max_inflight < 0 || max_inflight > 4)
        return set_err(LNBNN_EINVAL, "max_batch_desc >= 0 and 0 <= max_inflight <= 4 required");
    std::lock_guard<std::mutex> lock(ix->server_mu);
    if (!ix->server) ix->server = new Server();
    Server *sv = ix->server;
    sv->ix = ix;
    if (sv->started) return set_err(LNBNN_EBUSY, "the serving loop has already started");
    if (max_batch_desc) sv->max_batch_desc = max_batch_desc;
    if (max_inflight) sv->n_slots = max_inflight;
    return LNBNN_OK;
}

extern "C" int lnbnn_serve_info(lnbnn_index *ix, lnbnn_serve_stats *out)
{
    if (!ix || !out) return set_err(LNBNN_EINVAL, "NULL argument");
    *out = lnbnn_serve_stats{};
    out->hbm_budget = ix->hbm_budget;
    std::lock_guard<std::mutex> lock(ix->server_mu);
    Server *sv = ix->server;
    if (!sv || !sv->started) return LNBNN_OK;
    std::lock_guard<std::mutex> l2(sv->mu);
    out->started = 1;
    out->slots = sv->n_slots;
    out->device_bytes = sv->device_bytes;
    out->batch_desc_cap = sv->max_batch_desc;
    out->max_images = sv->max_images;
    out->queued_requests = (int64_t)sv->queue.size();
    out->queued_desc = sv->queued_desc;
    out->inflight_batches = (int32_t)sv->inflight.size();
    out->inflight_desc = sv->inflight_desc;
    out->peak_batch_desc = sv->peak_batch_desc;
    out->peak_inflight_desc = sv->peak_inflight_desc;
    return LNBNN_OK;
}

extern "C" int lnbnn_submit(lnbnn_index *ix, const void *queries, int dtype, int64_t n_desc, int32_t k, int mode,
                            uint64_t *ticket)
{
    if (!ix || !ticket) return set_err(LNBNN_EINVAL, "NULL argument");
    if (n_desc < 0) return set_err(LNBNN_EINVAL, "n_desc < 0");
    if (n_desc > 0 && !queries) return set_err(LNBNN_EINVAL, "NULL queries");
    if (mode < 0 || mode >= kNumModes || !(ix->modes & LNBNN_MODE_BIT(mode)))
        return set_err(LNBNN_EINVAL, "mode %d is not materialised in this index", mode);
    const int want = is_fp8_mode(mode) ? LNBNN_F32 : LNBNN_U8;
    if (dtype != want) return set_err(LNBNN_EINVAL, "dtype %d does not match mode %d", dtype, mode);
    if (k < 1 || k > LNBNN_MAX_K || (int64_t)k + 1 > ix->n_refs) return set_err(LNBNN_EINVAL, "bad k = %d", k);
    if (is_fp8_mode(mode) && (k > kMaxFp8K || (int64_t)fp8_candidates(k) > ix->n_refs))
        return set_err(LNBNN_EINVAL, "FP8 re-rank mode needs k <= %d and 4k <= n_refs", kMaxFp8K);
    std::lock_guard<std::mutex> lock(ix->server_mu);
    if (!ix->server) {
        ix->server = new Server();
        ix->server->ix = ix;
    }
    Server *sv = ix->server;
    if (!sv->started) {
        int rc = server_start(ix);
        if (rc) return rc;
    }
    if (n_desc > sv->max_batch_desc)
        return set_err(LNBNN_ENOMEM, "request of %lld descriptors exceeds the batch capacity %lld of the HBM budget",
                       (long long)n_desc, (long long)sv->max_batch_desc);
    Request *r = new Request();
    r->n_desc = n_desc;
    r->k = k;
    r->mode = mode;
    r->st.t_submit_ns = now_ns();
    r->st.n_desc = (int32_t)n_desc;
    const int64_t bytes = n_desc * row_bytes_for_mode(ix, mode);
    r->data.assign(static_cast<const uint8_t *>(queries), static_cast<const uint8_t *>(queries) + bytes);
    {
        std::lock_guard<std::mutex> l2(sv->mu);
        r->ticket = sv->next_ticket++;
        sv->reqs[r->ticket] = r;
        sv->queue.push_back(r);
        sv->queued_desc += n_desc;
        sv->pending += 1;
        *ticket = r->ticket;
    }
    sv->cv.notify_all();
    return LNBNN_OK;
}

extern "C" int lnbnn_poll(lnbnn_index *ix, uint64_t ticket, int32_t *out_class, void *out_totals,
                          lnbnn_req_stats *stats)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    Server *sv;
    {
        std::lock_guard<std::mutex> lock(ix->server_mu);
        sv = ix->server;
    }
    if (!sv) return set_err(LNBNN_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    std::lock_guard<std::mutex> lock(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return set_err(LNBNN_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->status == LNBNN_EAGAIN) return LNBNN_EAGAIN;
    const int status = r->status;
    if (status == LNBNN_OK) {
        if (out_class) *out_class = r->cls;
        if (out_totals) std::memcpy(out_totals, r->totals.data(), r->totals.size());
    } else {
        set_err(status, "%s", r->error.c_str());
    }
    if (stats) *stats = r->st;
    sv->reqs.erase(it);
    sv->pending -= 1;
    delete r;
    return status;
}
