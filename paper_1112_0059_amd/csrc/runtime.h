// Host runtime shared by the classify path and the serving loop.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/lnbnn.h"
#include "internal.h"

namespace lnbnn {

int set_err(int code, const char *fmt, ...);
int hip_err(hipError_t e, const char *what);
bool fault_injected(const char *site);
bool log_enabled();
void log_line(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

#define LN_HIP(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_err(e_, #expr); \
    } while (0)

// Device buffers for one batch in flight.  Capacities only grow.
struct Workspace {
    int64_t q_cap = 0;          // query descriptors
    int64_t img_cap = 0;        // images
    int64_t part_cap = 0;       // elements of part_d / part_i
    int64_t nbr_cap = 0;        // elements of nbr_idx / nbr_dist
    int64_t qbytes_cap = 0;     // bytes of staged queries
    void *q = nullptr;
    int64_t *offsets = nullptr;
    BatchDesc *bd = nullptr;
    float *part_d = nullptr;
    int32_t *part_i = nullptr;
    unsigned long long *totals = nullptr;
    double *totals_f64 = nullptr;
    int32_t *cls = nullptr;
    int32_t *nbr_idx = nullptr;
    float *nbr_dist = nullptr;
    // FP8 mode
    int64_t q8_cap = 0;         // queries
    int64_t cand_cap = 0;       // elements of cand
    int64_t upd_cap = 0;        // elements of upd_cls / upd_delta
    uint4 *q8 = nullptr;        // [q8_cap, 8] FP8 codes
    int32_t *qsc = nullptr;     // [q8_cap] E8M0 query scales
    int32_t *cand = nullptr;
    int32_t *upd_cls = nullptr;
    double *upd_delta = nullptr;
    // status word of the launch sequences run on this workspace (bit
    // kStatusWaitGaveUp: a bounded stage wait gave up), and its pinned host
    // copy, written after every sequence
    int32_t *status = nullptr;
    int32_t *h_status = nullptr;
    bool status_dirty = false;   // freshly allocated: cleared by the next sequence's stream
    int device = 0;
    ~Workspace();
    int64_t bytes() const;
};

struct Plan {
    int variant = 0;
    int fmt = 0;
    int kpb = 0;                // compiled list length
    int n_slices = 1;
    int n_lists = 2;            // partial lists per query: n_slices * lists per slice
    int tiles_per_slice = 0;
    int grid = 1;
    int chunk_tiles = 8;        // tiles per chunk of the chunk-major walk
    int64_t q_cap = 0;          // capacity the plan (and part buffers) serve
};

// Everything a batch launch sequence needs; pointers are device pointers.
struct BatchIO {
    const Workspace *ws = nullptr;      // owner of the buffers below (capacity checks)
    const void *q = nullptr;
    const int64_t *offsets = nullptr;
    const BatchDesc *bd = nullptr;
    int64_t q_cap = 0;
    int64_t img_cap = 0;
    int32_t k = 0;
    int mode = 0;
    int32_t *cls = nullptr;
    unsigned long long *totals = nullptr;
    double *totals_f64 = nullptr;
    int32_t *nbr_idx = nullptr;
    float *nbr_dist = nullptr;
    float *part_d = nullptr;
    int32_t *part_i = nullptr;
    // FP8 mode
    uint4 *q8 = nullptr;
    int32_t *qsc = nullptr;
    int32_t *cand = nullptr;
    int32_t *upd_cls = nullptr;
    double *upd_delta = nullptr;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;       // LRU stamp
};

// Captured launch sequences of one workspace, keyed by plan and capacity
// bucket (never by the caller's data pointers, which travel in the batch
// descriptor); at most kMaxGraphs are kept, the least recently used is
// destroyed first.
constexpr size_t kMaxGraphs = 8;

struct Server;

}  // namespace lnbnn

struct lnbnn_index {
    int device = 0;
    int dtype = 0;
    int dim = lnbnn::kDim;          // 128, or 160 (location-augmented, INT8 mode only)
    int64_t n_refs = 0;
    int64_t n_pad = 0;
    int32_t n_classes = 0;
    uint32_t modes = 0;
    int64_t hbm_budget = 0;
    int cu_count = 0;
    hipStream_t own_stream = nullptr;

    uint4 *frag[lnbnn::kNumFmt] = {};
    float *seed[lnbnn::kNumFmt] = {};
    int32_t *labels = nullptr;
    float *ref_f32 = nullptr;       // FP8 mode: FP32 references for the re-rank
    int32_t *row_scale = nullptr;   // FP8 mode: E8M0 exponent of every padded row
    uint32_t *parity = nullptr;     // INT8 mode: per-tile mask of ||r - 128||^2 parities
    // original NBNN mode: the class-sorted INT8 copy (each class's rows
    // grouped by the parity of ||r - 128||^2, every group padded to 256
    // rows), its parity masks and 2 x class + parity of each of its tiles
    uint32_t *parity_n = nullptr;
    int32_t *tile_class = nullptr;
    int64_t rows[lnbnn::kNumFmt] = {};   // padded rows of each packed format
    int64_t device_bytes = 0;

    std::mutex mu;                                     // classify path (workspace, graphs)
    std::mutex plan_mu;                                // tuning and occupancy caches
    lnbnn::Workspace ws;
    // (mode, kp bucket) -> launch tuning, for plans of at least min_q queries'
    // capacity (a tuned setting holds for batches of the size it was timed on)
    struct Pin {
        lnbnn_tuning t;
        int64_t min_q;
    };
    std::map<std::pair<int, int>, Pin> pinned;
    std::map<std::tuple<int, int, int>, int> occupancy;  // (variant, fmt, kpb) -> blocks/CU
    std::map<std::string, lnbnn::GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // device buffers replaced by a larger one: kept until the index is
    // freed, since work in flight (or a graph being captured elsewhere) may
    // still use them and hipFree would synchronise the whole device
    std::vector<void *> retired;
    std::mutex retired_mu;
    lnbnn_timing last_timing{};
    bool has_timing = false;
    hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ws_free = nullptr;   // recorded after the last use of `ws`
    bool ws_used = false;

    lnbnn::Server *server = nullptr;   // owned; created by the first submit, deleted by server_stop
    std::mutex server_mu;
};

namespace lnbnn {

// Argument checks shared by the classify entry points (no device call).
int validate_classify(const lnbnn_index *ix, const void *queries, int dtype, const int64_t *off, int32_t n_images,
                      int32_t k, int mode, uint32_t flags, bool has_out_class, const int32_t *nbr_idx,
                      const float *nbr_dist);
int mode_fmt(int mode);
bool is_fp8_mode(int mode);
int index_fmt(const lnbnn_index *ix, int mode);   // mode_fmt, with the 160-element INT8 tiles where they apply
int make_plan(lnbnn_index *ix, int mode, int kp, int64_t q_cap, int forced_variant, Plan *out);
int64_t part_elems(const Plan &p, int64_t q_cap);
// Elements of part_d / part_i a plan needs (the lists, or the original NBNN
// mode's per-class minima, whichever is larger).
int64_t work_elems(const lnbnn_index *ix, const Plan &p, int64_t q_cap);
// Enqueue fill + distance kernel + finish + argmin for one batch (the data
// pointers come from the batch descriptor io.bd).  When `kev` is not null,
// events 0/1 bracket the distance kernel.
int enqueue_batch(lnbnn_index *ix, const Plan &p, const BatchIO &io, hipStream_t s, hipEvent_t *kev);
// Bounded-wait spin limit for the distance kernel (LNBNN_WAIT_SPINS).
int32_t wait_spin_limit();
// Status word handling around a launch sequence on workspace `ws`.
int status_begin(Workspace &ws, hipStream_t s);
int status_end(Workspace &ws, hipStream_t s);
// After the sequence has completed: LNBNN_EDEVICE (and the word cleared) if
// a bounded wait gave up.
int status_check(Workspace &ws, hipStream_t s);
// Capacity bucket: the next power of two >= max(n, lo).
int64_t cap_bucket(int64_t n, int64_t lo);
int ensure_ws(lnbnn_index *ix, Workspace &ws, int64_t q_cap, int64_t img_cap, int64_t part,
              int64_t nbr, int64_t qbytes, bool need_f64);
int ensure_fp8_ws(lnbnn_index *ix, Workspace &ws, int64_t q_cap, int n_cand, int k);
int fp8_candidates(int k);
int dist_list_len(int mode, int k);
int64_t row_bytes(int dtype, int dim);

int launch_graph(std::map<std::string, GraphEntry> &graphs, uint64_t &clock, lnbnn_index *ix, const Plan &p,
                 const BatchIO &io, hipStream_t s);
void drop_graphs(std::map<std::string, GraphEntry> &graphs);
std::string graph_key(const Plan &p, const BatchIO &io);

void server_stop(lnbnn_index *ix);
bool server_pending(lnbnn_index *ix);

}  // namespace lnbnn
