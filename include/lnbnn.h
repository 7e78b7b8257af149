/*
 * lnbnn.h -- C ABI of the MI355X local NBNN library (liblnbnn.so).
 *
 * Local NBNN (McCann & Lowe, Sec. 5, Algorithm 2) classifies a query image
 * from its descriptors d_i: for every d_i it retrieves the k+1 nearest
 * references of one merged index over all classes, takes the (k+1)-th
 * squared distance as the background distance dist_B, and for every class C
 * found among the first k neighbours adds dist_C - dist_B to totals[C], where
 * dist_C is the squared distance to the nearest neighbour of class C.  The
 * image's class is argmin_C totals[C].  The neighbour search here is exact
 * (brute force on the GPU's matrix cores), not the approximate KD-forest the
 * paper uses (Sec. 5.1).
 *
 * Conventions shared by every entry point:
 *   - every function returns 0 (LNBNN_OK) or a negative status; no C++
 *     exception crosses this boundary; lnbnn_last_error() gives a message
 *     for the calling thread's last failure;
 *   - descriptors are row-major [n, dim] with dim == LNBNN_DIM (128, the
 *     SIFT dimension the paper uses, Sec. 6), or LNBNN_DIM_LOC (160) for
 *     location-augmented u8 descriptors (the paper weights a descriptor's
 *     image location by alpha = 1.6, Sec. 6): the library takes all 160
 *     bytes as one vector; how the location is coded into bytes 128..159
 *     is the caller's choice (one exact-integer coding: 16 copies each of
 *     the two coordinate codes, so that 16 (dx^2 + dy^2) carries the
 *     weight);
 *   - distances are squared Euclidean (no square root);
 *   - nearest neighbours are ordered by (distance, reference index): equal
 *     distances go to the lower index; argmin ties go to the lower class;
 *   - all class totals start at 0; classes that own no reference are legal
 *     and are never adjusted;
 *   - borrowed inputs are read only during the call; outputs are
 *     caller-allocated;
 *   - an index is immutable after it is built and may be shared by
 *     lnbnn_classify callers and the serving loop.
 *
 * Environment (read when the named call runs):
 *   LNBNN_HBM_BUDGET   serving budget in bytes (suffix K, M or G allowed) for
 *                      lnbnn_build_index calls that pass hbm_budget_bytes = 0
 *                      (otherwise a quarter of the free device memory);
 *   LNBNN_TUNE_CACHE   tuning cache file lnbnn_autotune reads and writes when
 *                      its cache_path is NULL;
 *   LNBNN_LOG          1: one line per index build, graph capture, tuner
 *                      decision and serving start on stderr, prefixed
 *                      "[lnbnn]"; unset or 0: silent;
 *   LNBNN_WAIT_SPINS   bound of the distance kernel's stage waits (see
 *                      lnbnn_classify);
 *   LNBNN_FAULT        alloc | launch: the named step fails with an error
 *                      (to exercise error paths; never set in production).
 */
#ifndef LNBNN_H
#define LNBNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LNBNN_DIM 128
#define LNBNN_DIM_LOC 160       /* location-augmented u8 descriptors: INT8 mode only */
#define LNBNN_MAX_K 32          /* k <= 32, so at most 33 neighbours */

typedef struct lnbnn_index lnbnn_index;   /* opaque, library-owned */

/* status codes */
enum {
    LNBNN_OK = 0,
    LNBNN_EINVAL = -1,    /* bad argument; nothing was done */
    LNBNN_ENOMEM = -2,    /* device allocation failed, or a request can never fit the budget */
    LNBNN_EDEVICE = -3,   /* a HIP call failed (message carries hipGetErrorString) */
    LNBNN_EAGAIN = -4,    /* ticket still pending */
    LNBNN_ENOENT = -5,    /* unknown or already consumed ticket */
    LNBNN_EBUSY = -6      /* index still has pending tickets */
};

/* descriptor element types */
enum { LNBNN_U8 = 0, LNBNN_F32 = 1 };

/* search modes (bit i of a mode mask selects mode i) */
enum {
    LNBNN_EXACT_F16 = 0,   /* u8 data, FP16 matrix cores, FP32 accumulate: exact */
    LNBNN_EXACT_BF16 = 1,  /* u8 data, BF16 matrix cores, FP32 accumulate: exact */
    LNBNN_FP8_RERANK = 2,  /* f32 data: FP8 e4m3 candidate pass, exact FP32 re-rank of 4k <= 128
                              candidates.  For k <= 16 the candidates are exactly the 4k
                              references with the smallest FP8 keys (ties: lower index), for
                              every launch plan; for k > 16 the best 4k of per-row-half lists
                              of 64 keys each (the FP8 top 64 are among them) */
    LNBNN_EXACT_I8 = 3,    /* u8 data shifted by -128, INT8 matrix cores, INT32 accumulate: exact
                              (the fastest exact mode; results identical to FP16/BF16) */
    LNBNN_FP8_RERANK_2K = 4,  /* as LNBNN_FP8_RERANK with shorter candidate lists: the best 4k FP8
                              keys of the union of per-row-half lists of 2k keys each (the FP8
                              top 2k are always among them); faster, and the candidates may
                              depend on the launch plan.  Built together with FP8_RERANK */
    LNBNN_NBNN_I8 = 5      /* u8 data: the original NBNN rule (Sec. 1, Algorithm 1; Sec. 3): totals
                              are sum over the image's descriptors d of ||d - NN_C(d)||^2 for
                              every class C, the class is their argmin; exact (INT8 matrix
                              cores on a class-sorted copy of the index, every class padded to
                              256 rows).  k is not used (Algorithm 1 has none) but must be
                              valid; no neighbour lists.  Needs every class to own a reference */
};
#define LNBNN_MODE_BIT(m) (1u << (m))

/* flags */
enum {
    LNBNN_DEVICE_PTRS = 1,        /* data pointers are device pointers, work is ordered on `stream` */
    LNBNN_PER_IMAGE_LAUNCH = 2,   /* classify: one launch sequence per image (plain baseline) */
    LNBNN_NO_GRAPH = 4,           /* classify: launch kernels directly instead of replaying a hipGraph */
    LNBNN_TIMING = 8              /* classify: record device time of the distance kernel
                                     (lnbnn_last_timing); implies direct launches */
};

/*
 * Build the merged reference index (Algorithm 2's first requirement: one
 * nearest-neighbour index over the descriptors of all classes; its second:
 * the class lookup Class(p), Sec. 6.1's per-descriptor "accessory data").
 *
 *   refs       [n_refs, dim] LNBNN_U8 (values 0..255) or LNBNN_F32
 *   dim        LNBNN_DIM, or LNBNN_DIM_LOC with U8 data and mode_mask =
 *              LNBNN_MODE_BIT(LNBNN_EXACT_I8) (queries then carry 160 bytes)
 *   labels     [n_refs] int32 class of every reference, in [0, n_classes)
 *   mode_mask  which search modes to materialise: U8 data allows the exact
 *              modes (F16, BF16, I8) and NBNN_I8, F32 data the two FP8 modes
 *              (they share one packed copy)
 *   hbm_budget_bytes  device workspace cap for the serving loop (0 = 1/4 of
 *              the free device memory after the index is resident)
 *   flags      LNBNN_DEVICE_PTRS: refs and labels are device pointers
 *   stream     hipStream_t for the upload and packing kernels, or NULL
 *   out        receives the index; *out is untouched on failure
 *
 * Memory: the packed references stay resident (N x 256 B per FP16/BF16
 * mode, N x dim B for INT8, N x 128 B FP8 plus N x 512 B FP32 for the
 * re-rank, about N x 132 B for the class-sorted NBNN copy), with FP32 norms
 * (4 B) and int32 labels (4 B) per reference.
 * Errors: EINVAL (NULL pointer, dim not 128 or 160, 160 with other data or
 * modes than u8 INT8, n_refs < 1 or >= 2^31-256,
 * n_classes < 1, label out of range, empty or data-incompatible mode mask),
 * ENOMEM, EDEVICE.  Blocks until the index is resident.
 */
int lnbnn_build_index(const void *refs, int dtype, int64_t n_refs, int32_t dim,
                      const int32_t *labels, int32_t n_classes,
                      uint32_t mode_mask, int64_t hbm_budget_bytes,
                      uint32_t flags, void *stream, lnbnn_index **out);

/* Release an index and every device buffer it owns.  EBUSY while serving
 * tickets are pending (nothing is freed then).  NULL is accepted. */
int lnbnn_index_free(lnbnn_index *ix);

/* Basic facts of an index (any pointer may be NULL). */
int lnbnn_index_info(const lnbnn_index *ix, int64_t *n_refs, int32_t *n_classes,
                     uint32_t *mode_mask, int64_t *device_bytes);

/*
 * Classify a batch of query images (Algorithm 2 for every image).
 *
 *   queries     [n_desc, dim] descriptors of all images, concatenated, with
 *               the index's dim; LNBNN_U8 for the exact modes, LNBNN_F32 for
 *               FP8_RERANK
 *   img_offsets host int64 [n_images + 1] CSR offsets (always host memory):
 *               image m owns descriptors [img_offsets[m], img_offsets[m+1]);
 *               must start at 0 and be non-decreasing; empty images are
 *               legal (their totals stay 0 and their class is 0)
 *   k           neighbourhood size, 1 <= k <= LNBNN_MAX_K and k + 1 <= n_refs
 *               (FP8_RERANK also needs 4k <= n_refs)
 *   mode        one materialised search mode
 *   flags       LNBNN_DEVICE_PTRS / LNBNN_PER_IMAGE_LAUNCH / LNBNN_NO_GRAPH /
 *               LNBNN_TIMING
 *   out_class   [n_images] int32 argmin class per image (required)
 *   out_totals  [n_images, n_classes] per-class totals, or NULL: int64 for the
 *               exact modes and NBNN_I8 (exact integers), double for the FP8
 *               modes
 *   out_nbr_idx, out_nbr_dist  [n_desc, k + 1] neighbour indices (int32) and
 *               squared distances (float; exact integers in the exact
 *               modes), or NULL (must be NULL for NBNN_I8)
 *   stream      hipStream_t the work is ordered on (NULL = the index's own)
 *
 * Host pointers (default): blocks until outputs are written.
 * LNBNN_DEVICE_PTRS: queries and outputs are device pointers; the call
 * returns once the work is enqueued on `stream` (outputs valid when the
 * stream reaches that point); img_offsets is still host memory.
 * Batched calls replay a captured launch sequence; one sequence serves
 * every batch up to power-of-two buckets of its descriptor and image
 * counts (the data pointers are read on the device), and at most eight
 * sequences per index are kept (least recently used first out).
 * The distance kernel's waits for its LDS stages are bounded
 * (LNBNN_WAIT_SPINS sleep rounds, default 2^20); a wait that gives up makes
 * the call's results invalid and is reported as LNBNN_EDEVICE by the call
 * itself when it blocks (host pointers, or LNBNN_TIMING), else by
 * lnbnn_sync_status.
 * Errors: EINVAL (NULL required pointer, dtype/mode mismatch, mode not
 * materialised, k out of range, bad offsets, n_images < 0), ENOMEM, EDEVICE.
 */
int lnbnn_classify(lnbnn_index *ix, const void *queries, int dtype,
                   const int64_t *img_offsets, int32_t n_images,
                   int32_t k, int mode, uint32_t flags,
                   int32_t *out_class, void *out_totals,
                   int32_t *out_nbr_idx, float *out_nbr_dist,
                   void *stream);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the batched
 * classification of lnbnn_classify with LNBNN_DEVICE_PTRS, which calls no
 * hipMalloc/hipFree or other allocating routine.  Everything the launch
 * sequence needs beyond the caller's buffers lives in a library-owned
 * device array of 64 MiB per GPU, held until the process ends.
 *
 *   queries_dev, out_class_dev  device pointers as in lnbnn_classify
 *   img_offsets  host int64 [n_images + 1] CSR offsets, as in lnbnn_classify
 *   out_totals_dev  device [n_images, n_classes] totals (int64, or double
 *               for FP8_RERANK), or NULL
 *   out_nbr_idx_dev, out_nbr_dist_dev  device [n_desc, k + 1], or NULL
 *   out_status_dev  device int32 or NULL: set to nonzero if a bounded stage
 *               wait of the distance kernel gave up (results invalid);
 *               cleared by the call itself
 *   stream      hipStream_t (NULL = the index's own); the call returns once
 *               the work is enqueued (direct launches, no graph)
 *
 * Every call on a GPU shares that GPU's scratch array: calls that overlap
 * on one GPU (other host threads, or streams not ordered after each other)
 * race on it.  A batch whose scratch need (partial lists, totals when
 * out_totals_dev is NULL, the FP8 mode's candidate buffers) exceeds the
 * array is refused with LNBNN_ENOMEM before anything is enqueued.
 * Errors: as lnbnn_classify, and ENOMEM for a batch too large for the array.
 */
int lnbnn_classify_noalloc(lnbnn_index *ix, const void *queries_dev, int dtype,
                           const int64_t *img_offsets, int32_t n_images, int32_t k, int mode,
                           int32_t *out_class_dev, void *out_totals_dev,
                           int32_t *out_nbr_idx_dev, float *out_nbr_dist_dev,
                           int32_t *out_status_dev, void *stream);

/* Wait for every lnbnn_classify call enqueued on this index and report
 * LNBNN_EDEVICE if a distance-kernel launch since the last report gave up a
 * bounded stage wait (the results of that call are invalid); LNBNN_OK
 * otherwise.  For LNBNN_DEVICE_PTRS callers, whose calls do not block. */
int lnbnn_sync_status(lnbnn_index *ix);

/* Device time of the last LNBNN_TIMING classify on this index: the summed
 * durations of the distance + top-(k+1) kernel launches and of the whole
 * launch sequence, in milliseconds (HIP events on the launch stream), and
 * the number of distance-kernel launches.  EINVAL if no timed call ran. */
typedef struct lnbnn_timing {
    double dist_kernel_ms;
    double total_ms;
    int32_t dist_launches;
    int32_t slices;            /* reference slices per query block */
    int32_t tile_variant;      /* kernel variant id chosen for the call */
} lnbnn_timing;
int lnbnn_last_timing(const lnbnn_index *ix, lnbnn_timing *out);

/*
 * Project autotuner for the batched launch: times every kernel variant that
 * can serve (mode, k) on the given query batch (same arguments as a
 * LNBNN_DEVICE_PTRS classify without outputs), then chunk lengths of the
 * chunk-major walk (lnbnn_tuning.chunk_tiles) for the two fastest, and keeps
 * the fastest setting for this index, keyed by (arch, n_refs, dim, k bucket,
 * mode).  The setting applies to batches of comparable size: those whose
 * capacity (the power of two >= max(descriptors, 1024)) is at least 1/8 of
 * this batch's; smaller batches (e.g. the serving loop's) keep the default
 * shapes.  If `cache_path` is not NULL the choice is merged into that JSON
 * file (value = variant | chunk_tiles << 8), and a later call with the same
 * key reads it back instead of timing again.  Results do not depend on the
 * setting: every variant and walk computes the same exact selection.
 * `best_variant` (may be NULL) receives the chosen variant id.
 */
int lnbnn_autotune(lnbnn_index *ix, const void *queries_dev, int dtype,
                   const int64_t *img_offsets, int32_t n_images,
                   int32_t k, int mode, const char *cache_path,
                   int32_t *best_variant, void *stream);

/* Pin a kernel variant for (mode, k) on this index (-1 = heuristic choice). */
int lnbnn_set_variant(lnbnn_index *ix, int mode, int32_t k, int32_t variant);

/* Full launch tuning for (mode, k) on this index, for batches of every size.
 * variant: kernel variant (-1 = heuristic); chunk_tiles: 32-row reference
 * tiles a workgroup runs for one query block before moving to its next block
 * (0 = default, else a multiple of 8); max_workgroups: cap on the persistent
 * grid (0 = every resident slot).  No setting changes any result. */
typedef struct lnbnn_tuning {
    int32_t variant;
    int32_t chunk_tiles;
    int32_t max_workgroups;
} lnbnn_tuning;
int lnbnn_set_tuning(lnbnn_index *ix, int mode, int32_t k, const lnbnn_tuning *t);

/* Number of kernel variants and a printable name of variant `v`. */
int32_t lnbnn_num_variants(void);
const char *lnbnn_variant_name(int32_t v);

/*
 * Serving: continuous batching over the resident index.
 *
 * lnbnn_submit copies one query image (host memory, [n_desc, dim]) into
 * library-owned pinned staging and returns a ticket at once.  A scheduler
 * thread admits queued requests in arrival order while their device
 * footprint fits the index's HBM budget, packs them into a batch, and keeps
 * up to two batches in flight on separate streams; requests that arrive while
 * a batch runs join the next one.  Results do not depend on the batch a
 * request lands in (exact modes: exact integer totals; FP8_RERANK: each
 * image's FP64 totals are summed by one workgroup in a fixed order:
 * descriptor, then neighbour rank).
 * Errors: EINVAL (bad pointer, n_desc < 0, k, mode, dtype), ENOMEM (the
 * request alone exceeds the budget), EDEVICE.
 */
typedef struct lnbnn_req_stats {
    int64_t t_submit_ns;   /* CLOCK_MONOTONIC */
    int64_t t_admit_ns;    /* admitted into a batch */
    int64_t t_start_ns;    /* batch enqueued on the device */
    int64_t t_done_ns;     /* batch finished on the device */
    int64_t batch_id;
    int32_t n_desc;
    int32_t batch_images;  /* images in the same batch */
} lnbnn_req_stats;

int lnbnn_submit(lnbnn_index *ix, const void *queries, int dtype, int64_t n_desc,
                 int32_t k, int mode, uint64_t *ticket);

/* LNBNN_EAGAIN while pending; LNBNN_OK once done (fills out_class, and
 * out_totals [n_classes] if not NULL, int64 or double as in classify, and
 * stats if not NULL) -- the ticket is then consumed; LNBNN_ENOENT for an
 * unknown or consumed ticket; a device failure of the request's batch is
 * reported here as LNBNN_EDEVICE (the ticket is consumed). */
int lnbnn_poll(lnbnn_index *ix, uint64_t ticket, int32_t *out_class,
               void *out_totals, lnbnn_req_stats *stats);

/* Serving parameters (before the first submit, else EBUSY): maximum
 * descriptors per batch and batches in flight (1..4); 0 keeps a default. */
int lnbnn_serve_config(lnbnn_index *ix, int64_t max_batch_desc, int32_t max_inflight);

/*
 * Memory accounting of the serving loop (a snapshot; the loop keeps running).
 * The slots' device workspaces are allocated once when the loop starts and
 * their measured size (device_bytes) never exceeds hbm_budget (the index's
 * budget, lnbnn_build_index): a start that would exceed it fails with ENOMEM.
 * Each request is admitted into a batch only while the batch's descriptors
 * stay within batch_desc_cap and its images within max_images, so at most
 * slots * batch_desc_cap descriptors are on the device at any time.
 * Before the loop has started only hbm_budget is filled (started = 0).
 * Errors: EINVAL (NULL argument).
 */
typedef struct lnbnn_serve_stats {
    int64_t hbm_budget;          /* bytes */
    int64_t device_bytes;        /* bytes held by the slots' workspaces */
    int64_t batch_desc_cap;      /* descriptors per batch */
    int64_t queued_requests;
    int64_t queued_desc;         /* descriptors waiting for a batch */
    int64_t inflight_desc;       /* descriptors of batches on the device */
    int64_t peak_batch_desc;     /* largest batch admitted so far */
    int64_t peak_inflight_desc;  /* most descriptors on the device at once so far */
    int32_t max_images;          /* images per batch */
    int32_t slots;               /* batches in flight at most */
    int32_t inflight_batches;
    int32_t started;
} lnbnn_serve_stats;

int lnbnn_serve_info(lnbnn_index *ix, lnbnn_serve_stats *out);

/* Thread-local message of the calling thread's last failure ("" if none). */
const char *lnbnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LNBNN_H */
