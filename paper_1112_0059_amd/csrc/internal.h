// Internal interface between the C-ABI runtime and the HIP kernels.
// Nothing here crosses the public boundary (include/lnbnn.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lnbnn {

constexpr int kDim = 128;
constexpr int kDimLoc = 160;             // location-augmented descriptors (INT8 mode only)
constexpr int kTileRows = 32;            // rows of one MFMA A tile
constexpr int kMaxLists = 64;            // partial lists per query a plan may split into
constexpr int kPadRows = 256;            // index rows are padded to this multiple
constexpr int kMaxKP = 33;               // k + 1 <= 33
constexpr int kMaxFp8K = 32;             // FP8 mode re-ranks 4k <= 128 candidates

// Element formats of the packed reference tiles (FMT_I8L: INT8 tiles of
// 160-element rows, five K steps; FMT_I8N: INT8 tiles of the class-sorted
// copy of the index that the original NBNN rule sweeps).
enum Fmt { FMT_F16 = 0, FMT_BF16 = 1, FMT_FP8 = 2, FMT_I8 = 3, FMT_I8L = 4, FMT_I8N = 5 };
constexpr int kNumFmt = 6;
constexpr int kNumModes = 6;             // search modes of include/lnbnn.h

// Batch shape and the batch's data pointers, read on the device, so one
// captured launch sequence serves every batch (and any caller buffers) up
// to the capacity it was captured for.
struct BatchDesc {
    int64_t n_q;        // query descriptors in the batch
    int64_t n_img;      // images in the batch
    const void *q;      // queries [n_q, dim]: u8 (exact modes) or f32 (FP8 mode)
    int32_t *cls;       // [n_img] argmin class per image
    int32_t *nbr_idx;   // [n_q, k+1] neighbour indices, or null
    float *nbr_dist;    // [n_q, k+1] squared distances, or null
};

// A distance-kernel variant: queries per wave = qt * nt, reference tiles
// per LDS stage = mt, waves per workgroup.  qt is the MFMA output block's
// query width (32: 32x32 blocks, two lists per query; 16: 16x16 blocks, four
// lists per query).  pl = 1: the two lanes of a query in a 32x32 block
// share one list (held by one of them).  The list length the kernel keeps
// (>= k + 1) is a separate compile-time parameter.
struct Variant {
    int nt;
    int mt;
    int waves;
    int buffers;    // LDS stages: the kernel keeps buffers - 1 stages in flight
    int qt;
    int pl;         // 1: one list per query (pair lists), else one per lane group
};

struct DistArgs {
    const void *q;              // FP8 codes [q_cap, 128] (FP8 mode); null: the u8 queries bd->q
    const int32_t *q_scale;     // fp8: per-query exponent bias (else null)
    const BatchDesc *bd;        // device batch descriptor
    const uint4 *frag;          // packed reference fragments
    const float *seed;          // per-row accumulator seed (norm), +inf on padding
    const int32_t *row_scale;   // fp8: per-row exponent bias (else null)
    const uint32_t *parity;     // int8: per-tile mask of the rows' ||r - 128||^2 parities
    int64_t n_tiles;            // 32-row tiles in the padded index (multiple of 8)
    int32_t tiles_per_slice;    // multiple of 8
    int32_t n_slices;
    int32_t chunk_tiles;        // tiles one item runs before the workgroup moves on (multiple of 8)
    int64_t q_cap;              // capacity: part buffers are laid out for q_cap queries
    float *part_d;              // [n_slices * lists per query][q_cap][kp]
    int32_t *part_i;
    int32_t *status;            // bit 0: a bounded stage wait gave up (set by the kernels that
                                // read the lists, which carry the mark as a NaN key)
    int32_t spin_limit;         // sleep rounds a stage wait allows before it gives up
    // original NBNN (FMT_I8N): 2 x class + parity of every 32-row tile (the
    // class-sorted copy holds one class and one parity of ||r - 128||^2 per
    // stage), and the per-class minimum key of every query,
    // [n_classes][q_cap] (atomic minima)
    const int32_t *tile_class;
    int32_t *cls_min;
};

struct NbnnArgs {
    const BatchDesc *bd;
    const int64_t *offsets;     // device [n_img + 1]
    const int32_t *cls_min;     // [n_classes][q_cap] minimum key per class and query
    int64_t q_cap;
    int32_t n_classes;
    unsigned long long *totals; // [n_img, n_classes] int64: sum over the image of the per-class distances
};

// Bits of the device status word of a launch sequence.
constexpr int32_t kStatusWaitGaveUp = 1;

struct RerankArgs {
    const BatchDesc *bd;
    const int64_t *offsets;     // device [n_img + 1]
    const float *ref_f32;       // f32 references [n_refs, 128]
    const int32_t *labels;
    int64_t n_refs;
    int32_t n_lists;            // n_slices * lists per query (at most 64)
    int32_t kp_stride;          // list length in the part buffers
    int32_t n_cand;             // candidates kept per query (4k)
    int32_t k;
    int32_t n_classes;
    int64_t q_cap;
    const float *part_d;
    const int32_t *part_i;
    int32_t *cand;              // [q_cap, n_cand]
    int32_t *upd_cls;           // [q_cap, k]: class of the update of rank j, -1 if none
    double *upd_delta;          // [q_cap, k]
    double *totals_f64;         // [n_img, n_classes]
    int32_t *status;            // set when a list carries a stage-wait mark
};

struct FinishArgs {
    int32_t dim;                // row length of the u8 queries bd->q (for ||q - shift||^2):
                                // 128, or 160 (location-augmented, INT8 mode)
    int32_t q_shift;            // 0, or 128 where the keys are those of r - 128 and q - 128
    const BatchDesc *bd;
    const int64_t *offsets;     // device [n_img + 1]
    const int32_t *labels;      // [n_refs]
    int64_t n_refs;
    int32_t n_lists;            // n_slices * lists per query (at most 64)
    int32_t kp_stride;          // list length in the part buffers
    int32_t k;
    int32_t n_classes;
    int64_t q_cap;
    const float *part_d;
    const int32_t *part_i;
    unsigned long long *totals; // [n_img, n_classes] int64 (two's complement)
    int32_t *status;            // set when a list carries a stage-wait mark
};

// number of kernel variants and their parameters
int num_variants();
Variant variant(int v);
const char *variant_name(int v);
bool variant_supports(int v, int fmt, int kp);
int kp_bucket(int kp, int fmt);         // list length compiled for kp (0 = unsupported)

// (tag, operand policy, format, list length) of every compiled distance
// kernel instance set; the build compiles dist_inst.hip once per entry.
#define LNBNN_DIST_INSTANCES(X)   \
    X(f16, OpF16, FMT_F16, 2)     \
    X(f16, OpF16, FMT_F16, 6)     \
    X(f16, OpF16, FMT_F16, 11)    \
    X(f16, OpF16, FMT_F16, 16)    \
    X(f16, OpF16, FMT_F16, 21)    \
    X(f16, OpF16, FMT_F16, 33)    \
    X(bf16, OpBF16, FMT_BF16, 2)  \
    X(bf16, OpBF16, FMT_BF16, 6)  \
    X(bf16, OpBF16, FMT_BF16, 11) \
    X(bf16, OpBF16, FMT_BF16, 16) \
    X(bf16, OpBF16, FMT_BF16, 21) \
    X(bf16, OpBF16, FMT_BF16, 33) \
    X(i8, OpI8, FMT_I8, 2)        \
    X(i8, OpI8, FMT_I8, 6)        \
    X(i8, OpI8, FMT_I8, 11)       \
    X(i8, OpI8, FMT_I8, 16)       \
    X(i8, OpI8, FMT_I8, 21)       \
    X(i8, OpI8, FMT_I8, 33)       \
    X(i8l, OpI8L, FMT_I8L, 2)     \
    X(i8l, OpI8L, FMT_I8L, 6)     \
    X(i8l, OpI8L, FMT_I8L, 11)    \
    X(i8l, OpI8L, FMT_I8L, 16)    \
    X(i8l, OpI8L, FMT_I8L, 21)    \
    X(i8l, OpI8L, FMT_I8L, 33)    \
    X(i8n, OpI8N, FMT_I8N, 1)     \
    X(fp8, OpFP8, FMT_FP8, 4)     \
    X(fp8, OpFP8, FMT_FP8, 8)     \
    X(fp8, OpFP8, FMT_FP8, 20)    \
    X(fp8, OpFP8, FMT_FP8, 40)    \
    X(fp8, OpFP8, FMT_FP8, 64)

// Upload-side packing.  refs_u8 / refs_f32 are device pointers.
hipError_t launch_pack_u8(const uint8_t *refs, int64_t n_refs, int64_t n_pad, int fmt,
                          uint4 *frag, float *seed, hipStream_t s);
// perm (device, may be null): row r of the packed index holds reference
// perm[r], or padding where perm[r] < 0 (null: row r holds reference r)
hipError_t launch_pack_i8(const uint8_t *refs, int64_t n_refs, int64_t n_pad, int dim, uint4 *frag,
                          int32_t *seed, uint32_t *parity, hipStream_t s, const int32_t *perm = nullptr);
hipError_t launch_fp8_index(const float *refs, int64_t n_refs, int64_t n_pad, uint4 *frag, float *seed,
                            int32_t *row_scale, hipStream_t s);
hipError_t launch_fp8_qprep(const BatchDesc *bd, int64_t q_cap, uint4 *q8, int32_t *qsc, hipStream_t s);
hipError_t launch_rerank(const RerankArgs &a, int64_t q_cap, int64_t img_cap, hipStream_t s);
int grid_for(int64_t n, int block, int cap);

hipError_t launch_dist_topk(int variant, int fmt, int kp, const DistArgs &a, int grid,
                            hipStream_t s);
int dist_topk_blocks_per_cu(int variant, int fmt, int kp);

hipError_t launch_fill_u64(unsigned long long *p, int64_t n_elems_cap, const BatchDesc *bd,
                           int32_t n_classes, hipStream_t s);
hipError_t launch_finish(const FinishArgs &a, int64_t q_cap, hipStream_t s);
hipError_t launch_argmin(const unsigned long long *totals, const BatchDesc *bd, int64_t img_cap,
                         int32_t n_classes, hipStream_t s);
hipError_t launch_set_i32(int32_t *p, int32_t v, hipStream_t s);
// per reference row: parity of ||r - 128||^2 (u8 rows, dim a multiple of 16)
hipError_t launch_row_parity(const uint8_t *refs, int64_t n_refs, int dim, uint8_t *out, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, int64_t stride, int64_t rows, const BatchDesc *bd,
                           hipStream_t s);
hipError_t launch_nbnn_totals(const NbnnArgs &a, int64_t img_cap, hipStream_t s);

}  // namespace lnbnn
