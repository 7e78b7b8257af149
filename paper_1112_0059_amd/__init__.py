"""Python binding of liblnbnn.so, the MI355X local NBNN library.

Argument marshalling only: every step of the search and scoring runs in the
library's HIP kernels.  Functions carry the names of the C ABI in
``include/lnbnn.h``.  Host inputs are numpy arrays; device inputs are torch
tensors on a ROCm device (their ``data_ptr()`` is passed with
``LNBNN_DEVICE_PTRS`` and the work is ordered on torch's current stream).

Importing this package does not need a GPU; loading the library does need
the built ``liblnbnn.so`` next to this file and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LNBNN_LIBRARY: another build of the same sources (the tests' host-sanitizer build)
LIB_PATH = os.environ.get("LNBNN_LIBRARY") or os.path.join(_HERE, "liblnbnn.so")

# status codes, element types, modes, flags (values of include/lnbnn.h)
LNBNN_OK, LNBNN_EINVAL, LNBNN_ENOMEM, LNBNN_EDEVICE = 0, -1, -2, -3
LNBNN_EAGAIN, LNBNN_ENOENT, LNBNN_EBUSY = -4, -5, -6
LNBNN_U8, LNBNN_F32 = 0, 1
LNBNN_EXACT_F16, LNBNN_EXACT_BF16, LNBNN_FP8_RERANK, LNBNN_EXACT_I8 = 0, 1, 2, 3
LNBNN_FP8_RERANK_2K, LNBNN_NBNN_I8 = 4, 5
FP8_MODES = (LNBNN_FP8_RERANK, LNBNN_FP8_RERANK_2K)
LNBNN_DEVICE_PTRS, LNBNN_PER_IMAGE_LAUNCH, LNBNN_NO_GRAPH, LNBNN_TIMING = 1, 2, 4, 8
LNBNN_DIM = 128
LNBNN_DIM_LOC = 160
LNBNN_MAX_K = 32


def LNBNN_MODE_BIT(m: int) -> int:
    return 1 << m


class LnbnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lnbnn error {code}: {msg}")
        self.code = code


class lnbnn_timing(ctypes.Structure):
    _fields_ = [("dist_kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("dist_launches", ctypes.c_int32), ("slices", ctypes.c_int32),
                ("tile_variant", ctypes.c_int32)]


class lnbnn_tuning(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("chunk_tiles", ctypes.c_int32),
                ("max_workgroups", ctypes.c_int32)]


class lnbnn_serve_stats(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("batch_desc_cap", ctypes.c_int64), ("queued_requests", ctypes.c_int64),
                ("queued_desc", ctypes.c_int64), ("inflight_desc", ctypes.c_int64),
                ("peak_batch_desc", ctypes.c_int64), ("peak_inflight_desc", ctypes.c_int64),
                ("max_images", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("inflight_batches", ctypes.c_int32), ("started", ctypes.c_int32)]


class lnbnn_req_stats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("batch_id", ctypes.c_int64), ("n_desc", ctypes.c_int32),
                ("batch_images", ctypes.c_int32)]


_lib = None


def load():
    """Load liblnbnn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # One HIP runtime per process: torch ships its own libamdhip64 with the
    # same SONAME as the system one the library links.  Loading torch first
    # makes the dynamic loader bind the library to torch's copy; the other
    # order would start a second runtime that torch can no longer use.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint32, ctypes.c_uint64)
    sig = {
        "lnbnn_build_index": ([P, ctypes.c_int, i64, i32, P, i32, u32, i64, u32, P,
                               ctypes.POINTER(P)], ctypes.c_int),
        "lnbnn_index_free": ([P], ctypes.c_int),
        "lnbnn_index_info": ([P, P, P, P, P], ctypes.c_int),
        "lnbnn_classify": ([P, P, ctypes.c_int, P, i32, i32, ctypes.c_int, u32, P, P, P, P, P],
                           ctypes.c_int),
        "lnbnn_last_timing": ([P, ctypes.POINTER(lnbnn_timing)], ctypes.c_int),
        "lnbnn_sync_status": ([P], ctypes.c_int),
        "lnbnn_classify_noalloc": ([P, P, ctypes.c_int, P, i32, i32, ctypes.c_int, P, P, P, P, P, P],
                                   ctypes.c_int),
        "lnbnn_autotune": ([P, P, ctypes.c_int, P, i32, i32, ctypes.c_int, ctypes.c_char_p, P, P],
                           ctypes.c_int),
        "lnbnn_set_variant": ([P, ctypes.c_int, i32, i32], ctypes.c_int),
        "lnbnn_set_tuning": ([P, ctypes.c_int, i32, ctypes.POINTER(lnbnn_tuning)], ctypes.c_int),
        "lnbnn_num_variants": ([], i32),
        "lnbnn_variant_name": ([i32], ctypes.c_char_p),
        "lnbnn_submit": ([P, P, ctypes.c_int, i64, i32, ctypes.c_int, ctypes.POINTER(u64)],
                         ctypes.c_int),
        "lnbnn_poll": ([P, u64, P, P, ctypes.POINTER(lnbnn_req_stats)], ctypes.c_int),
        "lnbnn_serve_config": ([P, i64, i32], ctypes.c_int),
        "lnbnn_serve_info": ([P, ctypes.POINTER(lnbnn_serve_stats)], ctypes.c_int),
        "lnbnn_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def lnbnn_last_error() -> str:
    return load().lnbnn_last_error().decode()


def _check(rc: int):
    if rc != LNBNN_OK:
        raise LnbnnError(rc, lnbnn_last_error())
    return rc


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if _is_torch(x):
        return ctypes.c_void_p(x.data_ptr())
    return x.ctypes.data_as(ctypes.c_void_p)


def _stream(x, stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    if x is not None and _is_torch(x) and x.is_cuda:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    return None


def _dtype_code(x) -> int:
    s = str(x.dtype)
    if s.endswith("uint8"):
        return LNBNN_U8
    if s.endswith("float32"):
        return LNBNN_F32
    raise TypeError(f"descriptors must be uint8 or float32, got {x.dtype}")


def _check_width(ix, queries):
    """Queries are read as [n, dim] rows of the index's width."""
    if len(queries.shape) != 2 or int(queries.shape[1]) != ix.dim:
        raise LnbnnError(LNBNN_EINVAL, f"queries must be [n, {ix.dim}], got {tuple(queries.shape)}")


class Index:
    """Owner of an lnbnn_index handle."""

    def __init__(self, handle, n_refs: int, n_classes: int, dtype: int, dim: int = LNBNN_DIM):
        self.handle = handle
        self.n_refs = n_refs
        self.n_classes = n_classes
        self.dtype = dtype
        self.dim = dim

    def free(self):
        if self.handle:
            _check(load().lnbnn_index_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                load().lnbnn_index_free(self.handle)
        except Exception:
            pass


def lnbnn_build_index(refs, labels, n_classes: int, mode_mask: int, hbm_budget_bytes: int = 0,
                      stream=None) -> Index:
    """Build the merged index (host numpy arrays or device torch tensors)."""
    dev = _is_torch(refs)
    if dev:
        assert refs.is_contiguous() and labels.is_contiguous()
        assert str(labels.dtype).endswith("int32")
    else:
        refs = np.ascontiguousarray(refs)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
    n_refs, dim = int(refs.shape[0]), int(refs.shape[1])
    out = ctypes.c_void_p()
    _check(load().lnbnn_build_index(_ptr(refs), _dtype_code(refs), n_refs, dim, _ptr(labels),
                                    int(n_classes), int(mode_mask), int(hbm_budget_bytes),
                                    LNBNN_DEVICE_PTRS if dev else 0, _stream(refs, stream),
                                    ctypes.byref(out)))
    return Index(out, n_refs, int(n_classes), _dtype_code(refs), dim)


def lnbnn_index_free(ix: Index):
    ix.free()


def lnbnn_index_info(ix: Index) -> dict:
    n_refs, nc = ctypes.c_int64(), ctypes.c_int32()
    mm, nb = ctypes.c_uint32(), ctypes.c_int64()
    _check(load().lnbnn_index_info(ix.handle, ctypes.byref(n_refs), ctypes.byref(nc),
                                   ctypes.byref(mm), ctypes.byref(nb)))
    return {"n_refs": n_refs.value, "n_classes": nc.value, "mode_mask": mm.value,
            "device_bytes": nb.value}


def lnbnn_classify(ix: Index, queries, img_offsets, k: int, mode: int, flags: int = 0,
                   want_totals: bool = True, want_neighbours: bool = False, stream=None, out=None):
    """Classify a batch of images.

    Returns (classes, totals or None, nbr_idx or None, nbr_dist or None).
    Host numpy queries give numpy outputs (blocking).  Torch device queries
    give torch device outputs, enqueued on torch's current stream (or
    `stream`); `out` may hold preallocated device outputs
    (keys "class", "totals", "nbr_idx", "nbr_dist").
    """
    offsets = np.ascontiguousarray(img_offsets, dtype=np.int64)
    n_img = offsets.shape[0] - 1
    n_q = int(offsets[-1]) if n_img >= 0 else 0
    kp = k + 1
    _check_width(ix, queries)
    float_totals = mode in FP8_MODES
    dev = _is_torch(queries)
    if dev:
        import torch
        flags |= LNBNN_DEVICE_PTRS
        d = queries.device
        out = out or {}
        cls = out.get("class")
        if cls is None:
            cls = torch.empty(max(n_img, 0), dtype=torch.int32, device=d)
        tot = out.get("totals")
        if tot is None and want_totals:
            tot = torch.empty((max(n_img, 0), ix.n_classes),
                              dtype=torch.float64 if float_totals else torch.int64, device=d)
        ni, nd = out.get("nbr_idx"), out.get("nbr_dist")
        if want_neighbours and ni is None:
            ni = torch.empty((n_q, kp), dtype=torch.int32, device=d)
            nd = torch.empty((n_q, kp), dtype=torch.float32, device=d)
    else:
        queries = np.ascontiguousarray(queries)
        cls = np.empty(max(n_img, 0), np.int32)
        tot = (np.empty((max(n_img, 0), ix.n_classes), np.float64 if float_totals else np.int64)
               if want_totals else None)
        ni = np.empty((n_q, kp), np.int32) if want_neighbours else None
        nd = np.empty((n_q, kp), np.float32) if want_neighbours else None
    _check(load().lnbnn_classify(ix.handle, _ptr(queries), _dtype_code(queries), _ptr(offsets),
                                 n_img, int(k), int(mode), int(flags), _ptr(cls), _ptr(tot),
                                 _ptr(ni), _ptr(nd), _stream(queries, stream)))
    return cls, tot, ni, nd


def lnbnn_sync_status(ix: Index):
    """Wait for the index's classify calls; raises LnbnnError(EDEVICE) if a
    bounded stage wait gave up since the last report."""
    _check(load().lnbnn_sync_status(ix.handle))


def lnbnn_classify_noalloc(ix: Index, queries_dev, img_offsets, k: int, mode: int, out: dict,
                           stream=None):
    """The allocation-free classify: device tensors only, outputs in `out`
    (keys "class" required; "totals", "nbr_idx", "nbr_dist", "status"
    optional), enqueued on torch's current stream (or `stream`)."""
    offsets = np.ascontiguousarray(img_offsets, dtype=np.int64)
    _check_width(ix, queries_dev)
    _check(load().lnbnn_classify_noalloc(
        ix.handle, _ptr(queries_dev), _dtype_code(queries_dev), _ptr(offsets), offsets.shape[0] - 1,
        int(k), int(mode), _ptr(out["class"]), _ptr(out.get("totals")), _ptr(out.get("nbr_idx")),
        _ptr(out.get("nbr_dist")), _ptr(out.get("status")), _stream(queries_dev, stream)))
    return out


def lnbnn_last_timing(ix: Index) -> dict:
    t = lnbnn_timing()
    _check(load().lnbnn_last_timing(ix.handle, ctypes.byref(t)))
    return {"dist_kernel_ms": t.dist_kernel_ms, "total_ms": t.total_ms,
            "dist_launches": t.dist_launches, "slices": t.slices, "tile_variant": t.tile_variant}


def lnbnn_autotune(ix: Index, queries_dev, img_offsets, k: int, mode: int,
                   cache_path: str | None = None, stream=None) -> int:
    offsets = np.ascontiguousarray(img_offsets, dtype=np.int64)
    _check_width(ix, queries_dev)
    best = ctypes.c_int32(-1)
    _check(load().lnbnn_autotune(ix.handle, _ptr(queries_dev), _dtype_code(queries_dev),
                                 _ptr(offsets), offsets.shape[0] - 1, int(k), int(mode),
                                 cache_path.encode() if cache_path else None, ctypes.byref(best),
                                 _stream(queries_dev, stream)))
    return best.value


def lnbnn_set_variant(ix: Index, mode: int, k: int, variant: int):
    _check(load().lnbnn_set_variant(ix.handle, int(mode), int(k), int(variant)))


def lnbnn_set_tuning(ix: Index, mode: int, k: int, variant: int = -1, chunk_tiles: int = 0,
                     max_workgroups: int = 0):
    t = lnbnn_tuning(int(variant), int(chunk_tiles), int(max_workgroups))
    _check(load().lnbnn_set_tuning(ix.handle, int(mode), int(k), ctypes.byref(t)))


def lnbnn_num_variants() -> int:
    return int(load().lnbnn_num_variants())


def lnbnn_variant_name(v: int) -> str:
    return load().lnbnn_variant_name(int(v)).decode()


def lnbnn_serve_config(ix: Index, max_batch_desc: int = 0, max_inflight: int = 0):
    _check(load().lnbnn_serve_config(ix.handle, int(max_batch_desc), int(max_inflight)))


def lnbnn_serve_info(ix: Index) -> dict:
    st = lnbnn_serve_stats()
    _check(load().lnbnn_serve_info(ix.handle, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in lnbnn_serve_stats._fields_}


def lnbnn_submit(ix: Index, queries, k: int, mode: int) -> int:
    queries = np.ascontiguousarray(queries)
    _check_width(ix, queries)
    t = ctypes.c_uint64()
    _check(load().lnbnn_submit(ix.handle, _ptr(queries), _dtype_code(queries),
                               int(queries.shape[0]), int(k), int(mode), ctypes.byref(t)))
    return t.value


def lnbnn_poll(ix: Index, ticket: int, want_totals: bool = True):
    """None while pending, else (class, totals or None, stats dict)."""
    cls = np.empty(1, np.int32)
    tot = None
    if want_totals:
        tot = np.empty(ix.n_classes, np.float64 if ix.dtype == LNBNN_F32 else np.int64)
    st = lnbnn_req_stats()
    rc = load().lnbnn_poll(ix.handle, ctypes.c_uint64(ticket), _ptr(cls), _ptr(tot), ctypes.byref(st))
    if rc == LNBNN_EAGAIN:
        return None
    _check(rc)
    stats = {f: getattr(st, f) for f, _ in lnbnn_req_stats._fields_}
    return int(cls[0]), tot, stats
