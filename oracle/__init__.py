"""Local NBNN oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU statement of local NBNN (McCann & Lowe, Sec. 5, Algorithm 2) and
of the original NBNN rule (Sec. 1, Algorithm 1; Sec. 3, the NBNN rule as an
argmin of summed squared distances).  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library; both consume the same generated arrays.

Two kinds of routes:

* the C library ``liblnbnn_oracle.so`` (built from ``lnbnn_oracle.c``):
  direct-form distances in int64 (u8) or double (f32), k+1 nearest by a full
  sort, by a single insertion scan, or by the same scan tiled for the cache
  (route "block", used for whole-image checks at full index size),
  Algorithm 2 as printed, Algorithm 1, and the closed form of Algorithm 2's
  totals;
* ``knn_expanded``: a numpy route for larger sampled checks.  It evaluates
  ||q||^2 + ||r||^2 - 2 q.r with a float64 matrix product, which is exact
  for u8 descriptors (every partial sum is an integer below 2^53), and
  selects by a composite (distance, index) key.  For float descriptors it
  uses the expanded form only to shortlist candidates and re-evaluates them
  in direct form.

Readings of points the paper leaves open (the same list is kept with the
design notes): squared L2 without a root; neighbour ties go to the lower
reference index; argmin ties go to the lower class; all classes start at 0.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lnbnn_oracle.c")
# LNBNN_ORACLE_LIB: load another build of the same source (the sanitizer
# build of the tests)
_LIB = os.environ.get("LNBNN_ORACLE_LIB") or os.path.join(_HERE, "liblnbnn_oracle.so")

_lib = None


def build(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP; ISO C, so no multiply-add
    contraction: every double operation is rounded as written).  The blocked
    route is compiled for several x86 vector widths and picked at load time;
    the arithmetic is the same IEEE operations on every width.

    sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build (any
    report aborts) into `out`; the process that loads it must preload gcc's
    libasan."""
    lib = out or _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        opt = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"] if sanitize else ["-O3"])
        cmd = ["gcc", *opt, "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared",
               "-fPIC", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    sigs = {
        "or_sqdist_u8": ([P, P, i32], ctypes.c_int64),
        "or_sqdist_u8_expanded": ([P, P, i32], ctypes.c_int64),
        "or_sqdist_f32": ([P, P, i32], ctypes.c_double),
        "or_knn_u8_sort": ([P, i64, P, i64, i32, i32, P, P], ctypes.c_int),
        "or_knn_u8_scan": ([P, i64, P, i64, i32, i32, P, P], ctypes.c_int),
        "or_knn_f32_sort": ([P, i64, P, i64, i32, i32, P, P], ctypes.c_int),
        "or_knn_f32_scan": ([P, i64, P, i64, i32, i32, P, P], ctypes.c_int),
        "or_knn_u8_block": ([P, i64, P, i64, i32, i32, P, i32, P, P, P], ctypes.c_int),
        "or_knn_f32_block": ([P, i64, P, i64, i32, i32, P, P], ctypes.c_int),
        "or_local_nbnn_i64": ([P, P, i64, i32, P, i32, P, i32, P, P], ctypes.c_int),
        "or_local_nbnn_f64": ([P, P, i64, i32, P, i32, P, i32, P, P], ctypes.c_int),
        "or_class_nn_u8": ([P, i64, P, i64, i32, P, i32, i32, P, P], ctypes.c_int),
        "or_closed_form_i64": ([P, P, i64, i32, P, i32, P, P], ctypes.c_int),
        "or_nbnn_i64": ([P, i64, i32, P, i32, P, P], ctypes.c_int),
        "or_num_threads": ([], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(_load().or_num_threads())


# ---------------------------------------------------------------- distances
def sqdist_u8(a, b) -> int:
    a, b = _c(a, np.uint8), _c(b, np.uint8)
    assert a.shape == b.shape and a.ndim == 1
    return int(_load().or_sqdist_u8(_p(a), _p(b), a.shape[0]))


def sqdist_u8_expanded(a, b) -> int:
    a, b = _c(a, np.uint8), _c(b, np.uint8)
    assert a.shape == b.shape and a.ndim == 1
    return int(_load().or_sqdist_u8_expanded(_p(a), _p(b), a.shape[0]))


def sqdist_f32(a, b) -> float:
    a, b = _c(a, np.float32), _c(b, np.float32)
    assert a.shape == b.shape and a.ndim == 1
    return float(_load().or_sqdist_f32(_p(a), _p(b), a.shape[0]))


# ------------------------------------------------- NN(d_i, k+1), Algorithm 2
def knn(Q, R, kp: int, route: str = "scan"):
    """k+1 nearest references of every query in (distance, index) order.

    Returns (idx int32 [n, kp], dist [n, kp]) with int64 distances for u8
    inputs and float64 distances for float32 inputs.
    """
    lib = _load()
    is_u8 = np.asarray(Q).dtype == np.uint8
    dt = np.uint8 if is_u8 else np.float32
    Q, R = _c(Q, dt), _c(R, dt)
    n, dim = Q.shape
    N = R.shape[0]
    assert R.shape[1] == dim
    idx = np.empty((n, kp), np.int32)
    dist = np.empty((n, kp), np.int64 if is_u8 else np.float64)
    if route == "block":
        if is_u8:
            rc = lib.or_knn_u8_block(_p(Q), n, _p(R), N, dim, kp, None, 0,
                                     _p(idx), _p(dist), None)
        else:
            rc = lib.or_knn_f32_block(_p(Q), n, _p(R), N, dim, kp, _p(idx), _p(dist))
        if rc != 0:
            raise ValueError("oracle knn failed (kp > N or out of memory)")
        return idx, dist
    fn = {("u8", "sort"): lib.or_knn_u8_sort, ("u8", "scan"): lib.or_knn_u8_scan,
          ("f32", "sort"): lib.or_knn_f32_sort, ("f32", "scan"): lib.or_knn_f32_scan}[
        ("u8" if is_u8 else "f32", route)]
    rc = fn(_p(Q), n, _p(R), N, dim, kp, _p(idx), _p(dist))
    if rc != 0:
        raise ValueError("oracle knn failed (kp > N or out of memory)")
    return idx, dist


def knn_expanded(Q, R, kp: int, chunk: int = 1 << 20, margin: int = 8):
    """Numpy route for sampled checks at full index size.

    u8: distance = ||q||^2 + ||r||^2 - 2 q.r in float64, exact for u8 data
    (all products and sums are integers < 2^53).  Selection uses the exact
    composite key distance * 2^24 + index (< 2^53 for distances < 2^29 and
    fewer than 2^24 references), whose order is the (distance, index) order.
    float32: the expanded form shortlists kp + margin candidates per chunk;
    the shortlist is re-evaluated in direct form (double) and ordered by
    (distance, index).
    """
    is_u8 = np.asarray(Q).dtype == np.uint8
    Q = np.ascontiguousarray(Q)
    n, dim = Q.shape
    N = R.shape[0]
    if kp < 1 or kp > N:
        raise ValueError("kp must be in [1, N]")
    Qd = Q.astype(np.float64)
    qq = np.einsum("ij,ij->i", Qd, Qd)
    if is_u8:
        assert N < (1 << 24) and dim * 255 * 255 < (1 << 29)
        best_key = np.full((n, 0), np.inf)
        for s in range(0, N, chunk):
            Rc = R[s:s + chunk].astype(np.float64)
            rr = np.einsum("ij,ij->i", Rc, Rc)
            d = qq[:, None] + rr[None, :] - 2.0 * (Qd @ Rc.T)
            key = d * float(1 << 24) + (np.arange(s, s + Rc.shape[0], dtype=np.float64))[None, :]
            take = min(kp, key.shape[1])
            part = np.partition(key, take - 1, axis=1)[:, :take]
            best_key = np.concatenate([best_key, part], axis=1)
            take = min(kp, best_key.shape[1])
            best_key = np.partition(best_key, take - 1, axis=1)[:, :take]
        best_key = np.sort(best_key, axis=1)
        dist = np.floor(best_key / float(1 << 24))
        idx = best_key - dist * float(1 << 24)
        return idx.astype(np.int32), dist.astype(np.int64)
    # float descriptors
    cand_idx = np.zeros((n, 0), np.int64)
    for s in range(0, N, chunk):
        Rc = R[s:s + chunk].astype(np.float64)
        rr = np.einsum("ij,ij->i", Rc, Rc)
        d = qq[:, None] + rr[None, :] - 2.0 * (Qd @ Rc.T)
        take = min(kp + margin, d.shape[1])
        part = np.argpartition(d, take - 1, axis=1)[:, :take] + s
        cand_idx = np.concatenate([cand_idx, part], axis=1)
        # shortlist by direct form, keeping kp + margin per row
        dd = _direct_rows(Q, R, cand_idx)
        take = min(kp + margin, cand_idx.shape[1])
        order = np.lexsort((cand_idx, dd), axis=1)[:, :take]
        cand_idx = np.take_along_axis(cand_idx, order, axis=1)
    dd = _direct_rows(Q, R, cand_idx)
    order = np.lexsort((cand_idx, dd), axis=1)[:, :kp]
    idx = np.take_along_axis(cand_idx, order, axis=1)
    dist = np.take_along_axis(dd, order, axis=1)
    return idx.astype(np.int32), dist


def _direct_rows(Q, R, cand_idx):
    """Direct-form double distances from each query to its candidate rows."""
    Qd = Q.astype(np.float64)
    out = np.empty(cand_idx.shape, np.float64)
    for i in range(Q.shape[0]):
        diff = R[cand_idx[i]].astype(np.float64) - Qd[i][None, :]
        out[i] = np.sum(diff * diff, axis=1)
    return out


# ------------------------------------------------------ Algorithm 2 scoring
def local_nbnn(nbr_idx, nbr_dist, k: int, labels, n_classes: int, offsets):
    """Algorithm 2 totals and per-image argmin from k+1 neighbour lists."""
    lib = _load()
    nbr_idx = _c(nbr_idx, np.int32)
    is_int = np.asarray(nbr_dist).dtype.kind in "iu"
    nbr_dist = _c(nbr_dist, np.int64 if is_int else np.float64)
    labels = _c(labels, np.int32)
    offsets = _c(offsets, np.int64)
    n = nbr_idx.shape[0]
    assert nbr_idx.shape == (n, k + 1) and nbr_dist.shape == (n, k + 1)
    n_img = offsets.shape[0] - 1
    totals = np.empty((n_img, n_classes), np.int64 if is_int else np.float64)
    cls = np.empty(n_img, np.int32)
    fn = lib.or_local_nbnn_i64 if is_int else lib.or_local_nbnn_f64
    rc = fn(_p(nbr_idx), _p(nbr_dist), n, k, _p(labels), n_classes, _p(offsets),
            n_img, _p(totals), _p(cls))
    if rc != 0:
        raise ValueError("invalid arguments to local_nbnn")
    return totals, cls


def class_nn(Q, R, labels, n_classes: int, k: int):
    """Per-class nearest distance D[i, C] (Algorithm 1's ||d - NN_C(d)||^2;
    INT64_MAX for an empty class) and the (k+1)-th smallest distance."""
    lib = _load()
    Q, R = _c(Q, np.uint8), _c(R, np.uint8)
    labels = _c(labels, np.int32)
    n, dim = Q.shape
    D = np.empty((n, n_classes), np.int64)
    kth = np.empty(n, np.int64)
    rc = lib.or_class_nn_u8(_p(Q), n, _p(R), R.shape[0], dim, _p(labels), n_classes,
                            k, _p(D), _p(kth))
    if rc != 0:
        raise ValueError("invalid arguments to class_nn")
    return D, kth


def knn_class_block(Q, R, labels, n_classes: int, kp: int):
    """u8 descriptors, one blocked pass: the kp nearest (distance, index)
    pairs of every query (as ``knn``) and the per-class nearest distance
    D[i, C] (as ``class_nn``; INT64_MAX for an empty class).  The (k+1)-th
    smallest distance that ``class_nn`` returns is ``dist[:, kp - 1]``."""
    lib = _load()
    Q, R = _c(Q, np.uint8), _c(R, np.uint8)
    labels = _c(labels, np.int32)
    n, dim = Q.shape
    idx = np.empty((n, kp), np.int32)
    dist = np.empty((n, kp), np.int64)
    D = np.empty((n, n_classes), np.int64)
    rc = lib.or_knn_u8_block(_p(Q), n, _p(R), R.shape[0], dim, kp, _p(labels), n_classes,
                             _p(idx), _p(dist), _p(D))
    if rc != 0:
        raise ValueError("invalid arguments to knn_class_block")
    return idx, dist, D


def closed_form(D, kth, offsets):
    """Algorithm 2 totals via sum of min(0, D_C(d) - delta_(k+1)(d))."""
    lib = _load()
    D, kth, offsets = _c(D, np.int64), _c(kth, np.int64), _c(offsets, np.int64)
    n, nc = D.shape
    n_img = offsets.shape[0] - 1
    totals = np.empty((n_img, nc), np.int64)
    cls = np.empty(n_img, np.int32)
    rc = lib.or_closed_form_i64(_p(D), _p(kth), n, nc, _p(offsets), n_img,
                                _p(totals), _p(cls))
    if rc != 0:
        raise ValueError("invalid arguments to closed_form")
    return totals, cls


def nbnn(D, offsets):
    """Algorithm 1 (original NBNN) totals and argmin from per-class NN."""
    lib = _load()
    D, offsets = _c(D, np.int64), _c(offsets, np.int64)
    n, nc = D.shape
    n_img = offsets.shape[0] - 1
    totals = np.empty((n_img, nc), np.int64)
    cls = np.empty(n_img, np.int32)
    rc = lib.or_nbnn_i64(_p(D), n, nc, _p(offsets), n_img, _p(totals), _p(cls))
    if rc != 0:
        raise ValueError("invalid arguments to nbnn (empty class?)")
    return totals, cls


def classify(Q, R, labels, n_classes: int, offsets, k: int, route: str = "scan"):
    """Whole local NBNN (Algorithm 2) for a batch of images: k+1 nearest by
    brute force, then the per-class update and argmin."""
    idx, dist = knn(Q, R, k + 1, route=route)
    totals, cls = local_nbnn(idx, dist, k, labels, n_classes, offsets)
    return totals, cls, idx, dist
