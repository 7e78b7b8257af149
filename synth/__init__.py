"""Seeded synthetic descriptor sets shaped like the paper's workloads.

Input data only: this module holds none of local NBNN's arithmetic and is
shared by the oracle-side tests and by the GPU-side tests and benchmark.

The paper classifies Caltech 101 / Caltech 256 images from dense SIFT
(Sec. 6; 15 or 30 training images per class).  Neither the datasets nor a
feature extractor is available here, so these sets stand in for them: they
keep the number of classes, training images per class and a descriptor count
per image, and they put clustered structure into 128-d descriptors so that
neighbour searches behave like searches among real local features (each class
owns a few prototype means, and a shared pool of background means stands in
for features common to all classes).

Recipe (every config):
  * world: class prototype means and background means, drawn first from the
    index seed (spawn key 0);
  * reference j belongs to class j // (n_train * n_desc) -- classes occupy
    contiguous index ranges, images are contiguous within a class;
  * each descriptor, independently: with probability f_bg its mean is a
    uniformly chosen background mean, otherwise a uniformly chosen prototype
    of its class;
  * u8 configs: x = clip(rint(mean + N(0, sigma^2 I)), 0, 255) as uint8, means
    uniform in [0, 255]^128;
  * float configs: means are normalize(relu(g)), g ~ N(0, I); descriptors are
    normalize(relu(mean + N(0, sigma^2 I))) in float32 (an all-zero vector is
    redrawn);
  * query image m has true class m mod n_classes; its descriptor count is fixed
    or uniform in [lo, hi] (inclusive), drawn from the query seed;
  * generation is chunked (65536 descriptors per chunk, each chunk its own
    PCG64 stream from SeedSequence(seed, spawn_key=(1, chunk))) so results do
    not depend on the thread count.

Location-augmented u8 sets (the paper weights a descriptor's image location
by alpha = 1.6, Sec. 6; the augmented form is Boiman et al.'s):
  * every class prototype has a location centre in [0.15, 0.85]^2 (index
    seed, spawn key 2); a prototype descriptor lies at its centre plus
    N(0, 0.08^2) per coordinate, clipped to [0, 1]; a background descriptor
    anywhere in the unit square (own stream per chunk, spawn key (3, chunk),
    so the 128 descriptor bytes equal the plain generator's);
  * a row is 160 bytes: the descriptor, then 16 copies of the x code, then
    16 of the y code, code = rint(204.8 * coordinate) in 0..205.  u8 SIFT is
    512 times the unit-norm descriptor, so alpha at that scale is 819.2, and
    16 copies of 819.2 / 4 make 16 * dcode^2 = (819.2 * dcoord)^2 up to
    rounding while every byte stays an exact u8.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, replace

import numpy as np

DIM = 128
CHUNK = 65536
ALPHA = 1.6                  # location weight (Sec. 6)
LOC_COPIES = 16              # copies of each coordinate code
LOC_SCALE = 512.0            # u8 SIFT units per unit-norm descriptor unit
DIM_LOC = DIM + 2 * LOC_COPIES
LOC_SPREAD = 0.08


@dataclass(frozen=True)
class Config:
    name: str
    n_classes: int
    n_train: int          # training images per class
    n_desc: int           # descriptors per training image
    n_proto: int          # prototype means per class
    n_bg: int             # shared background means
    f_bg: float           # probability that a descriptor is background
    sigma: float          # per-dimension noise
    n_img: int            # query images
    q_lo: int             # query descriptors per image, lower bound
    q_hi: int             # ... upper bound (inclusive)
    k: int                # default neighbourhood size
    kind: str             # "u8" or "f32"
    index_seed: int
    query_seed: int

    @property
    def n_refs(self) -> int:
        return self.n_classes * self.n_train * self.n_desc


CONFIGS = {
    # tiny parity case: 10 classes x 5 images x 200 descriptors
    "T": Config("T", 10, 5, 200, 8, 16, 0.30, 20.0, 20, 200, 200, 10, "u8", 1000, 2000),
    # Caltech-101-like, 15 training images: 101 x 15 x 1500
    "M": Config("M", 101, 15, 1500, 12, 16, 0.25, 20.0, 1000, 1500, 1500, 10, "u8", 1001, 2001),
    # Caltech-256-like, 30 training images: 256 x 30 x 2000 = 15.36M refs,
    # 512 query images of 500..4000 descriptors
    "L": Config("L", 256, 30, 2000, 12, 16, 0.25, 20.0, 512, 500, 4000, 10, "u8", 1002, 2002),
    # float descriptors with L's structure (FP8 candidate pass + FP32 rerank)
    "P": Config("P", 256, 30, 2000, 12, 16, 0.25, 0.08, 512, 500, 4000, 10, "f32", 1003, 2003),
}


def scaled(cfg: Config, **kw) -> Config:
    """A copy of a config with some sizes changed (tests use this for small
    cases with the same recipe)."""
    return replace(cfg, **kw)


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=key)))


def _unit_relu(x: np.ndarray, rng: np.random.Generator, redraw) -> np.ndarray:
    np.maximum(x, 0, out=x)
    nrm = np.sqrt(np.einsum("ij,ij->i", x, x))
    zero = nrm == 0
    while zero.any():
        x[zero] = np.maximum(redraw(int(zero.sum())), 0)
        nrm = np.sqrt(np.einsum("ij,ij->i", x, x))
        zero = nrm == 0
    x /= nrm[:, None]
    return x


def world(cfg: Config):
    """(prototype means [n_classes, n_proto, DIM], background means [n_bg, DIM])
    as float32."""
    rng = _rng(cfg.index_seed, 0)
    if cfg.kind == "u8":
        protos = rng.uniform(0.0, 255.0, size=(cfg.n_classes, cfg.n_proto, DIM))
        bg = rng.uniform(0.0, 255.0, size=(cfg.n_bg, DIM))
        return protos.astype(np.float32), bg.astype(np.float32)
    g = rng.standard_normal(size=(cfg.n_classes * cfg.n_proto, DIM)).astype(np.float32)
    protos = _unit_relu(g, rng, lambda m: rng.standard_normal((m, DIM)).astype(np.float32))
    b = rng.standard_normal(size=(cfg.n_bg, DIM)).astype(np.float32)
    bg = _unit_relu(b, rng, lambda m: rng.standard_normal((m, DIM)).astype(np.float32))
    return protos.reshape(cfg.n_classes, cfg.n_proto, DIM), bg


def loc_centres(cfg: Config) -> np.ndarray:
    """Location centre of every class prototype: [n_classes, n_proto, 2]."""
    rng = _rng(cfg.index_seed, 2)
    return rng.uniform(0.15, 0.85, size=(cfg.n_classes, cfg.n_proto, 2))


def loc_code(xy: np.ndarray) -> np.ndarray:
    """Coordinates in [0, 1] -> u8 codes rint(alpha * 512 / 4 * x)."""
    return np.rint(np.asarray(xy, np.float64) * (ALPHA * LOC_SCALE / np.sqrt(LOC_COPIES))).astype(np.uint8)


def augment(desc: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """[n, 128] u8 descriptors and [n, 2] coordinates -> [n, 160] u8 rows."""
    n = desc.shape[0]
    out = np.empty((n, DIM_LOC), np.uint8)
    out[:, :DIM] = desc
    c = loc_code(xy)
    out[:, DIM:DIM + LOC_COPIES] = c[:, 0:1]
    out[:, DIM + LOC_COPIES:] = c[:, 1:2]
    return out


def _locations(cfg: Config, centres, is_bg, cls, pick_pr, seed: int, chunk: int) -> np.ndarray:
    rng = _rng(seed, 3, chunk)
    m = cls.shape[0]
    near = centres[cls, pick_pr] + LOC_SPREAD * rng.standard_normal((m, 2))
    anywhere = rng.random((m, 2))
    return np.clip(np.where(is_bg[:, None], anywhere, near), 0.0, 1.0)


def _descriptors(cfg: Config, protos, bg, cls: np.ndarray, seed: int, chunk: int, out, centres=None):
    """Fill out[chunk rows] for descriptors whose class is cls (one chunk);
    with location centres given, out has DIM_LOC columns."""
    rng = _rng(seed, 1, chunk)
    m = cls.shape[0]
    is_bg = rng.random(m) < cfg.f_bg
    pick_bg = rng.integers(0, cfg.n_bg, size=m)
    pick_pr = rng.integers(0, cfg.n_proto, size=m)
    if centres is not None:
        desc = np.empty((m, DIM), np.uint8)
        _descriptors(cfg, protos, bg, cls, seed, chunk, desc)
        out[:] = augment(desc, _locations(cfg, centres, is_bg, cls, pick_pr, seed, chunk))
        return
    means = np.where(is_bg[:, None], bg[pick_bg], protos[cls, pick_pr])
    z = rng.standard_normal(size=(m, DIM), dtype=np.float32)
    x = means.astype(np.float32, copy=False)
    x = x + np.float32(cfg.sigma) * z
    if cfg.kind == "u8":
        np.rint(x, out=x)
        np.clip(x, 0.0, 255.0, out=x)
        out[:] = x.astype(np.uint8)
    else:
        out[:] = _unit_relu(x, rng, lambda k: rng.standard_normal((k, DIM), dtype=np.float32))


def _fill(cfg: Config, cls: np.ndarray, seed: int, loc: bool = False) -> np.ndarray:
    protos, bg = world(cfg)
    centres = loc_centres(cfg) if loc else None
    assert not loc or cfg.kind == "u8"
    n = cls.shape[0]
    out = np.empty((n, DIM_LOC if loc else DIM), np.uint8 if cfg.kind == "u8" else np.float32)
    nch = (n + CHUNK - 1) // CHUNK

    def job(c):
        s = c * CHUNK
        e = min(n, s + CHUNK)
        _descriptors(cfg, protos, bg, cls[s:e], seed, c, out[s:e], centres)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(job, range(nch)))
    return out


def index_labels(cfg: Config) -> np.ndarray:
    """Class of every reference descriptor (int32 [n_refs])."""
    per_class = cfg.n_train * cfg.n_desc
    return np.repeat(np.arange(cfg.n_classes, dtype=np.int32), per_class)


def gen_index(cfg: Config, loc: bool = False):
    """(refs [n_refs, DIM] uint8 or float32, labels int32 [n_refs]); with
    loc, u8 rows of DIM_LOC bytes (location-augmented)."""
    labels = index_labels(cfg)
    return _fill(cfg, labels, cfg.index_seed, loc), labels


def query_layout(cfg: Config):
    """(CSR offsets int64 [n_img + 1], true class int32 [n_img])."""
    rng = _rng(cfg.query_seed, 0)
    if cfg.q_lo == cfg.q_hi:
        counts = np.full(cfg.n_img, cfg.q_lo, np.int64)
    else:
        counts = rng.integers(cfg.q_lo, cfg.q_hi + 1, size=cfg.n_img).astype(np.int64)
    offsets = np.zeros(cfg.n_img + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    true_cls = (np.arange(cfg.n_img) % cfg.n_classes).astype(np.int32)
    return offsets, true_cls


def gen_queries(cfg: Config, loc: bool = False):
    """(queries [n, DIM] (DIM_LOC with loc), CSR offsets int64 [n_img + 1],
    true class [n_img])."""
    offsets, true_cls = query_layout(cfg)
    per_desc = np.repeat(true_cls, np.diff(offsets))
    return _fill(cfg, per_desc, cfg.query_seed, loc), offsets, true_cls


def gen_query_images(cfg: Config, images):
    """Only the listed query images, identical to the same images of
    gen_queries (used for sampled checks): ([n_sel, DIM], offsets [len+1])."""
    offsets, true_cls = query_layout(cfg)
    images = list(images)
    # regenerate only the chunks the images touch
    protos, bg = world(cfg)
    per_desc_cls = np.repeat(true_cls, np.diff(offsets))
    parts = []
    for m in images:
        s, e = int(offsets[m]), int(offsets[m + 1])
        rows = np.empty((e - s, DIM), np.uint8 if cfg.kind == "u8" else np.float32)
        c0, c1 = s // CHUNK, (e - 1) // CHUNK if e > s else s // CHUNK
        for c in range(c0, c1 + 1):
            cs = c * CHUNK
            ce = min(int(offsets[-1]), cs + CHUNK)
            buf = np.empty((ce - cs, DIM), rows.dtype)
            _descriptors(cfg, protos, bg, per_desc_cls[cs:ce], cfg.query_seed, c, buf)
            a, b = max(s, cs), min(e, ce)
            if a < b:
                rows[a - s:b - s] = buf[a - cs:b - cs]
        parts.append(rows)
    sub_off = np.zeros(len(images) + 1, np.int64)
    np.cumsum([p.shape[0] for p in parts], out=sub_off[1:])
    return (np.concatenate(parts) if parts else np.empty((0, DIM), np.uint8)), sub_off


def request_stream(n_req: int, rate_per_s: float, seed: int = 3000,
                   median: float = 1500.0, sigma: float = 0.6, lo: int = 100, hi: int = 8000):
    """Serving trace: Poisson arrival times (s) and per-request descriptor
    counts ~ clip(round(LogNormal(ln median, sigma)), lo, hi)."""
    rng = _rng(seed, 0)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    n = np.clip(np.rint(rng.lognormal(np.log(median), sigma, size=n_req)), lo, hi).astype(np.int64)
    return t, n


def gen_requests(cfg: Config, counts, seed: int = 3001):
    """Descriptors of a request stream: request r is an image of class
    r mod n_classes with counts[r] descriptors; returns ([sum counts, DIM],
    offsets)."""
    counts = np.asarray(counts, np.int64)
    offsets = np.zeros(counts.shape[0] + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    cls = (np.arange(counts.shape[0]) % cfg.n_classes).astype(np.int32)
    per_desc = np.repeat(cls, counts)
    return _fill(cfg, per_desc, seed), offsets
