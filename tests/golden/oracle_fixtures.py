"""Stored oracle results for whole query images at full index size.

Test infrastructure.  The full-size parity tests compare the GPU library with
these arrays; every value in them comes from ``oracle/`` (the blocked route
of the C oracle, then Algorithm 2's scoring and Algorithm 1's totals) on
inputs from ``synth/``.  Nothing here, and nothing the fixtures hold, comes
from the GPU path.

Fixtures (written by ``python tests/golden/oracle_fixtures.py NAME``; hours of
CPU for the float one):

* ``M``: the 101-class, 2.27M-reference u8 set; query images 0, 10, ..., 990
  (100 whole images, 150,000 descriptors); lists of k+1 = 11, so k = 1, 5
  and 10 are prefixes of one run.
* ``L``: the 256-class, 15.36M-reference u8 set; query images 0, 32, ..., 480
  (16 whole images); lists of 21, so k = 5, 10 and 20.
* ``P``: the float set with L's structure; query images 0, 8, ..., 504 (64
  whole images, spread over the 500..4000 descriptor range); lists of 11
  (k = 10), double distances.

Stored per fixture: the images; their CSR offsets within the subset; per k
the int64 (u8) or double (float) totals of Algorithm 2 and the per-image
argmin; a digest of each image's neighbour lists (u8); the lists of every
STRIDE-th descriptor (u8) or of every descriptor (float, indices only, plus
the distances of every STRIDE-th); for the u8 sets, Algorithm 1's totals and
argmin (the original NBNN rule).  The script checks on the way that literal
Algorithm 2 on the lists equals the closed form from the per-class nearest
distances.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

STRIDE = 8          # every STRIDE-th descriptor keeps its whole list

SPECS = {
    "M": dict(cfg="M", images=tuple(range(0, 1000, 10)), kp=11, ks=(1, 5, 10)),
    "L": dict(cfg="L", images=tuple(range(0, 512, 32)), kp=21, ks=(5, 10, 20)),
    "P": dict(cfg="P", images=tuple(range(0, 512, 8)), kp=11, ks=(10,)),
}


def path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def list_digest(idx: np.ndarray, dist: np.ndarray) -> bytes:
    """16-byte digest of neighbour lists: indices as int32, distances as
    int64, both C-contiguous [rows, kp]."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(idx, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(dist, dtype=np.int64).tobytes())
    return h.digest()[:16]


def load(name: str):
    """The stored arrays of a fixture (no pickled objects), or None if the
    fixture has not been written."""
    p = path(name)
    if not os.path.exists(p):
        return None
    with np.load(p, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _compute(name: str, scratch: str, chunk_images: int) -> dict:
    sys.path.insert(0, ROOT)
    import oracle
    import synth

    spec = SPECS[name]
    cfg = synth.CONFIGS[spec["cfg"]]
    images = list(spec["images"])
    kp = spec["kp"]
    t0 = time.time()
    R, labels = synth.gen_index(cfg)
    Q, sub_off = synth.gen_query_images(cfg, images)
    print(f"[{name}] inputs: {R.shape[0]} refs, {len(images)} images, {Q.shape[0]} "
          f"descriptors ({time.time() - t0:.0f} s); oracle threads {oracle.num_threads()}",
          flush=True)
    is_u8 = cfg.kind == "u8"
    os.makedirs(scratch, exist_ok=True)
    parts_idx, parts_dist, parts_D = [], [], []
    for c0 in range(0, len(images), chunk_images):
        c1 = min(len(images), c0 + chunk_images)
        s, e = int(sub_off[c0]), int(sub_off[c1])
        part = os.path.join(scratch, f"{name}_{c0}_{c1}.npz")
        if os.path.exists(part):
            with np.load(part, allow_pickle=False) as z:
                idx, dist = z["idx"], z["dist"]
                D = z["D"] if is_u8 else None
        else:
            t1 = time.time()
            if is_u8:
                idx, dist, D = oracle.knn_class_block(Q[s:e], R, labels, cfg.n_classes, kp)
                np.savez(part + ".tmp.npz", idx=idx, dist=dist, D=D)
            else:
                idx, dist = oracle.knn(Q[s:e], R, kp, route="block")
                D = None
                np.savez(part + ".tmp.npz", idx=idx, dist=dist)
            os.replace(part + ".tmp.npz", part)
            print(f"[{name}] images {c0}..{c1 - 1}: {e - s} descriptors in "
                  f"{time.time() - t1:.0f} s", flush=True)
        parts_idx.append(idx)
        parts_dist.append(dist)
        if is_u8:
            parts_D.append(D)
    idx = np.concatenate(parts_idx)
    dist = np.concatenate(parts_dist)
    out = {
        "images": np.asarray(images, np.int32),
        "offsets": sub_off.astype(np.int64),
        "kp": np.int32(kp),
        "ks": np.asarray(spec["ks"], np.int32),
        "n_refs": np.int64(R.shape[0]),
        "n_classes": np.int32(cfg.n_classes),
    }
    n_img = len(images)
    for k in spec["ks"]:
        tot, cls = oracle.local_nbnn(idx[:, :k + 1], dist[:, :k + 1], k, labels,
                                     cfg.n_classes, sub_off)
        out[f"totals_k{k}"] = tot
        out[f"classes_k{k}"] = cls
        if is_u8:
            D = np.concatenate(parts_D)
            ct, cc = oracle.closed_form(D, dist[:, k], sub_off)
            assert np.array_equal(ct, tot) and np.array_equal(cc, cls), \
                "Algorithm 2 and its closed form disagree"
            dig = np.zeros((n_img, 16), np.uint8)
            for m in range(n_img):
                a, b = int(sub_off[m]), int(sub_off[m + 1])
                dig[m] = np.frombuffer(list_digest(idx[a:b, :k + 1], dist[a:b, :k + 1]), np.uint8)
            out[f"digest_k{k}"] = dig
    rows = np.arange(0, idx.shape[0], STRIDE)
    out["sample_rows"] = rows.astype(np.int64)
    out["sample_dist"] = dist[rows]
    if is_u8:
        out["sample_idx"] = idx[rows]
        D = np.concatenate(parts_D)
        nt, nc = oracle.nbnn(D, sub_off)
        out["nbnn_totals"] = nt
        out["nbnn_classes"] = nc
    else:
        out["nbr_idx"] = idx
    print(f"[{name}] done in {time.time() - t0:.0f} s", flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("name", choices=sorted(SPECS))
    ap.add_argument("--scratch", default="/tmp/lnbnn_fixture_parts",
                    help="where finished chunks are kept, so an interrupted run resumes")
    ap.add_argument("--chunk-images", type=int, default=4)
    a = ap.parse_args(argv)
    out = _compute(a.name, a.scratch, a.chunk_images)
    tmp = path(a.name) + ".tmp.npz"
    np.savez_compressed(tmp, **out)
    os.replace(tmp, path(a.name))
    print(f"wrote {path(a.name)} ({os.path.getsize(path(a.name)) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
