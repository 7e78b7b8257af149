"""Autotuner front end: time every tile variant that can serve (mode, k) on a
synthetic workload of a named shape and record the fastest in a tuning
cache (flat JSON, key = arch, n_refs, dim, list-length bucket, mode).

    python -m paper_1112_0059_amd.tune --config L --mode f16 --k 10 --cache out.json
    python -m paper_1112_0059_amd.tune --config L --mode i8 --loc --k 10 --cache out.json

A later lnbnn_autotune call with the same cache and an index of the same
shape pins the recorded variant without timing anything.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

MODES = {"f16": 0, "bf16": 1, "fp8": 2, "i8": 3, "fp8_2k": 4, "nbnn": 5}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="L", help="synthetic workload (synth.CONFIGS key)")
    ap.add_argument("--mode", default="f16", choices=sorted(MODES))
    ap.add_argument("--k", type=int, nargs="+", default=[10])
    ap.add_argument("--images", type=int, default=0, help="query images to time on (0 = all)")
    ap.add_argument("--cache", required=True)
    ap.add_argument("--loc", action="store_true", help="location-augmented 160-byte rows (INT8 mode)")
    args = ap.parse_args(argv)

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import paper_1112_0059_amd as L
    import synth

    cfg = synth.CONFIGS[args.config]
    mode = MODES[args.mode]
    if (mode in L.FP8_MODES) != (cfg.kind == "f32"):
        sys.exit(f"config {args.config} holds {cfg.kind} descriptors; mode {args.mode} needs "
                 f"{'f32' if mode in L.FP8_MODES else 'u8'}")
    if args.loc and mode != L.LNBNN_EXACT_I8:
        sys.exit("--loc needs --mode i8")
    R, labels = synth.gen_index(cfg, loc=args.loc)
    Q, off, _ = synth.gen_queries(cfg, loc=args.loc)
    if args.images:
        off = off[:args.images + 1]
        Q = Q[:off[-1]]
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(mode))
    del R
    dq = torch.from_numpy(Q).cuda()
    try:
        for k in args.k:
            t0 = time.perf_counter()
            v = L.lnbnn_autotune(ix, dq, off, k, mode, cache_path=args.cache)
            print(f"{args.config}{' loc' if args.loc else ''} mode={args.mode} k={k}: variant {v} ({L.lnbnn_variant_name(v)}) "
                  f"in {time.perf_counter() - t0:.1f} s", flush=True)
    finally:
        ix.free()


if __name__ == "__main__":
    main()
