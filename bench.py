"""Benchmark of the local NBNN hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a merged
index of 256 classes x 30 training images x 2000 descriptors = 15.36M
references (u8, 128-d), 512 query images of 500..4000 descriptors
(1.15M query descriptors in total), k = 10, exact path on the INT8 matrix
cores (bit-identical to the FP16 form, which is timed beside it for
context).  One step = one classification of the whole batch: distance +
top-(k+1) kernel, merge + class update, argmin, with the queries already
resident in HBM.

Prints one JSON line with the throughput (query descriptors/s), the
roofline of the dominant kernel (distance + top-(k+1), timed with HIP events
on its launch stream over the timed steps), the same batch through the
default launch path (captured graph replays, host-timed) and the CPU oracle
timed on a bounded sample of the same workload; then, in the same line, the
original NBNN rule on the same batch ("nbnn_original"), the FP8 candidate
pass + exact FP32 re-rank on float descriptors of the same shape with both
candidate rules and their quality against stored FP64 oracle results
("fp8_rerank", "fp8_rerank_2k"), the serving loop under a Poisson request
trace with p50/p99 image latency for the batched exact, batched FP8 and
plain per-image exact forms ("serving"), the class-count sweep for both
rules ("class_sweep") and the location-augmented rows.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_MFMA_F16_TFLOPS = 2500.0       # MI355X dense FP16/BF16 matrix peak
PEAK_MFMA_FP8_TFLOPS = 5000.0       # MI355X dense FP8 matrix peak
PEAK_MFMA_I8_TOPS = 5000.0          # MI355X dense INT8 matrix peak (TOP/s)
METRIC = "query descriptors/s at 15.4M refs k=10, exact vs FP8+rerank; p99 image ms"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dist_topk_traffic.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_1112_0059_amd", "csrc", f) for f in ("dist_topk.h", "dist_inst.hip")]
TUNING_CACHE = os.path.join(ROOT, "paper_1112_0059_amd", "tuning_cache.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the distance kernel's sources (template + instance unit)."""
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch(leg: str):
    """HBM bytes per launch of one leg's distance kernel (FETCH_SIZE +
    WRITE_SIZE, scaled by a device copy's reading) from the committed
    rocprofv3 counter summaries, or None when the kernel sources changed since
    the counters were taken.  Legs: exact_i8, exact_f16, nbnn, fp8_topk,
    fp8_2k, loc."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f).get(leg)
    except (OSError, ValueError):
        return None
    if not t or t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(R, Q, target_s: float = 15.0):
    """Time the oracle (its cache-blocked C route, OpenMP on every host core)
    on a bounded sample of query descriptors against the full index."""
    import oracle
    n = 64 * oracle.num_threads()          # one 64-query block per thread at least
    while True:
        t0 = time.perf_counter()
        oracle.knn(Q[:n], R, 11, route="block")
        dt = time.perf_counter() - t0
        if dt >= target_s / 3 or n >= Q.shape[0]:
            break
        n = min(Q.shape[0], max(n * 2, int(n * target_s / max(dt, 1e-3))))
    return {"value": n / dt, "unit": "query descriptors/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"the first {n} query descriptors against all 15.36M references, "
                      f"k+1 = 11 nearest by brute force (oracle block route, int32 direct form); {dt:.1f} s"}


def time_exact(args, L, torch, np, ix, dq, off, n_classes, mode, steps, warmup):
    """Classify the whole batch `steps` times (after `warmup` untimed runs)
    with direct launches and HIP events around the distance kernel; returns
    (wall s per step, mean distance-kernel ms, last timing, classes)."""
    n_img = off.shape[0] - 1
    out = {"class": torch.empty(n_img, dtype=torch.int32, device="cuda"),
           "totals": torch.empty((n_img, n_classes), dtype=torch.int64, device="cuda")}

    def step():
        L.lnbnn_classify(ix, dq, off, args.k, mode, flags=L.LNBNN_TIMING, out=out)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"mode {mode}: warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k1_ms = []
    for i in range(steps):
        step()
        k1_ms.append(L.lnbnn_last_timing(ix)["dist_kernel_ms"])   # waits for this step
        log(f"mode {mode}: step {i + 1}/{steps}: distance kernel {k1_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, float(np.mean(k1_ms)), L.lnbnn_last_timing(ix), out["class"].cpu().numpy()


def time_graph(args, L, torch, ix, dq, off, n_classes, mode, steps, f64=False):
    """The default launch path (captured graph, replayed), host-timed
    between synchronisations; wall s per step."""
    n_img = off.shape[0] - 1
    out = {"class": torch.empty(n_img, dtype=torch.int32, device="cuda"),
           "totals": torch.empty((n_img, n_classes), dtype=torch.float64 if f64 else torch.int64, device="cuda")}
    L.lnbnn_classify(ix, dq, off, args.k, mode, out=out)          # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        L.lnbnn_classify(ix, dq, off, args.k, mode, out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def exact_leg(args, L, torch, np, synth):
    cfg = synth.CONFIGS["L"]
    t0 = time.perf_counter()
    R, labels = synth.gen_index(cfg)
    Q, off, true_cls = synth.gen_queries(cfg)
    log(f"generated {R.shape[0]} refs, {Q.shape[0]} queries in {time.perf_counter() - t0:.1f}s")
    I8, F16, NB = L.LNBNN_EXACT_I8, L.LNBNN_EXACT_F16, L.LNBNN_NBNN_I8
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes,
                             L.LNBNN_MODE_BIT(I8) | L.LNBNN_MODE_BIT(F16) | L.LNBNN_MODE_BIT(NB))
    dq = torch.from_numpy(Q).cuda()
    n_img = off.shape[0] - 1
    tuned = {}
    if os.path.exists(TUNING_CACHE):
        # project autotuner: the cache holds the variant chosen on this
        # workload; a hit pins it without timing anything
        for mode in (I8, F16, NB):
            tuned[mode] = L.lnbnn_autotune(ix, dq, off, args.k, mode, cache_path=TUNING_CACHE)
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n_q = int(Q.shape[0])
    flop = 2.0 * 128 * cfg.n_refs * n_q
    dt, k1_ms, timing, cls = time_exact(args, L, torch, np, ix, dq, off, cfg.n_classes, I8, args.steps, args.warmup)
    achieved = flop / (k1_ms / 1e3) / 1e12
    res = {
        "metric": METRIC,
        "value": n_q / dt,
        "unit": "query descriptors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "L: merged index 256 classes x 30 images x 2000 u8 128-d "
                               "descriptors = 15.36M refs; 512 query images of 500..4000 "
                               f"descriptors ({n_q} total); k={args.k}; exact path on the INT8 "
                               "matrix cores (INT32 accumulation, bit-exact)",
                   "n_refs": cfg.n_refs, "n_query_desc": n_q, "n_images": n_img, "k": args.k,
                   "mode": "EXACT_I8",
                   "variant": L.lnbnn_variant_name(timing["tile_variant"]),
                   "autotuned": I8 in tuned,
                   "slices": timing["slices"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_I8_TOPS,
                     "unit": "TOP/s", "frac": achieved / PEAK_MFMA_I8_TOPS,
                     "traffic": traffic_per_launch("exact_i8"), "kernel": "k_dist_topk<OpI8T<4, FMT_I8>, 11, ...>",
                     "kernel_ms": k1_ms, "algorithmic_ops_per_launch": flop},
        "accuracy_statistic": float(np.mean(cls == true_cls)),
    }
    # the product's default path: the same batch replayed from a captured graph
    gsteps = max(1, min(args.steps, 5))
    dtg = time_graph(args, L, torch, ix, dq, off, cfg.n_classes, I8, gsteps)
    res["graph_path"] = {"ms_per_step": dtg * 1e3, "steps": gsteps, "value": n_q / dtg,
                         "vs_direct_launches": dt / dtg}
    log(f"graph path: {dtg * 1e3:.1f} ms per step (direct launches {dt * 1e3:.1f} ms)")
    # the original NBNN rule (Algorithm 1) on the same batch and index shape
    nsteps = max(1, min(args.steps, 3))
    dtn, k1n, tn, clsn = time_exact(args, L, torch, np, ix, dq, off, cfg.n_classes, NB, nsteps, 1)
    an = flop / (k1n / 1e3) / 1e12
    res["nbnn_original"] = {"value": n_q / dtn, "unit": "query descriptors/s", "steps": nsteps,
                            "ms_per_step": dtn * 1e3, "dtype": "i8",
                            "variant": L.lnbnn_variant_name(tn["tile_variant"]),
                            "same_classes_as_local": bool(np.array_equal(clsn, cls)),
                            "accuracy_statistic": float(np.mean(clsn == true_cls)),
                            "roofline": {"bound": "mfma", "achieved": an, "peak": PEAK_MFMA_I8_TOPS,
                                         "unit": "TOP/s", "frac": an / PEAK_MFMA_I8_TOPS, "kernel_ms": k1n,
                                         "traffic": traffic_per_launch("nbnn")}}
    if not args.no_f16:
        # the same exact classification on the FP16 matrix cores, for context
        steps16 = max(1, min(args.steps, 2))
        dt16, k1_16, t16, cls16 = time_exact(args, L, torch, np, ix, dq, off, cfg.n_classes, F16, steps16, 1)
        a16 = flop / (k1_16 / 1e3) / 1e12
        res["exact_f16"] = {"value": n_q / dt16, "unit": "query descriptors/s", "steps": steps16,
                            "ms_per_step": dt16 * 1e3, "dtype": "f16",
                            "variant": L.lnbnn_variant_name(t16["tile_variant"]),
                            "same_classes_as_i8": bool(np.array_equal(cls16, cls)),
                            "roofline": {"bound": "mfma", "achieved": a16, "peak": PEAK_MFMA_F16_TFLOPS,
                                         "unit": "TFLOP/s", "frac": a16 / PEAK_MFMA_F16_TFLOPS,
                                         "kernel_ms": k1_16, "traffic": traffic_per_launch("exact_f16")}}
    return res, ix, R, Q, cfg


def loc_leg(args, L, torch, np, synth):
    """The exact path on location-augmented rows at L's sizes: 160 u8 bytes
    per descriptor (the descriptor, then 16 copies of each coordinate code
    carrying the location weight alpha = 1.6), INT8 mode."""
    cfg = synth.CONFIGS["L"]
    t0 = time.perf_counter()
    R, labels = synth.gen_index(cfg, loc=True)
    Q, off, true_cls = synth.gen_queries(cfg, loc=True)
    log(f"generated {R.shape[0]} x {R.shape[1]} location-augmented refs, {Q.shape[0]} queries "
        f"in {time.perf_counter() - t0:.1f}s")
    I8 = L.LNBNN_EXACT_I8
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    del R
    try:
        dq = torch.from_numpy(Q).cuda()
        tuned = os.path.exists(TUNING_CACHE)
        if tuned:
            L.lnbnn_autotune(ix, dq, off, args.k, I8, cache_path=TUNING_CACHE)
        steps = max(1, min(args.steps, 3))
        dt, k1_ms, timing, cls = time_exact(args, L, torch, np, ix, dq, off, cfg.n_classes, I8, steps, 1)
    finally:
        ix.free()
    n_q = int(Q.shape[0])
    ops = 2.0 * synth.DIM_LOC * cfg.n_refs * n_q
    a = ops / (k1_ms / 1e3) / 1e12
    return {"value": n_q / dt, "unit": "query descriptors/s", "steps": steps, "ms_per_step": dt * 1e3,
            "dtype": "i8",
            "config": {"workload": "L with location-augmented rows: 15.36M refs x 160 u8 (descriptor "
                                   "+ 16 copies of each alpha-weighted coordinate code); 512 query "
                                   f"images ({n_q} descriptors); k={args.k}; exact, INT8 matrix cores",
                       "variant": L.lnbnn_variant_name(timing["tile_variant"]), "autotuned": tuned},
            "roofline": {"bound": "mfma", "achieved": a, "peak": PEAK_MFMA_I8_TOPS, "unit": "TOP/s",
                         "frac": a / PEAK_MFMA_I8_TOPS, "kernel": "k_dist_topk<OpI8T<5, FMT_I8L>, 11, ...>",
                         "kernel_ms": k1_ms, "algorithmic_ops_per_launch": ops,
                         "traffic": traffic_per_launch("loc")},
            "accuracy_statistic": float(np.mean(cls == true_cls))}


def fp8_quality(L, torch, np, ix, dq, off, k, mode, n_classes):
    """Neighbour recall, identical lists, decision agreement and score error
    of the FP8 path against stored FP64 oracle results for 64 whole images
    of this batch (tests/golden/oracle_P.npz, written from the oracle), or
    None if they have not been written."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        import oracle_fixtures as F
        fx = F.load("P")
    except Exception:
        return None
    if fx is None or k != 10:
        return None
    imgs = fx["images"]
    rows = np.concatenate([np.arange(off[m], off[m + 1]) for m in imgs])
    if not np.array_equal(np.diff(fx["offsets"]), np.diff(off)[imgs]):
        return {"error": "stored images do not match this batch"}
    cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, k, mode, want_neighbours=True)
    torch.cuda.synchronize()
    cls, tot, ni = cls.cpu().numpy()[imgs], tot.cpu().numpy()[imgs], ni.cpu().numpy()[rows]
    wi = fx["nbr_idx"]
    hits = (ni[:, :, None] == wi[:, None, :]).any(axis=2).sum(axis=1)
    wt, wc = fx["totals_k10"], fx["classes_k10"]
    err = np.abs(tot - wt).max(axis=1) / np.abs(wt).max(axis=1)
    return {"images": int(len(imgs)), "descriptors": int(rows.size),
            "recall": float(hits.mean() / (k + 1)),
            "identical_lists": float(np.mean(np.all(ni == wi, axis=1))),
            "decision_agreement": f"{int(np.sum(cls == wc))}/{len(imgs)}",
            "max_score_error_rel": float(err.max()),
            "against": "FP64 oracle (Algorithm 2 on exact kNN), every 8th image of the batch"}


def fp8_leg(args, L, torch, np, synth):
    """FP8 candidate pass (4k) + exact FP32 re-rank on float descriptors with
    config L's structure, with both candidate rules: the FP8 top 4k
    (LNBNN_FP8_RERANK) and the best 4k of per-row-half lists of 2k
    (LNBNN_FP8_RERANK_2K); each with its quality against stored FP64 oracle
    results when they exist."""
    cfg = synth.CONFIGS["P"]
    t0 = time.perf_counter()
    R, labels = synth.gen_index(cfg)
    Q, off, true_cls = synth.gen_queries(cfg)
    log(f"fp8: generated {R.shape[0]} float refs, {Q.shape[0]} queries in {time.perf_counter() - t0:.1f}s")
    FP8, FP8_2K = L.LNBNN_FP8_RERANK, L.LNBNN_FP8_RERANK_2K
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(FP8) | L.LNBNN_MODE_BIT(FP8_2K))
    del R
    dq = torch.from_numpy(Q).cuda()
    n_img = off.shape[0] - 1
    n_q = int(Q.shape[0])
    flop = 2.0 * 128 * cfg.n_refs * n_q
    out = {"class": torch.empty(n_img, dtype=torch.int32, device="cuda"),
           "totals": torch.empty((n_img, cfg.n_classes), dtype=torch.float64, device="cuda")}
    tuned = os.path.exists(TUNING_CACHE)
    legs = {}
    for mode, name in ((FP8, "top 4k"), (FP8_2K, "best 4k of per-half 2k lists")):
        if tuned:
            # the tuned launch for this workload (a cache hit times nothing)
            L.lnbnn_autotune(ix, dq, off, args.k, mode, cache_path=TUNING_CACHE)
        L.lnbnn_classify(ix, dq, off, args.k, mode, flags=L.LNBNN_TIMING, out=out)
        torch.cuda.synchronize()
        steps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        k1_ms, tot_ms = [], []
        for i in range(steps):
            L.lnbnn_classify(ix, dq, off, args.k, mode, flags=L.LNBNN_TIMING, out=out)
            t = L.lnbnn_last_timing(ix)
            k1_ms.append(t["dist_kernel_ms"])
            tot_ms.append(t["total_ms"])
            log(f"fp8 mode {mode} step {i + 1}/{steps}: candidate pass {k1_ms[-1]:.1f} ms, "
                f"whole sequence {tot_ms[-1]:.1f} ms")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc = float(np.mean(out["class"].cpu().numpy() == true_cls))
        k1 = float(np.mean(k1_ms)) / 1e3
        achieved = flop / k1 / 1e12
        legs[mode] = {
            "metric": "query descriptors/s at 15.4M refs k=10 (FP8 candidates + exact FP32 re-rank)",
            "value": n_q * steps / dt, "unit": "query descriptors/s", "steps": steps,
            "ms_per_step": dt / steps * 1e3, "dtype": "fp8 e4m3 -> f32",
            "config": {"workload": "P: 15.36M float32 refs (L structure, unit-norm ReLU descriptors, noise 0.08), "
                                   f"{n_q} query descriptors in 512 images; k={args.k}, 4k candidates ({name})",
                       "variant": L.lnbnn_variant_name(L.lnbnn_last_timing(ix)["tile_variant"]),
                       "autotuned": tuned},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_FP8_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_MFMA_FP8_TFLOPS, "kernel": "k_dist_topk (FP8 candidate pass)",
                         "kernel_ms": k1 * 1e3, "sequence_ms": float(np.mean(tot_ms)),
                         "traffic": traffic_per_launch("fp8_topk" if mode == FP8 else "fp8_2k")},
            "quality": fp8_quality(L, torch, np, ix, dq, off, args.k, mode, cfg.n_classes),
            "accuracy_statistic": acc,
        }
        log(f"fp8 mode {mode}: quality {legs[mode]['quality']}")
    return legs[FP8], legs[FP8_2K], ix


def serving_leg(args, L, torch, np, synth, ix_exact, ix_fp8, mu_exact_qps, out=None):
    """Poisson request trace at offered load rho * (batched exact capacity);
    n ~ clip(LogNormal(ln 1500, 0.6), 100, 8000).  Batched exact and FP8 go
    through lnbnn_submit/lnbnn_poll; the plain form classifies each request
    alone with per-image launches, in arrival order.  Runs the exact forms
    when ix_exact is given and the FP8 form when ix_fp8 is given, adding to
    `out` (the same trace and rates either way)."""
    import threading
    from collections import deque
    n_warm, n_meas = args.serve_warmup, args.serve_requests
    n_req = n_warm + n_meas
    unit_arrivals, counts = synth.request_stream(n_req, 1.0, seed=3000)
    mu_img = mu_exact_qps / float(np.mean(counts))        # batched exact capacity, images/s
    if out is None:
        out = {}
    out.update({"capacity_images_per_s": mu_img, "requests_measured": n_meas, "requests_warmup": n_warm,
                "trace": "Poisson arrivals at rho x capacity; n ~ clip(round(LogNormal(ln 1500, 0.6)), 100, 8000)"})
    arrivals = unit_arrivals

    def run_batched(ix, mode, Qr, offr):
        tickets = [None] * n_req
        lat = np.zeros(n_req)
        done = np.zeros(n_req, bool)
        t_base = time.monotonic()
        next_poll = deque()
        for i in range(n_req):
            while time.monotonic() - t_base < arrivals[i]:
                if next_poll:
                    j = next_poll[0]
                    r = L.lnbnn_poll(ix, tickets[j], want_totals=False)
                    if r is not None:
                        lat[j] = (r[2]["t_done_ns"] - r[2]["t_submit_ns"]) / 1e6
                        done[j] = True
                        next_poll.popleft()
                        continue
                time.sleep(0.0002)
            tickets[i] = L.lnbnn_submit(ix, Qr[offr[i]:offr[i + 1]], args.k, mode)
            next_poll.append(i)
        while next_poll:
            j = next_poll[0]
            r = L.lnbnn_poll(ix, tickets[j], want_totals=False)
            if r is None:
                time.sleep(0.0002)
                continue
            lat[j] = (r[2]["t_done_ns"] - r[2]["t_submit_ns"]) / 1e6
            done[j] = True
            next_poll.popleft()
        wall = time.monotonic() - t_base - arrivals[n_warm]
        return lat[n_warm:], n_meas / wall

    def run_plain(ix, mode, Qr, offr):
        lat = np.zeros(n_req)
        q = deque()
        cv = threading.Condition()
        t_base = time.monotonic()
        end = [0.0]

        def worker():
            for _ in range(n_req):
                with cv:
                    while not q:
                        cv.wait()
                    i = q.popleft()
                L.lnbnn_classify(ix, Qr[offr[i]:offr[i + 1]], np.array([0, offr[i + 1] - offr[i]]), args.k, mode,
                                 flags=L.LNBNN_PER_IMAGE_LAUNCH | L.LNBNN_NO_GRAPH)
                lat[i] = (time.monotonic() - t_base - arrivals[i]) * 1e3
            end[0] = time.monotonic()

        th = threading.Thread(target=worker)
        th.start()
        for i in range(n_req):
            dtw = arrivals[i] - (time.monotonic() - t_base)
            if dtw > 0:
                time.sleep(dtw)
            with cv:
                q.append(i)
                cv.notify()
        th.join()
        wall = end[0] - t_base - arrivals[n_warm]
        return lat[n_warm:], n_meas / wall

    def summary(lat, ips):
        return {"images_per_s": ips, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(np.mean(lat))}

    Qr = offr = Qf = offf = None
    if ix_exact is not None:
        Qr, offr = synth.gen_requests(synth.CONFIGS["L"], counts)
    if ix_fp8 is not None:
        Qf, offf = synth.gen_requests(synth.CONFIGS["P"], counts)
    for rho in (0.7, 0.9):
        lam = rho * mu_img
        arrivals = unit_arrivals / lam
        r = out.setdefault(f"rho_{rho}", {})
        r.update({"offered_load": rho, "arrival_rate_per_s": lam})
        log(f"serving rho={rho}: {n_req} requests, rate {lam:.1f}/s")
        if Qr is not None:
            r["batched_exact"] = summary(*run_batched(ix_exact, L.LNBNN_EXACT_I8, Qr, offr))
            log(f"serving batched exact: {r['batched_exact']}")
            # the plain form (one launch per image, no batching) at both loads
            r["plain_per_image_exact"] = summary(*run_plain(ix_exact, L.LNBNN_EXACT_I8, Qr, offr))
            log(f"serving plain exact: {r['plain_per_image_exact']}")
        if Qf is not None:
            r["batched_fp8_rerank"] = summary(*run_batched(ix_fp8, L.LNBNN_FP8_RERANK, Qf, offf))
            log(f"serving batched fp8: {r['batched_fp8_rerank']}")
    return out


def class_sweep_leg(args, L, torch, np, synth):
    """Local NBNN (exact, INT8) and the original NBNN rule (Algorithm 1, on
    the same tiles) as the number of classes grows at a fixed 30 x 2000
    references per class (64 query images of the same size mix per point):
    the two curves of the paper's class-count experiment (Fig. 5).  With
    exact search both rules visit every reference, so both are linear in the
    number of references; the paper's 100x gap belongs to its approximate
    per-class indexes."""
    base = synth.CONFIGS["L"]
    rows = []
    I8, NB = L.LNBNN_EXACT_I8, L.LNBNN_NBNN_I8
    for nc in (2, 8, 32, 128, 256):
        cfg = synth.scaled(base, n_classes=nc, n_img=64)
        R, labels = synth.gen_index(cfg)
        Q, off, true_cls = synth.gen_queries(cfg)
        ix = L.lnbnn_build_index(R, labels, nc, L.LNBNN_MODE_BIT(I8) | L.LNBNN_MODE_BIT(NB))
        del R
        dq = torch.from_numpy(Q).cuda()
        n_q = int(Q.shape[0])
        row = {"n_classes": nc, "n_refs": cfg.n_refs, "query_desc": n_q}
        for mode, name in ((I8, "local_nbnn"), (NB, "nbnn_original")):
            dt, k1, _, cls = time_exact(args, L, torch, np, ix, dq, off, nc, mode, 2, 1)
            row[name] = {"query_desc_per_s": n_q / dt, "ms_per_image": dt * 1e3 / 64, "dist_kernel_ms": k1,
                         "dist_kernel_ops_per_s": 2.0 * 128 * cfg.n_refs * n_q / (k1 / 1e3),
                         "accuracy_statistic": float(np.mean(cls == true_cls))}
        ix.free()
        rows.append(row)
        log(f"class sweep: {rows[-1]}")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--legs", default="exact,fp8,serving,sweep,loc",
                    help="comma list: exact (always), fp8, serving, sweep, loc")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f16", action="store_true", help="skip the FP16 context timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    legs = set(args.legs.split(","))

    import numpy as np
    import torch

    import paper_1112_0059_amd as L
    import synth

    torch.cuda.set_device(0)
    res, ix, R, Q, cfg = exact_leg(args, L, torch, np, synth)
    # Each serving form runs right after its own workload's leg, and the
    # host-side CPU baseline last: with both the CPU baseline and the float
    # workload's leg run before it in this process, exact serving latency
    # tripled (host-side state of the benchmark process, not of the GPU).
    if "serving" in legs:
        try:
            res["serving"] = serving_leg(args, L, torch, np, synth, ix, None, res["value"])
            res["p99_image_ms"] = res["serving"]["rho_0.7"]["batched_exact"]["p99_ms"]
        except Exception as e:
            res["serving"] = {"error": repr(e)}
    ix8 = None
    if "fp8" in legs:
        try:
            res["fp8_rerank"], res["fp8_rerank_2k"], ix8 = fp8_leg(args, L, torch, np, synth)
        except Exception as e:  # the headline line must still be printed
            res["fp8_rerank"] = {"error": repr(e)}
    if "serving" in legs and ix8 is not None and "error" not in res.get("serving", {}):
        try:
            serving_leg(args, L, torch, np, synth, None, ix8, res["value"], out=res["serving"])
        except Exception as e:
            res["serving"]["fp8_error"] = repr(e)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(R, Q)
    del R, Q
    for x in (ix8, ix):
        try:
            if x is not None:
                x.free()                  # frees the HBM for the sweep's indexes
        except Exception as e:
            log(f"index free: {e!r}")
    if "sweep" in legs:
        try:
            res["class_sweep"] = class_sweep_leg(args, L, torch, np, synth)
        except Exception as e:
            res["class_sweep"] = {"error": repr(e)}
    if "loc" in legs:
        try:
            res["location_augmented"] = loc_leg(args, L, torch, np, synth)
        except Exception as e:
            res["location_augmented"] = {"error": repr(e)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
