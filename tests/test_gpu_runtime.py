"""Runtime behaviour around the kernels: the bounded stage waits report when
they give up, the graph cache stays bounded and correct across evictions,
a classify call whose workspace grows while the serving loop runs on the
same index, the serving loop's recovery from a failed start, and the timing
record of the per-image form."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth

pytestmark = pytest.mark.gpu
I8 = L.LNBNN_EXACT_I8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wait(ix, t, timeout=60.0):
    t0 = time.time()
    while True:
        r = L.lnbnn_poll(ix, t)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {t} not done after {timeout} s")
        time.sleep(0.001)


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    want = oracle.classify(Q, R, labels, cfg.n_classes, off, 10)
    return cfg, R, labels, Q, off, want


def test_wait_that_gives_up_is_reported(tiny):
    """The host sets the stage waits' bound to zero rounds: the kernel still
    runs to its end (every wait simply stops waiting), and the call reports
    LNBNN_EDEVICE instead of returning silently wrong lists.  With the
    normal bound the same index classifies exactly again."""
    import torch
    cfg, R, labels, Q, off, (wt, wc, wi, wd) = tiny
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        # an 8-bit-tile variant with per-buffer counters (the bounded waits)
        L.lnbnn_set_variant(ix, I8, 10, 8)
        os.environ["LNBNN_WAIT_SPINS"] = "0"
        try:
            _say("host pointers, zero wait bound")
            with pytest.raises(L.LnbnnError) as e:
                L.lnbnn_classify(ix, Q, off, 10, I8)
            assert e.value.code == L.LNBNN_EDEVICE and "bounded wait" in str(e.value)
            _say("device pointers, zero wait bound: reported by lnbnn_sync_status")
            dq = torch.from_numpy(Q).cuda()
            L.lnbnn_classify(ix, dq, off, 10, I8)
            with pytest.raises(L.LnbnnError) as e:
                L.lnbnn_sync_status(ix)
            assert e.value.code == L.LNBNN_EDEVICE
        finally:
            del os.environ["LNBNN_WAIT_SPINS"]
        L.lnbnn_sync_status(ix)                      # reported once, then clear
        cls, tot, ni, nd = L.lnbnn_classify(ix, Q, off, 10, I8, want_neighbours=True)
        assert np.array_equal(ni, wi) and np.array_equal(tot, wt) and np.array_equal(cls, wc)
    finally:
        ix.free()


@pytest.mark.parametrize("mode", [L.LNBNN_FP8_RERANK, L.LNBNN_NBNN_I8])
def test_wait_that_gives_up_is_reported_other_modes(tiny, mode):
    """The same for the FP8 candidate pass (the candidate merge reads the
    mark) and the original NBNN rule (its per-class flush reads it)."""
    cfg, R, labels, Q, off, _ = tiny
    if mode == L.LNBNN_FP8_RERANK:
        R = (R.astype(np.float32) + 1.0) / 256.0
        Q = (Q.astype(np.float32) + 1.0) / 256.0
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(mode))
    try:
        L.lnbnn_set_variant(ix, mode, 10, 11 if mode == L.LNBNN_FP8_RERANK else 8)
        want = L.lnbnn_classify(ix, Q, off, 10, mode)
        os.environ["LNBNN_WAIT_SPINS"] = "0"
        try:
            _say(f"mode {mode}, zero wait bound")
            with pytest.raises(L.LnbnnError) as e:
                L.lnbnn_classify(ix, Q, off, 10, mode)
            assert e.value.code == L.LNBNN_EDEVICE
        finally:
            del os.environ["LNBNN_WAIT_SPINS"]
        got = L.lnbnn_classify(ix, Q, off, 10, mode)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    finally:
        ix.free()


def test_graph_cache_bounded_and_exact(tiny):
    """Twelve launch shapes (k = 1..12) through the default graph path: more
    than the cache keeps, so entries are evicted and recaptured; every call
    equals the oracle, and a shape seen again after its eviction too."""
    cfg, R, labels, Q, off, _ = tiny
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        for k in list(range(1, 13)) + [1, 2]:
            _say(f"graph path k={k}")
            wt, wc, wi, wd = oracle.classify(Q, R, labels, cfg.n_classes, off, k)
            cls, tot, ni, nd = L.lnbnn_classify(ix, Q, off, k, I8, want_neighbours=True)
            assert np.array_equal(ni, wi) and np.array_equal(tot, wt) and np.array_equal(cls, wc)
    finally:
        ix.free()


def test_graph_serves_other_buffers_and_sizes(tiny):
    """One bucket's graph serves batches of other sizes and other device
    buffers (the data pointers travel in the batch descriptor)."""
    import torch
    cfg, R, labels, Q, off, _ = tiny
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        for n_img in (20, 17, 9, 20):
            sub = off[:n_img + 1]
            wt, wc, wi, wd = oracle.classify(Q[:sub[-1]], R, labels, cfg.n_classes, sub, 10)
            dq = torch.from_numpy(Q[:sub[-1]].copy()).cuda()        # a fresh buffer each time
            cls, tot, ni, nd = L.lnbnn_classify(ix, dq, sub, 10, I8, want_neighbours=True)
            torch.cuda.synchronize()
            assert np.array_equal(ni.cpu().numpy(), wi) and np.array_equal(tot.cpu().numpy(), wt)
            assert np.array_equal(cls.cpu().numpy(), wc)
    finally:
        ix.free()


def test_classify_grows_while_serving(tiny):
    """Requests in flight on the serving loop while classify calls on the
    same index grow its workspace twice: every result equals the oracle."""
    cfg, R, labels, Q, off, _ = tiny
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        L.lnbnn_serve_config(ix, max_batch_desc=4096, max_inflight=2)
        tickets = [L.lnbnn_submit(ix, Q[off[m]:off[m + 1]], 10, I8) for m in range(cfg.n_img)]
        for n_img in (2, 8, 20):                      # each call larger than any before
            sub = off[:n_img + 1]
            _say(f"classify {n_img} images with {len(tickets)} tickets submitted")
            wt, wc, _, _ = oracle.classify(Q[:sub[-1]], R, labels, cfg.n_classes, sub, 10)
            cls, tot, _, _ = L.lnbnn_classify(ix, Q[:sub[-1]], sub, 10, I8)
            assert np.array_equal(tot, wt) and np.array_equal(cls, wc)
            tickets += [L.lnbnn_submit(ix, Q[off[m]:off[m + 1]], 10, I8) for m in range(3)]
        wt, wc, _, _ = oracle.classify(Q, R, labels, cfg.n_classes, off, 10)
        for i, t in enumerate(tickets):
            m = i if i < cfg.n_img else (i - cfg.n_img) % 3
            c, tot, _ = _wait(ix, t)
            assert c == wc[m] and np.array_equal(tot, wt[m])
    finally:
        ix.free()


def test_serving_recovers_from_failed_start(tiny):
    """The first submit finds no device memory for its slots (injected): it
    fails and leaves nothing half-built behind; the next submit starts the
    loop afresh and its result equals the oracle."""
    cfg, R, labels, Q, off, (wt, wc, _, _) = tiny
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        os.environ["LNBNN_FAULT"] = "alloc"
        try:
            with pytest.raises(L.LnbnnError) as e:
                L.lnbnn_submit(ix, Q[:200], 10, I8)
            assert e.value.code in (L.LNBNN_ENOMEM, L.LNBNN_EDEVICE)
        finally:
            del os.environ["LNBNN_FAULT"]
        t = L.lnbnn_submit(ix, Q[off[3]:off[4]], 10, I8)
        c, tot, _ = _wait(ix, t)
        assert c == wc[3] and np.array_equal(tot, wt[3])
    finally:
        ix.free()


def test_per_image_timing_covers_every_launch(tiny):
    """The timed per-image form: the whole-sequence time is at least the
    summed distance-kernel time of its per-image launches."""
    cfg, R, labels, Q, off, (wt, wc, _, _) = tiny
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        cls, tot, _, _ = L.lnbnn_classify(ix, Q, off, 10, I8, flags=L.LNBNN_PER_IMAGE_LAUNCH | L.LNBNN_TIMING)
        assert np.array_equal(tot, wt) and np.array_equal(cls, wc)
        t = L.lnbnn_last_timing(ix)
        assert t["dist_launches"] == cfg.n_img
        assert t["total_ms"] >= t["dist_kernel_ms"] > 0
    finally:
        ix.free()


def test_environment_settings(tiny, tmp_path, capfd):
    """LNBNN_HBM_BUDGET sets the serving budget of an index built with
    budget 0; LNBNN_TUNE_CACHE is the cache lnbnn_autotune uses without a
    path; LNBNN_LOG=1 writes one line per build, graph capture, tuner
    decision and serving start to stderr."""
    import json
    import torch
    cfg, R, labels, Q, off, (wt, wc, _, _) = tiny
    cache = str(tmp_path / "env_cache.json")
    env = {"LNBNN_HBM_BUDGET": "96M", "LNBNN_TUNE_CACHE": cache, "LNBNN_LOG": "1"}
    os.environ.update(env)
    try:
        ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
        try:
            assert L.lnbnn_serve_info(ix)["hbm_budget"] == 96 << 20
            v = L.lnbnn_autotune(ix, torch.from_numpy(Q).cuda(), off, 10, I8)
            with open(cache) as f:
                entries = json.load(f)
            assert len(entries) == 1 and (next(iter(entries.values())) & 0xFF) == v
            cls, tot, _, _ = L.lnbnn_classify(ix, Q, off, 10, I8)
            assert np.array_equal(tot, wt) and np.array_equal(cls, wc)
            c, t, _ = _wait(ix, L.lnbnn_submit(ix, Q[off[2]:off[3]], 10, I8))
            assert c == wc[2] and np.array_equal(t, wt[2])
        finally:
            ix.free()
    finally:
        for name in env:
            del os.environ[name]
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("[lnbnn]")]
    for what in ("index built", "tuner:", "graph captured", "serving started"):
        assert any(what in ln for ln in lines), (what, lines)
