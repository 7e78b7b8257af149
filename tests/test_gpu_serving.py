"""Serving loop (continuous batching): every request's result equals the same
image classified alone (bit for bit) and the oracle's; admission, errors
and per-request timestamps behave as specified."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth

pytestmark = pytest.mark.gpu
F16 = L.LNBNN_EXACT_F16


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wait(ix, t, timeout=60.0, want_totals=True):
    t0 = time.time()
    while True:
        r = L.lnbnn_poll(ix, t, want_totals=want_totals)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {t} not done after {timeout} s")
        time.sleep(0.001)


@pytest.fixture(scope="module")
def served():
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(F16))
    L.lnbnn_serve_config(ix, max_batch_desc=8192, max_inflight=2)
    _, counts = synth.request_stream(48, 1000.0, median=300, lo=1, hi=3000)
    Q, off = synth.gen_requests(cfg, counts)
    yield cfg, R, labels, ix, Q, off
    ix.free()


def test_serving_matches_alone_and_oracle(served):
    cfg, R, labels, ix, Q, off = served
    n = len(off) - 1
    tickets = [L.lnbnn_submit(ix, Q[off[i]:off[i + 1]], 10, F16) for i in range(n)]
    results = [_wait(ix, t) for t in tickets]
    alone = L.lnbnn_classify(ix, Q, off, 10, F16, flags=L.LNBNN_PER_IMAGE_LAUNCH)
    want_t, want_c, _, _ = oracle.classify(Q, R, labels, cfg.n_classes, off, 10)
    batches = set()
    for i, (c, tot, st) in enumerate(results):
        assert c == alone[0][i] == want_c[i]
        assert np.array_equal(tot, alone[1][i]) and np.array_equal(tot, want_t[i])
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_start_ns"] <= st["t_done_ns"]
        assert st["n_desc"] == off[i + 1] - off[i] and st["batch_images"] >= 1
        batches.add(st["batch_id"])
    _say(f"{n} requests in {len(batches)} batches")
    assert len(batches) < n            # requests were batched together


def test_serving_mixed_k(served):
    cfg, R, labels, ix, Q, off = served
    ks = [5 if i % 3 else 10 for i in range(12)]
    tickets = [L.lnbnn_submit(ix, Q[off[i]:off[i + 1]], ks[i], F16) for i in range(12)]
    for i, t in enumerate(tickets):
        c, tot, _ = _wait(ix, t)
        want_t, want_c, _, _ = oracle.classify(Q[off[i]:off[i + 1]], R, labels, cfg.n_classes,
                                               np.array([0, off[i + 1] - off[i]]), ks[i])
        assert c == want_c[0] and np.array_equal(tot, want_t[0])


def test_serving_errors(served):
    cfg, R, labels, ix, Q, off = served
    big = np.zeros((8193, 128), np.uint8)
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_submit(ix, big, 10, F16)
    assert e.value.code == L.LNBNN_ENOMEM
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_poll(ix, 10 ** 9)
    assert e.value.code == L.LNBNN_ENOENT
    t = L.lnbnn_submit(ix, Q[:10], 10, F16)
    _wait(ix, t)
    with pytest.raises(L.LnbnnError) as e:            # consumed
        L.lnbnn_poll(ix, t)
    assert e.value.code == L.LNBNN_ENOENT
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_serve_config(ix, 1024, 2)             # already running
    assert e.value.code == L.LNBNN_EBUSY
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_submit(ix, Q[:10].astype(np.float32), 10, F16)
    assert e.value.code == L.LNBNN_EINVAL
    # an empty request is a legal image: class 0, totals 0
    c, tot, _ = _wait(ix, L.lnbnn_submit(ix, Q[:0], 10, F16))
    assert c == 0 and np.all(tot == 0)


def test_serving_busy_and_injected_failure():
    cfg = synth.scaled(synth.CONFIGS["T"], n_classes=4)
    R, labels = synth.gen_index(cfg)
    ix = L.lnbnn_build_index(R, labels, 4, L.LNBNN_MODE_BIT(F16))
    try:
        os.environ["LNBNN_FAULT"] = "launch"
        try:
            t = L.lnbnn_submit(ix, R[:50], 5, F16)
            with pytest.raises(L.LnbnnError) as e:
                _wait(ix, t)
            assert e.value.code == L.LNBNN_EDEVICE
        finally:
            del os.environ["LNBNN_FAULT"]
        ticket = L.lnbnn_submit(ix, R[:2000], 5, F16)
        # a pending ticket keeps the index alive
        rc = L.load().lnbnn_index_free(ix.handle)
        assert rc in (L.LNBNN_EBUSY, L.LNBNN_OK)
        if rc == L.LNBNN_OK:          # the ticket finished first: nothing was pending
            ix.handle = None
            return
        c, _, _ = _wait(ix, ticket)
        assert 0 <= c < 4
    finally:
        if ix.handle:
            ix.free()


@pytest.mark.parametrize("k", [10, 32])
def test_serving_fp8_matches_classify(k):
    """FP8 requests through the serving loop equal the batched classify,
    up to the largest k (64-entry candidate lists, 128 re-ranked)."""
    cfg = synth.scaled(synth.CONFIGS["P"], n_classes=6, n_train=3, n_desc=300, n_img=10, q_lo=100, q_hi=400,
                       index_seed=5100, query_seed=6100)
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(L.LNBNN_FP8_RERANK))
    try:
        tickets = [L.lnbnn_submit(ix, Q[off[i]:off[i + 1]], k, L.LNBNN_FP8_RERANK) for i in range(10)]
        batch = L.lnbnn_classify(ix, Q, off, k, L.LNBNN_FP8_RERANK)
        for i, t in enumerate(tickets):
            c, tot, _ = _wait(ix, t)
            assert c == batch[0][i] and np.array_equal(tot, batch[1][i])
    finally:
        ix.free()


def test_serving_exact_k32_matches_classify():
    """Exact requests at the largest k through the serving loop equal the
    batched classify and the oracle."""
    cfg = synth.scaled(synth.CONFIGS["T"], n_img=8, q_lo=50, q_hi=300)
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    I8 = L.LNBNN_EXACT_I8
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(I8))
    try:
        tickets = [L.lnbnn_submit(ix, Q[off[i]:off[i + 1]], 32, I8) for i in range(8)]
        want_t, want_c, _, _ = oracle.classify(Q, R, labels, cfg.n_classes, off, 32)
        for i, t in enumerate(tickets):
            c, tot, _ = _wait(ix, t)
            assert c == want_c[i] and np.array_equal(tot, want_t[i])
    finally:
        ix.free()


def test_serving_memory_budget_holds_under_load():
    """A small HBM budget (160 MiB, room for two slots of 4096 descriptors
    with lists for every k): the loop picks
    the batch capacity that fits it, the slots' measured workspace bytes stay
    within it, and while 120 requests of mixed sizes are queued and on the
    device no batch exceeds the capacity and no more than slots x capacity
    descriptors are in flight; a request above the capacity is refused with
    ENOMEM; every result equals the oracle."""
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    budget = 160 << 20
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(F16), hbm_budget_bytes=budget)
    try:
        info = L.lnbnn_serve_info(ix)
        assert info["started"] == 0 and info["hbm_budget"] == budget
        _, counts = synth.request_stream(120, 1000.0, median=600, lo=1, hi=4000)
        Q, off = synth.gen_requests(cfg, counts)
        tickets = [L.lnbnn_submit(ix, Q[off[i]:off[i + 1]], 10, F16) for i in range(len(off) - 1)]
        info = L.lnbnn_serve_info(ix)
        _say(f"serving: {info}")
        assert info["started"] == 1 and 0 < info["device_bytes"] <= budget
        cap, slots = info["batch_desc_cap"], info["slots"]
        assert cap >= 4000 and cap < (1 << 17)          # the budget, not the default, set it
        with pytest.raises(L.LnbnnError) as e:
            L.lnbnn_submit(ix, np.zeros((cap + 1, 128), np.uint8), 10, F16)
        assert e.value.code == L.LNBNN_ENOMEM
        results = {}
        while len(results) < len(tickets):
            info = L.lnbnn_serve_info(ix)
            assert info["device_bytes"] <= budget
            assert info["inflight_desc"] <= slots * cap and info["inflight_batches"] <= slots
            for i, t in enumerate(tickets):
                if i not in results:
                    r = L.lnbnn_poll(ix, t)
                    if r is not None:
                        results[i] = r
            time.sleep(0.0005)
        info = L.lnbnn_serve_info(ix)
        assert 0 < info["peak_batch_desc"] <= cap and info["peak_inflight_desc"] <= slots * cap
        assert info["queued_desc"] == 0 and info["inflight_desc"] == 0
        want_t, want_c, _, _ = oracle.classify(Q, R, labels, cfg.n_classes, off, 10)
        for i, (c, tot, _) in results.items():
            assert c == want_c[i] and np.array_equal(tot, want_t[i])
    finally:
        ix.free()
