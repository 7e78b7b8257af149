"""Location-augmented descriptors on the INT8 path (160-byte rows: the
descriptor, then the alpha-weighted location codes of Sec. 6), through the
C ABI, bit-exact against the oracle: neighbour indices and squared
distances, int64 totals and decisions.  The 160-element rows use their own
tiles (five K steps) and stage shapes, so every one of those shapes, the
chunked walk, the launch forms, device pointers, edge cases and the serving
loop are covered here."""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth

pytestmark = pytest.mark.gpu
I8 = L.LNBNN_EXACT_I8
BIT = L.LNBNN_MODE_BIT(I8)
LOC_VARIANTS = (2, 7, 10, 11, 19)      # the stage shapes built for 5 KB tiles


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_exact(got, want):
    cls, tot, ni, nd = got
    wt, wc, wi, wd = want
    assert np.array_equal(ni, wi), "neighbour indices differ"
    assert np.array_equal(nd.astype(np.int64), wd), "neighbour distances differ"
    assert np.array_equal(tot, wt), "totals differ"
    assert np.array_equal(cls, wc), "classes differ"


@pytest.fixture(scope="module")
def small():
    # 10 x 5 x 203 = 10,150 references (a ragged last tile), 24 images of
    # 1..400 descriptors
    cfg = synth.scaled(synth.CONFIGS["T"], n_desc=203, n_img=24, q_lo=1, q_hi=400)
    R, labels = synth.gen_index(cfg, loc=True)
    Q, off, _ = synth.gen_queries(cfg, loc=True)
    assert R.shape[1] == Q.shape[1] == L.LNBNN_DIM_LOC
    _say(f"loc small: {R.shape[0]} refs, {Q.shape[0]} queries")
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, BIT)
    ref = {k: oracle.classify(Q, R, labels, cfg.n_classes, off, k) for k in (1, 5, 10, 20, 32)}
    yield cfg, R, labels, Q, off, ix, ref
    ix.free()


@pytest.mark.parametrize("k", [1, 5, 10, 20, 32])
def test_loc_bit_exact(small, k):
    cfg, R, labels, Q, off, ix, ref = small
    _say(f"loc k={k}")
    _check_exact(L.lnbnn_classify(ix, Q, off, k, I8, want_neighbours=True), ref[k])


def test_loc_every_variant(small):
    cfg, R, labels, Q, off, ix, ref = small
    for v in range(L.lnbnn_num_variants()):
        for k in (10, 32):
            _say(f"loc variant {v} k={k}")
            try:
                L.lnbnn_set_variant(ix, I8, k, v)
            except L.LnbnnError:      # not built for 160-element rows / this list length
                assert v not in LOC_VARIANTS or (k == 32 and v not in (11, 19))
                continue
            assert v in LOC_VARIANTS
            try:
                _check_exact(L.lnbnn_classify(ix, Q, off, k, I8, want_neighbours=True), ref[k])
            finally:
                L.lnbnn_set_variant(ix, I8, k, -1)


@pytest.mark.parametrize("variant", [7, 10, 11, 19])
def test_loc_chunked_walk(small, variant):
    """Few resident workgroups and 8-tile chunks: lists are parked and
    restored between chunks."""
    cfg, R, labels, Q, off, ix, ref = small
    _say(f"loc chunked walk variant {variant}")
    L.lnbnn_set_tuning(ix, I8, 10, variant=variant, chunk_tiles=8, max_workgroups=3)
    try:
        _check_exact(L.lnbnn_classify(ix, Q, off, 10, I8, want_neighbours=True), ref[10])
    finally:
        L.lnbnn_set_tuning(ix, I8, 10)


@pytest.mark.parametrize("flags", [L.LNBNN_NO_GRAPH, L.LNBNN_PER_IMAGE_LAUNCH, L.LNBNN_TIMING])
def test_loc_launch_forms(small, flags):
    cfg, R, labels, Q, off, ix, ref = small
    _say(f"loc flags={flags}")
    _check_exact(L.lnbnn_classify(ix, Q, off, 10, I8, flags=flags, want_neighbours=True), ref[10])


def test_loc_device_pointers(small):
    import torch
    cfg, R, labels, Q, off, ix, ref = small
    dq = torch.from_numpy(Q).cuda()
    for rep in range(3):
        got = L.lnbnn_classify(ix, dq, off, 5, I8, want_neighbours=True)
        torch.cuda.synchronize()
        _check_exact(tuple(x.cpu().numpy() for x in got), ref[5])


def test_loc_edge_cases():
    """Tiny indexes (k + 1 = n_refs, two references), duplicate rows, a
    query equal to a reference, all-zero and all-255 rows, empty images."""
    rng = np.random.default_rng(8)
    for n_refs, k in ((2, 1), (11, 10), (300, 10), (257, 32)):
        R = rng.integers(0, 256, size=(n_refs, 160)).astype(np.uint8)
        R[0] = 0
        if n_refs > 2:
            R[2] = R[1]
            R[-1] = 255
        labels = rng.integers(0, 4, size=n_refs).astype(np.int32)
        Q = rng.integers(0, 256, size=(40, 160)).astype(np.uint8)
        Q[5] = R[1]
        Q[6] = 255
        off = np.array([0, 0, 1, 40, 40], np.int64)
        _say(f"loc edge n_refs={n_refs} k={k}")
        want = oracle.classify(Q, R, labels, 4, off, k)
        ix = L.lnbnn_build_index(R, labels, 4, BIT)
        try:
            _check_exact(L.lnbnn_classify(ix, Q, off, k, I8, want_neighbours=True), want)
        finally:
            ix.free()


def test_loc_rejects():
    R = np.zeros((64, 160), np.uint8)
    lab = np.zeros(64, np.int32)
    for mask in (L.LNBNN_MODE_BIT(L.LNBNN_EXACT_F16), BIT | L.LNBNN_MODE_BIT(L.LNBNN_EXACT_BF16)):
        with pytest.raises(L.LnbnnError):
            L.lnbnn_build_index(R, lab, 1, mask)
    with pytest.raises(L.LnbnnError):
        L.lnbnn_build_index(R.astype(np.float32), lab, 1, L.LNBNN_MODE_BIT(L.LNBNN_FP8_RERANK))
    with pytest.raises(L.LnbnnError):
        L.lnbnn_build_index(np.zeros((64, 144), np.uint8), lab, 1, BIT)
    ix = L.lnbnn_build_index(R, lab, 1, BIT)
    try:
        with pytest.raises(L.LnbnnError):     # 128-byte queries against 160-byte rows
            L.lnbnn_classify(ix, np.zeros((3, 128), np.uint8), np.array([0, 3], np.int64), 5, I8)
    finally:
        ix.free()


def test_loc_serving_matches_classify(small):
    cfg, R, labels, Q, off, ix, ref = small
    tickets = []
    for m in (0, 3, 9):
        s, e = int(off[m]), int(off[m + 1])
        tickets.append((m, L.lnbnn_submit(ix, Q[s:e], 10, I8)))
    for m, t in tickets:
        res, t0 = None, time.time()
        while res is None and time.time() - t0 < 60:
            res = L.lnbnn_poll(ix, t)
            if res is None:
                time.sleep(0.001)
        assert res is not None, f"request for image {m} did not finish"
        cls, tot, _ = res
        assert cls == ref[10][1][m] and np.array_equal(tot, ref[10][0][m])


@pytest.mark.timeout(600)
def test_loc_mid_size_sampled():
    """900,000 references (40 classes x 15 x 1500) and 40 images: every list
    is in (distance, index) order with its exact squared distances, the totals
    follow from the lists by Algorithm 2's update, and 64 sampled descriptors'
    lists plus one whole image equal the oracle's."""
    cfg = synth.scaled(synth.CONFIGS["M"], n_classes=40, n_img=40, q_lo=300, q_hi=3000)
    R, labels = synth.gen_index(cfg, loc=True)
    Q, off, _ = synth.gen_queries(cfg, loc=True)
    _say(f"loc mid: {R.shape[0]} refs, {Q.shape[0]} queries")
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, BIT)
    try:
        cls, tot, ni, nd = L.lnbnn_classify(ix, Q, off, 10, I8, want_neighbours=True)
    finally:
        ix.free()
    dd, di = np.diff(nd, axis=1), np.diff(ni.astype(np.int64), axis=1)
    assert np.all((dd > 0) | ((dd == 0) & (di > 0)))
    d = np.sum((R[ni].astype(np.int32) - Q[:, None, :].astype(np.int32)) ** 2, axis=2)
    assert np.array_equal(d, nd.astype(np.int64))
    # Algorithm 2's update re-derived from the returned lists
    k = 10
    lab = labels[ni[:, :k]]
    delta = nd[:, :k].astype(np.int64) - nd[:, k:k + 1].astype(np.int64)
    first = np.ones_like(lab, bool)
    for j in range(1, k):
        first[:, j] = np.all(lab[:, :j] != lab[:, j:j + 1], axis=1)
    img = np.repeat(np.arange(len(off) - 1), np.diff(off))
    T = np.zeros_like(tot)
    np.add.at(T, (np.repeat(img, k)[first.ravel()], lab.ravel()[first.ravel()]), delta.ravel()[first.ravel()])
    assert np.array_equal(T, tot) and np.array_equal(np.argmin(tot, axis=1), cls)
    sel = np.concatenate([np.arange(off[m], off[m] + 16) for m in (0, 13, 27, 39)])
    wi, wd = oracle.knn_expanded(Q[sel], R, 11)
    assert np.array_equal(ni[sel], wi) and np.array_equal(nd[sel].astype(np.int64), wd)
    m = int(np.argmin(np.diff(off)))
    s, e = int(off[m]), int(off[m + 1])
    _say(f"loc mid: oracle classification of image {m} ({e - s} descriptors)")
    wt, wc, _, _ = oracle.classify(Q[s:e], R, labels, cfg.n_classes, np.array([0, e - s]), 10)
    assert np.array_equal(tot[m], wt[0]) and cls[m] == wc[0]
