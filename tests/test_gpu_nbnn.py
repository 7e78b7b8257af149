"""The original NBNN rule (Algorithm 1) on the GPU, through the C ABI,
against the oracle's Algorithm 1 (per-class nearest distances, then their
sums): int64 totals and classes bit-exact.  Also the relation Sec. 5 states
between the two rules: discounting by the background distance does not
change the minimum, checked on the device's own outputs: at k = N - 1, and
wherever the k+1 neighbours cover every class, the local totals are the
NBNN totals minus the summed (k+1)-th distances, and the argmins agree."""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth

pytestmark = pytest.mark.gpu
NB = L.LNBNN_NBNN_I8
I8 = L.LNBNN_EXACT_I8
BITS = L.LNBNN_MODE_BIT(NB) | L.LNBNN_MODE_BIT(I8)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _nbnn_oracle(Q, R, labels, n_classes, off):
    D, _ = oracle.class_nn(Q, R, labels, n_classes, 1)
    return oracle.nbnn(D, off)


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, BITS)
    want = _nbnn_oracle(Q, R, labels, cfg.n_classes, off)
    yield cfg, R, labels, Q, off, ix, want
    ix.free()


def _check(got, want):
    cls, tot = got[0], got[1]
    if hasattr(cls, "cpu"):
        cls, tot = cls.cpu().numpy(), tot.cpu().numpy()
    assert np.array_equal(tot, want[0]), "NBNN totals differ"
    assert np.array_equal(cls, want[1]), "NBNN classes differ"


def test_nbnn_tiny_bit_exact(tiny):
    cfg, R, labels, Q, off, ix, want = tiny
    for flags in (0, L.LNBNN_NO_GRAPH, L.LNBNN_PER_IMAGE_LAUNCH, L.LNBNN_TIMING):
        _say(f"nbnn flags={flags}")
        _check(L.lnbnn_classify(ix, Q, off, 10, NB, flags=flags), want)


def test_nbnn_every_variant_and_chunked_walk(tiny):
    """Every kernel variant; then few workgroups with short chunks and a
    split reference set, so each class's minimum is combined over several
    flushes."""
    cfg, R, labels, Q, off, ix, want = tiny
    for v in range(L.lnbnn_num_variants()):
        try:
            L.lnbnn_set_variant(ix, NB, 10, v)
        except L.LnbnnError:
            assert v in (10, 12, 14, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27)    # other widths, formats or lists
            continue
        _say(f"nbnn variant {v}")
        _check(L.lnbnn_classify(ix, Q, off, 10, NB), want)
        L.lnbnn_set_tuning(ix, NB, 10, variant=v, chunk_tiles=8, max_workgroups=3)
        _check(L.lnbnn_classify(ix, Q, off, 10, NB), want)
    L.lnbnn_set_tuning(ix, NB, 10)


def test_nbnn_device_pointers_and_replays(tiny):
    import torch
    cfg, R, labels, Q, off, ix, want = tiny
    dq = torch.from_numpy(Q).cuda()
    out = {"class": torch.empty(cfg.n_img, dtype=torch.int32, device="cuda"),
           "totals": torch.empty((cfg.n_img, cfg.n_classes), dtype=torch.int64, device="cuda")}
    for rep in range(3):
        for t in out.values():
            t.fill_(-7)
        junk = torch.randn(1000, device="cuda").sum()
        got = L.lnbnn_classify(ix, dq, off, 10, NB, out=out)
        torch.cuda.synchronize()
        _check(got, want)
        del junk


def test_nbnn_unsorted_uneven_classes():
    """Labels in no particular order and classes of very different sizes
    (1, 255, 256, 257 references ...): the class-sorted copy pads every
    class to its own tiles."""
    rng = np.random.default_rng(11)
    sizes = [1, 255, 256, 257, 3, 600, 40]
    labels = np.concatenate([np.full(n, c, np.int32) for c, n in enumerate(sizes)])
    perm = rng.permutation(labels.shape[0])
    labels = labels[perm]
    R = rng.integers(0, 256, size=(labels.shape[0], 128)).astype(np.uint8)
    R[10] = R[500]                                   # a duplicate pair
    Q = rng.integers(0, 256, size=(230, 128)).astype(np.uint8)
    Q[5] = R[7]
    off = np.array([0, 1, 1, 100, 230], np.int64)    # with an empty image
    ix = L.lnbnn_build_index(R, labels, len(sizes), BITS)
    try:
        _check(L.lnbnn_classify(ix, Q, off, 5, NB), _nbnn_oracle(Q, R, labels, len(sizes), off))
    finally:
        ix.free()


def test_nbnn_rejects():
    R = np.zeros((50, 128), np.uint8)
    lab = np.zeros(50, np.int32)
    with pytest.raises(L.LnbnnError) as e:           # class 1 owns no reference
        L.lnbnn_build_index(R, lab, 2, L.LNBNN_MODE_BIT(NB))
    assert e.value.code == L.LNBNN_EINVAL
    with pytest.raises(L.LnbnnError):                # 160-byte rows
        L.lnbnn_build_index(np.zeros((50, 160), np.uint8), lab, 1, L.LNBNN_MODE_BIT(NB))
    ix = L.lnbnn_build_index(R, lab, 1, L.LNBNN_MODE_BIT(NB))
    try:
        with pytest.raises(L.LnbnnError):            # no neighbour lists in this mode
            L.lnbnn_classify(ix, R[:3], np.array([0, 3], np.int64), 5, NB, want_neighbours=True)
        with pytest.raises(L.LnbnnError):            # float queries
            L.lnbnn_classify(ix, R[:3].astype(np.float32), np.array([0, 3], np.int64), 5, NB)
    finally:
        ix.free()


def test_equivalence_k_full():
    """k = N - 1 on a 33-reference index: the (k+1)-th neighbour is the
    farthest reference, every class lies within it, so local NBNN's totals
    (INT8 mode) equal Algorithm 1's (NBNN mode) minus the summed largest
    distances, and the two decisions agree -- all on device outputs."""
    rng = np.random.default_rng(5)
    R = rng.integers(0, 256, size=(33, 128)).astype(np.uint8)
    labels = (np.arange(33) % 4).astype(np.int32)
    Q = rng.integers(0, 256, size=(120, 128)).astype(np.uint8)
    off = np.array([0, 7, 30, 31, 90, 120], np.int64)
    ix = L.lnbnn_build_index(R, labels, 4, BITS)
    try:
        cl, tl, ni, nd = L.lnbnn_classify(ix, Q, off, 32, I8, want_neighbours=True)
        cn, tn, _, _ = L.lnbnn_classify(ix, Q, off, 32, NB)
    finally:
        ix.free()
    dmax = nd[:, 32].astype(np.int64)
    shift = np.array([dmax[off[m]:off[m + 1]].sum() for m in range(len(off) - 1)])
    assert np.array_equal(tl, tn - shift[:, None])
    assert np.array_equal(cl, cn)
    _check((cn, tn), _nbnn_oracle(Q, R, labels, 4, off))


def test_equivalence_under_coverage():
    """Two classes sharing most descriptors (mostly background): wherever a
    descriptor's k+1 neighbours hold both classes, its local update is its
    NBNN term minus its (k+1)-th distance.  One descriptor per image, so
    the identity is checked per descriptor on device outputs."""
    cfg = synth.scaled(synth.CONFIGS["T"], n_classes=2, n_train=5, n_desc=200, f_bg=0.9,
                       n_img=300, q_lo=1, q_hi=1, index_seed=7100, query_seed=7200)
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    k = 10
    ix = L.lnbnn_build_index(R, labels, 2, BITS)
    try:
        cl, tl, ni, nd = L.lnbnn_classify(ix, Q, off, k, I8, want_neighbours=True)
        cn, tn, _, _ = L.lnbnn_classify(ix, Q, off, k, NB)
    finally:
        ix.free()
    covered = np.array([len(set(labels[ni[i]])) == 2 for i in range(Q.shape[0])])
    _say(f"descriptors whose {k + 1} neighbours cover both classes: {covered.sum()}/{covered.size}")
    assert covered.sum() >= 50
    shift = nd[:, k].astype(np.int64)
    assert np.array_equal(tl[covered], tn[covered] - shift[covered][:, None])
    assert np.array_equal(cl[covered], cn[covered])
    _check((cn, tn), _nbnn_oracle(Q, R, labels, 2, off))


def test_nbnn_serving_and_noalloc(tiny):
    """The NBNN mode through the serving loop and the allocation-free entry
    point equals the batched classify."""
    import torch
    cfg, R, labels, Q, off, ix, want = tiny
    tickets = [L.lnbnn_submit(ix, Q[off[m]:off[m + 1]], 10, NB) for m in range(cfg.n_img)]
    for m, t in enumerate(tickets):
        t0 = time.time()
        while (r := L.lnbnn_poll(ix, t)) is None:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        assert r[0] == want[1][m] and np.array_equal(r[1], want[0][m])
    dq = torch.from_numpy(Q).cuda()
    out = {"class": torch.full((cfg.n_img,), -7, dtype=torch.int32, device="cuda"),
           "totals": torch.full((cfg.n_img, cfg.n_classes), -7, dtype=torch.int64, device="cuda")}
    L.lnbnn_classify_noalloc(ix, dq, off, 10, NB, out)
    torch.cuda.synchronize()
    _check((out["class"], out["totals"]), want)
