"""Full-size checks at the benchmarked workloads, in the launch configuration
the benchmark times (device pointers, one batched launch sequence, the tile
variant and chunk walk the committed tuning cache pins for the workload).

Exact path, 15.36M references, 512 query images, k = 10 (INT8 mode):
  * every returned neighbour carries its exact squared distance and every
    list is in (distance, index) order (all 1.16M query descriptors);
  * the image totals and classes follow from the returned lists by
    Algorithm 2's update (re-derived here, all 512 images);
  * 16 stored whole images (every 32nd) equal the oracle's results at
    k = 5, 10 and 20 (totals, classes, list digests), in INT8 and FP16, and
    their original-NBNN totals (Algorithm 1) too;
  * sampled descriptors' neighbour lists and one whole image's totals and
    class equal the oracle's computed here.
FP8 + re-rank, float descriptors of the same shape:
  * every returned distance is the FP32 direct-form distance within the
    rounding bound, lists in (distance, index) order;
  * 64 stored whole images against the FP64 oracle: recall, identical
    lists, decisions (all must agree for the top-4k rule) and totals within
    the rounding bound wherever the lists match, for both candidate rules.
Location-augmented rows (160 bytes), INT8 mode, L's sizes: the same three
exact checks as the 128-byte exact path.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import oracle_fixtures as F  # noqa: E402
from test_gpu_fixtures import compare_exact  # noqa: E402

pytestmark = pytest.mark.gpu
GAMMA = 130 * 2.0 ** -24
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1112_0059_amd", "tuning_cache.json")


def _bench_launch(ix, dq, off, k, mode):
    """Pin the tuned launch the benchmark uses (a cache hit times nothing)."""
    v = L.lnbnn_autotune(ix, dq, off, k, mode, cache_path=CACHE)
    _say(f"launch configuration: variant {L.lnbnn_variant_name(v)}")
    return v


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sorted_lists(ni, nd):
    dd, di = np.diff(nd, axis=1), np.diff(ni.astype(np.int64), axis=1)
    return np.all((dd > 0) | ((dd == 0) & (di > 0)))


def _totals_from_lists(ni, nd, labels, n_classes, off, k):
    """Algorithm 2's update from given neighbour lists (numpy, exact int64):
    each class met among the first k, at its first occurrence, adds its
    distance minus the (k+1)-th."""
    n_img = len(off) - 1
    lab = labels[ni[:, :k]]                                      # [n, k]
    d = nd.astype(np.int64)
    delta = d[:, :k] - d[:, k:k + 1]
    first = np.ones_like(lab, bool)
    for j in range(1, k):
        first[:, j] = np.all(lab[:, :j] != lab[:, j:j + 1], axis=1)
    img = np.repeat(np.arange(n_img), np.diff(off))
    T = np.zeros((n_img, n_classes), np.int64)
    rows = np.repeat(img, k)[first.ravel()]
    np.add.at(T, (rows, lab.ravel()[first.ravel()]), delta.ravel()[first.ravel()])
    return T


@pytest.fixture(scope="module")
def big():
    import torch
    cfg = synth.CONFIGS["L"]
    _say("generating the 15.36M-reference index")
    R, labels = synth.gen_index(cfg)
    Q, off, true_cls = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(L.LNBNN_EXACT_I8))
    dq = torch.from_numpy(Q).cuda()
    _bench_launch(ix, dq, off, 10, L.LNBNN_EXACT_I8)
    _say("classifying 512 images")
    cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_EXACT_I8, want_neighbours=True)
    torch.cuda.synchronize()
    got = (cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy())
    yield cfg, R, labels, Q, off, ix, got
    ix.free()


@pytest.mark.timeout(900)
def test_full_exact_lists_are_exact_distances(big):
    cfg, R, labels, Q, off, ix, (cls, tot, ni, nd) = big
    k = 10
    assert ni.shape == (Q.shape[0], k + 1) and ni.min() >= 0 and ni.max() < cfg.n_refs
    assert _sorted_lists(ni, nd)
    _say("recomputing 12.7M neighbour distances")
    for s in range(0, Q.shape[0], 1 << 16):
        q = Q[s:s + (1 << 16)].astype(np.int32)
        r = R[ni[s:s + (1 << 16)]].astype(np.int32)              # [b, k+1, 128]
        d = np.sum((r - q[:, None, :]) ** 2, axis=2)
        assert np.array_equal(d, nd[s:s + (1 << 16)].astype(np.int64)), s


@pytest.mark.timeout(900)
def test_full_exact_totals_follow_from_lists(big):
    cfg, R, labels, Q, off, ix, (cls, tot, ni, nd) = big
    T = _totals_from_lists(ni, nd, labels, cfg.n_classes, off, 10)
    assert np.array_equal(T, tot)
    assert np.all(tot <= 0)
    best = np.argmin(tot, axis=1)                               # lowest class on ties
    assert np.array_equal(best, cls)


@pytest.mark.timeout(900)
def test_full_exact_sampled_against_oracle(big):
    """64 sampled descriptors (4 images x 16) and the smallest whole image."""
    cfg, R, labels, Q, off, ix, (cls, tot, ni, nd) = big
    imgs = [3, 200, 377, 511]
    sel = np.concatenate([np.arange(off[m], off[m] + 16) for m in imgs])
    _say("oracle kNN for 64 sampled descriptors")
    wi, wd = oracle.knn_expanded(Q[sel], R, 11)
    assert np.array_equal(ni[sel], wi) and np.array_equal(nd[sel].astype(np.int64), wd)
    m = int(np.argmin(np.diff(off)))
    s, e = int(off[m]), int(off[m + 1])
    _say(f"oracle classification of image {m} ({e - s} descriptors)")
    wt, wc, wi, wd = oracle.classify(Q[s:e], R, labels, cfg.n_classes, np.array([0, e - s]), 10)
    assert np.array_equal(ni[s:e], wi)
    assert np.array_equal(tot[m], wt[0]) and cls[m] == wc[0]


def _fixture_rows(fx, off):
    """The fixture's images inside the full batch: (image ids, their CSR
    offsets in the batch's descriptor order, row index map)."""
    imgs = fx["images"]
    rows = np.concatenate([np.arange(off[m], off[m + 1]) for m in imgs])
    assert np.array_equal(np.diff(fx["offsets"]), np.diff(off)[imgs])
    return imgs, rows


@pytest.mark.timeout(900)
def test_full_exact_whole_images_against_stored_oracle(big):
    """The 16 stored whole images (every 32nd) of the benchmarked batch:
    totals, classes, list digests and sampled lists equal the oracle's."""
    fx = F.load("L")
    if fx is None:
        pytest.skip("oracle_L.npz has not been written")
    cfg, R, labels, Q, off, ix, (cls, tot, ni, nd) = big
    imgs, rows = _fixture_rows(fx, off)
    compare_exact(fx, fx["offsets"], 10, cls[imgs], tot[imgs], ni[rows], nd[rows], "INT8 L k 10")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("k", [5, 20])
def test_full_exact_other_k_sampled(big, k):
    """The other neighbourhood sizes of the large configuration: 64 sampled
    descriptors' lists and one whole image's totals, in the batched launch."""
    import torch
    cfg, R, labels, Q, off, ix, _ = big
    dq = torch.from_numpy(Q).cuda()
    _say(f"classifying 512 images at k={k}")
    cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, k, L.LNBNN_EXACT_I8, want_neighbours=True)
    torch.cuda.synchronize()
    cls, tot, ni, nd = cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy()
    assert _sorted_lists(ni, nd)
    T = _totals_from_lists(ni, nd, labels, cfg.n_classes, off, k)
    assert np.array_equal(T, tot) and np.array_equal(np.argmin(tot, axis=1), cls)
    fx = F.load("L")
    if fx is not None:
        _say(f"16 stored whole images at k={k}")
        imgs, rows = _fixture_rows(fx, off)
        compare_exact(fx, fx["offsets"], k, cls[imgs], tot[imgs], ni[rows], nd[rows], f"INT8 L k {k}")
    imgs = [7, 300]
    sel = np.concatenate([np.arange(off[m], off[m] + 32) for m in imgs])
    wi, wd = oracle.knn_expanded(Q[sel], R, k + 1)
    assert np.array_equal(ni[sel], wi) and np.array_equal(nd[sel].astype(np.int64), wd)


@pytest.mark.timeout(900)
def test_full_f16_and_nbnn_whole_images_against_stored_oracle(big):
    """FP16 at the benchmarked size (all 512 images in one batch, k = 10),
    and the original NBNN rule on the same batch: the 16 stored whole images
    equal the oracle's (FP16: totals, classes, list digests, sampled lists;
    NBNN: Algorithm 1's totals and classes)."""
    import torch
    fx = F.load("L")
    if fx is None:
        pytest.skip("oracle_L.npz has not been written")
    cfg, R, labels, Q, off, _, _ = big
    imgs, rows = _fixture_rows(fx, off)
    dq = torch.from_numpy(Q).cuda()
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes,
                             L.LNBNN_MODE_BIT(L.LNBNN_EXACT_F16) | L.LNBNN_MODE_BIT(L.LNBNN_NBNN_I8))
    try:
        _bench_launch(ix, dq, off, 10, L.LNBNN_EXACT_F16)
        _say("FP16: classifying 512 images")
        cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_EXACT_F16, want_neighbours=True)
        torch.cuda.synchronize()
        cls, tot, ni, nd = cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy()
        compare_exact(fx, fx["offsets"], 10, cls[imgs], tot[imgs], ni[rows], nd[rows], "FP16 L k 10")
        del ni, nd
        _say("original NBNN: classifying 512 images")
        cls, tot, _, _ = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_NBNN_I8)
        torch.cuda.synchronize()
        assert np.array_equal(tot.cpu().numpy()[imgs], fx["nbnn_totals"])
        assert np.array_equal(cls.cpu().numpy()[imgs], fx["nbnn_classes"])
    finally:
        ix.free()


@pytest.fixture(scope="module")
def bigf():
    import torch
    cfg = synth.CONFIGS["P"]
    _say("generating the 15.36M-reference float index")
    R, labels = synth.gen_index(cfg)
    Q, off, true_cls = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes,
                             L.LNBNN_MODE_BIT(L.LNBNN_FP8_RERANK) | L.LNBNN_MODE_BIT(L.LNBNN_FP8_RERANK_2K))
    dq = torch.from_numpy(Q).cuda()
    _bench_launch(ix, dq, off, 10, L.LNBNN_FP8_RERANK)
    _say("classifying 512 float images")
    cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_FP8_RERANK, want_neighbours=True)
    torch.cuda.synchronize()
    got = (cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy())
    yield cfg, R, labels, Q, off, ix, got, true_cls
    ix.free()


@pytest.mark.timeout(900)
def test_full_fp8_distances_and_order(bigf):
    cfg, R, labels, Q, off, ix, (cls, tot, ni, nd), true_cls = bigf
    assert ni.min() >= 0 and ni.max() < cfg.n_refs
    assert _sorted_lists(ni, nd)
    _say("recomputing float neighbour distances")
    for s in range(0, Q.shape[0], 1 << 15):
        q = Q[s:s + (1 << 15)].astype(np.float64)
        r = R[ni[s:s + (1 << 15)]].astype(np.float64)
        d = np.sum((r - q[:, None, :]) ** 2, axis=2)
        assert np.all(np.abs(nd[s:s + (1 << 15)] - d) <= GAMMA * d + 1e-30), s
    # statistic, not a pin: the synthetic images' true classes
    _say(f"accuracy (statistic) {np.mean(cls == true_cls):.4f}")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [L.LNBNN_FP8_RERANK, L.LNBNN_FP8_RERANK_2K])
def test_full_fp8_whole_images_against_stored_oracle(bigf, mode):
    """64 whole images (every 8th of the batch) against stored FP64 oracle
    results: neighbour recall, identical lists, decisions and score error.
    Decisions must all agree for the top-4k rule (the 99.9 % target at this
    size); wherever an image's lists all equal the oracle's, its totals must
    lie within the FP32 re-rank's rounding bound of the FP64 totals."""
    import torch
    fx = F.load("P")
    if fx is None:
        pytest.skip("oracle_P.npz has not been written")
    cfg, R, labels, Q, off, ix, got, true_cls = bigf
    imgs, rows = _fixture_rows(fx, off)
    dq = torch.from_numpy(Q).cuda()
    L.lnbnn_autotune(ix, dq, off, 10, mode, cache_path=CACHE)
    cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, 10, mode, want_neighbours=True)
    torch.cuda.synchronize()
    cls, tot = cls.cpu().numpy()[imgs], tot.cpu().numpy()[imgs]
    ni, nd = ni.cpu().numpy()[rows], nd.cpu().numpy()[rows]
    wi, wt, wc = fx["nbr_idx"], fx["totals_k10"], fx["classes_k10"]
    hits = (ni[:, :, None] == wi[:, None, :]).any(axis=2).sum(axis=1)
    same = np.all(ni == wi, axis=1)
    err = np.abs(tot - wt).max(axis=1) / np.abs(wt).max(axis=1)
    agree = int(np.sum(cls == wc))
    _say(f"mode {mode}: {rows.size} descriptors of {len(imgs)} images: recall {hits.mean() / 11:.6f}, "
         f"identical lists {same.mean():.5f}, decisions {agree}/{len(imgs)}, max score error {err.max():.3e}")
    sub = fx["offsets"]
    bounds = 0
    for j in range(len(imgs)):
        a, b = int(sub[j]), int(sub[j + 1])
        if not np.all(same[a:b]):
            continue
        bounds += 1
        lab = labels[wi[a:b, :10]]
        d64 = np.sum((R[wi[a:b]].astype(np.float64) - Q[rows[a:b]].astype(np.float64)[:, None, :]) ** 2, axis=2)
        B = np.zeros(cfg.n_classes)
        for i in range(b - a):
            seen = set()
            for r in range(10):
                c = int(lab[i, r])
                if c not in seen:
                    seen.add(c)
                    B[c] += GAMMA * (d64[i, r] + d64[i, 10])
        assert np.all(np.abs(tot[j] - wt[j]) <= B + 1e-12), f"image {imgs[j]}: totals outside the rounding bound"
    _say(f"images whose lists all equal the oracle's (totals within the bound): {bounds}/{len(imgs)}")
    if mode == L.LNBNN_FP8_RERANK:
        assert agree == len(imgs)


@pytest.fixture(scope="module")
def bigloc():
    import torch
    cfg = synth.CONFIGS["L"]
    _say("generating the 15.36M x 160 location-augmented index")
    R, labels = synth.gen_index(cfg, loc=True)
    Q, off, _ = synth.gen_queries(cfg, loc=True)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(L.LNBNN_EXACT_I8))
    dq = torch.from_numpy(Q).cuda()
    _bench_launch(ix, dq, off, 10, L.LNBNN_EXACT_I8)
    _say("classifying 512 location-augmented images")
    cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_EXACT_I8, want_neighbours=True)
    torch.cuda.synchronize()
    got = (cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy())
    yield cfg, R, labels, Q, off, got
    ix.free()


@pytest.mark.timeout(900)
def test_full_loc_exact(bigloc):
    """Every list holds exact 160-element squared distances in (distance,
    index) order, the totals and classes follow from the lists, and 64
    sampled descriptors plus the smallest whole image equal the oracle."""
    cfg, R, labels, Q, off, (cls, tot, ni, nd) = bigloc
    assert ni.shape == (Q.shape[0], 11) and ni.min() >= 0 and ni.max() < cfg.n_refs
    assert _sorted_lists(ni, nd)
    _say("recomputing 12.7M neighbour distances over 160 elements")
    for s in range(0, Q.shape[0], 1 << 15):
        q = Q[s:s + (1 << 15)].astype(np.int32)
        r = R[ni[s:s + (1 << 15)]].astype(np.int32)
        d = np.sum((r - q[:, None, :]) ** 2, axis=2)
        assert np.array_equal(d, nd[s:s + (1 << 15)].astype(np.int64)), s
    T = _totals_from_lists(ni, nd, labels, cfg.n_classes, off, 10)
    assert np.array_equal(T, tot) and np.array_equal(np.argmin(tot, axis=1), cls)
    imgs = [3, 200, 377, 511]
    sel = np.concatenate([np.arange(off[m], off[m] + 16) for m in imgs])
    _say("oracle kNN for 64 sampled location-augmented descriptors")
    wi, wd = oracle.knn_expanded(Q[sel], R, 11)
    assert np.array_equal(ni[sel], wi) and np.array_equal(nd[sel].astype(np.int64), wd)
    m = int(np.argmin(np.diff(off)))
    s, e = int(off[m]), int(off[m + 1])
    _say(f"oracle classification of image {m} ({e - s} descriptors)")
    wt, wc, _, _ = oracle.classify(Q[s:e], R, labels, cfg.n_classes, np.array([0, e - s]), 10)
    assert np.array_equal(tot[m], wt[0]) and cls[m] == wc[0]
