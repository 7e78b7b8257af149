"""FP8 candidate pass + exact FP32 re-rank (float descriptors) against the
oracle.

Two references.  (1) The FP8 candidate model (oracle/fp8.py: per-row
power-of-two scales, OCP e4m3 rounding, keys of the dequantised values in
float64): LNBNN_FP8_RERANK keeps exactly the model's top 4k candidates, so
wherever the model's candidate set and the k+1 nearest among it are not
within rounding of a tie, the GPU's neighbour set must be the model's --
an exact check of the candidate pass, not a quality floor.  (2) The FP64
oracle of Algorithm 2: recall and decision agreement are reported, and
wherever a descriptor's k+1 neighbours match the oracle's, its contribution
to the totals is within the rounding bound: the re-rank sums 128 FP32 terms
(q_t - r_t)^2 sequentially, so each distance carries a relative error below
GAMMA = 130 * 2^-24, and an update dist_C - dist_B is off by at most
GAMMA * (dist_C + dist_B).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth
from oracle import fp8 as fp8model

pytestmark = pytest.mark.gpu
FP8 = L.LNBNN_FP8_RERANK
FP8_2K = L.LNBNN_FP8_RERANK_2K
GAMMA = 130 * 2.0 ** -24
# bound on the GPU candidate key's error against the float64 model: FP32
# accumulation of 129 terms (seed and 128 products) in any order, twice over
KEY_TOL = 2 * 130 * 2.0 ** -24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(seed=0, n_classes=8, n_train=4, n_desc=300, n_img=16, q=(200, 400)):
    cfg = synth.scaled(synth.CONFIGS["P"], n_classes=n_classes, n_train=n_train, n_desc=n_desc,
                       n_img=n_img, q_lo=q[0], q_hi=q[1], index_seed=5000 + seed, query_seed=6000 + seed)
    R, labels = synth.gen_index(cfg)
    Q, off, true_cls = synth.gen_queries(cfg)
    return cfg, R, labels, Q, off, true_cls


def _bound_per_image(wi, wd, labels, off, k, n_classes):
    """Upper bound on |T_gpu - T_oracle| per (image, class) when the
    neighbour lists match: sum of GAMMA * (dist_C + dist_B) over updates."""
    n_img = len(off) - 1
    B = np.zeros((n_img, n_classes))
    for m in range(n_img):
        for i in range(off[m], off[m + 1]):
            seen = set()
            for j in range(k):
                c = labels[wi[i, j]]
                if c in seen:
                    continue
                seen.add(c)
                B[m, c] += GAMMA * (wd[i, j] + wd[i, k])
    return B


def model_check(Q, R, ni, nd, k, mode):
    """The GPU's neighbour sets against the FP8 candidate model.

    Per descriptor: the model's candidates are the n_cand smallest (key,
    index) pairs; the set is decided if every key inside stays below every
    key outside by more than the keys' rounding bound.  The expected
    neighbours are the k+1 candidates of smallest squared distance; decided
    if the (k+1)-th and (k+2)-th candidate distances are further apart than
    the FP32 re-rank's bound.  Where both are decided the GPU's set must be
    the model's (FP8_RERANK_2K: only where the expected neighbours lie
    among the model's top 2k, which that rule always keeps).  Returns the
    number of descriptors checked exactly."""
    n_cand = 4 * k
    cand, K = fp8model.candidates(Q, R, n_cand)
    Qd, Rd = fp8model.dequantised(Q), fp8model.dequantised(R)
    mag = (np.einsum("ij,ij->i", Rd, Rd)[None, :] + 2.0 * (np.abs(Qd) @ np.abs(Rd).T)) * KEY_TOL
    Q64, R64 = Q.astype(np.float64), R.astype(np.float64)
    checked = 0
    for i in range(Q.shape[0]):
        inside = np.zeros(R.shape[0], bool)
        inside[cand[i]] = True
        if n_cand < R.shape[0] and (K[i][inside] + mag[i][inside]).max() >= (K[i][~inside] - mag[i][~inside]).min():
            continue                                   # candidate set within rounding of a tie
        c = cand[i]
        d = np.sum((R64[c] - Q64[i][None, :]) ** 2, axis=1)
        order = np.lexsort((c, d))
        if len(c) > k + 1 and d[order[k]] * (1 + GAMMA) >= d[order[k + 1]] * (1 - GAMMA):
            continue                                   # re-rank within rounding of a tie
        want = set(c[order[:k + 1]].tolist())
        if mode == FP8_2K and not want <= set(c[:2 * k].tolist()):
            continue
        assert set(ni[i].tolist()) == want, f"descriptor {i}: {sorted(ni[i].tolist())} != {sorted(want)}"
        checked += 1
    return checked


def _compare(got, want, labels, off, k, n_classes):
    cls, tot, ni, nd = got
    wt, wc, wi, wd = want
    kp = k + 1
    recall = np.mean([len(set(ni[i]) & set(wi[i])) / kp for i in range(ni.shape[0])])
    same = np.all(ni == wi, axis=1)
    _say(f"recall against the FP64 oracle {recall:.5f}, identical lists {same.mean():.4f}")
    # distances of matching lists: FP32 re-rank within the rounding bound
    rel = np.abs(nd[same].astype(np.float64) - wd[same]) / np.maximum(wd[same], 1e-30)
    assert np.all(rel <= GAMMA), rel.max()
    # totals of images whose every list matches the oracle's
    B = _bound_per_image(wi, wd, labels, off, k, n_classes)
    n_checked = 0
    for m in range(len(off) - 1):
        if np.all(same[off[m]:off[m + 1]]):
            n_checked += 1
            assert np.all(np.abs(tot[m] - wt[m]) <= B[m] + 1e-12), m
    # decisions: must agree wherever the oracle's margin exceeds the bound
    for m in range(len(off) - 1):
        if cls[m] != wc[m]:
            margin = np.sort(wt[m])[1] - np.sort(wt[m])[0]
            assert not np.all(same[off[m]:off[m + 1]]) or margin <= 2 * B[m].max(), m
    agree = np.mean(cls == wc)
    _say(f"decision agreement {agree:.4f}, images with all lists identical {n_checked}/{len(off) - 1}")
    return recall, agree


@pytest.fixture(scope="module")
def small():
    cfg, R, labels, Q, off, true_cls = _problem()
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(FP8) | L.LNBNN_MODE_BIT(FP8_2K))
    want = {k: oracle.classify(Q, R, labels, cfg.n_classes, off, k) for k in (1, 5, 10, 16, 20, 32)}
    yield cfg, R, labels, Q, off, ix, want
    ix.free()


@pytest.mark.parametrize("k", [1, 5, 10, 16])
@pytest.mark.parametrize("mode", [FP8, FP8_2K])
def test_fp8_small_against_model_and_oracle(small, k, mode):
    cfg, R, labels, Q, off, ix, want = small
    _say(f"fp8 small mode={mode} k={k}")
    got = L.lnbnn_classify(ix, Q, off, k, mode, want_neighbours=True)
    _check_mechanics(Q, R, got, k)
    n = model_check(Q, R, got[2], got[3], k, mode)
    _say(f"descriptors decided by the FP8 model and equal to it: {n}/{Q.shape[0]}")
    assert n >= Q.shape[0] // 2 if mode == FP8 else n > 0
    _, agree = _compare(got, want[k], labels, off, k, cfg.n_classes)
    assert agree == 1.0


@pytest.mark.parametrize("k", [20, 32])
def test_fp8_small_long_lists(small, k):
    """k > 16: 64-entry lists per row half (the top 64 FP8 keys are kept);
    mechanics, and decisions against the FP64 oracle."""
    cfg, R, labels, Q, off, ix, want = small
    got = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True)
    _check_mechanics(Q, R, got, k)
    _, agree = _compare(got, want[k], labels, off, k, cfg.n_classes)
    assert agree == 1.0


@pytest.mark.parametrize("flags", [L.LNBNN_NO_GRAPH, L.LNBNN_PER_IMAGE_LAUNCH, L.LNBNN_TIMING])
def test_fp8_launch_forms_identical(small, flags):
    """Every launch form gives bit-identical results (per-image launches use
    other slice splits: results may not depend on them)."""
    cfg, R, labels, Q, off, ix, want = small
    base = L.lnbnn_classify(ix, Q, off, 10, FP8, want_neighbours=True)
    got = L.lnbnn_classify(ix, Q, off, 10, FP8, flags=flags, want_neighbours=True)
    for x, y in zip(base, got):
        assert np.array_equal(x, y)


def test_fp8_alone_equals_in_mix(small):
    """An image classified alone gives bit-for-bit the totals, class and
    neighbours it gets inside a batch."""
    cfg, R, labels, Q, off, ix, want = small
    batch = L.lnbnn_classify(ix, Q, off, 10, FP8, want_neighbours=True)
    for m in (0, 7, 15):
        s, e = off[m], off[m + 1]
        alone = L.lnbnn_classify(ix, Q[s:e], np.array([0, e - s], np.int64), 10, FP8, want_neighbours=True)
        assert alone[0][0] == batch[0][m]
        assert np.array_equal(alone[1][0], batch[1][m])
        assert np.array_equal(alone[2], batch[2][s:e]) and np.array_equal(alone[3], batch[3][s:e])


@pytest.mark.parametrize("k", [1, 5, 10, 16, 20])
def test_fp8_pair_lists_identical(small, k):
    """The pair-list variants (one candidate list per query) keep the same
    exact FP8 top 4k as the per-half lists, so every result is bit-identical
    to the default variant's, with whole-slice sweeps and with few
    workgroups walking 8-tile chunks; the union-of-halves rule refuses them."""
    cfg, R, labels, Q, off, ix, want = small
    base = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True)
    ran = 0
    for v in (16, 18, 21):
        for chunk, wg in ((0, 0), (8, 3)):
            try:
                L.lnbnn_set_tuning(ix, FP8, k, variant=v, chunk_tiles=chunk, max_workgroups=wg)
            except L.LnbnnError:
                # two waves per SIMD: lists up to 40; one wave per SIMD: lists
                # above 20
                assert ((v == 16 and 4 * k > 40) or (v == 18 and 4 * k <= 20)
                        or (v == 21 and 4 * k > 40))
                continue
            try:
                _say(f"fp8 pair lists k={k} variant {v} chunk={chunk}")
                got = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True, flags=L.LNBNN_TIMING)
                assert L.lnbnn_last_timing(ix)["tile_variant"] == v
            finally:
                L.lnbnn_set_tuning(ix, FP8, k)
            for x, y in zip(base, got):
                assert np.array_equal(x, y)
            ran += 1
    assert ran >= 2
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_set_tuning(ix, FP8_2K, k, variant=18)
    assert e.value.code == L.LNBNN_EINVAL


@pytest.mark.parametrize("k", [1, 5, 10])
def test_fp8_16x16_blocks(small, k):
    """The candidate pass on 16x16 blocks (v_mfma_scale_f32_16x16x128_f8f6f4,
    four query tiles, one 4k list per query), with and without the next-tile
    prefetch, whole-slice sweeps and few workgroups walking 8-tile chunks.
    One instruction sums all 128 products where the 32x32 form sums two
    halves, so an FP8 key may differ in its last place: the results are
    held to the candidate model and to the FP64 oracle's decisions, not
    compared bit-for-bit with the 32x32 form."""
    cfg, R, labels, Q, off, ix, want = small
    base = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True)
    for v in (25, 27):
        for chunk, wg in ((0, 0), (8, 3)):
            L.lnbnn_set_tuning(ix, FP8, k, variant=v, chunk_tiles=chunk, max_workgroups=wg)
            try:
                _say(f"fp8 16x16 blocks k={k} variant {v} chunk={chunk}")
                got = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True, flags=L.LNBNN_TIMING)
                assert L.lnbnn_last_timing(ix)["tile_variant"] == v
            finally:
                L.lnbnn_set_tuning(ix, FP8, k)
            _check_mechanics(Q, R, got, k)
            n = model_check(Q, R, got[2], got[3], k, FP8)
            same = np.all(got[2] == base[2], axis=1).mean()
            _say(f"decided by the FP8 model and equal to it: {n}/{Q.shape[0]}; lists as the 32x32 form's: {same:.4f}")
            assert n >= Q.shape[0] // 2
            _, agree = _compare(got, want[k], labels, off, k, cfg.n_classes)
            assert agree == 1.0
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_set_tuning(ix, FP8_2K, k, variant=27)
    assert e.value.code == L.LNBNN_EINVAL


@pytest.mark.parametrize("variant", [0, 8, 11, 22])
def test_fp8_2k_rule_variants_identical(small, variant):
    """The union-of-halves rule on per-half-list variants, among them the one
    without next-tile prefetch: bit-identical results, whole-slice sweeps
    and few workgroups walking 8-tile chunks."""
    cfg, R, labels, Q, off, ix, want = small
    base = L.lnbnn_classify(ix, Q, off, 10, FP8_2K, want_neighbours=True)
    for chunk, wg in ((0, 0), (8, 3)):
        L.lnbnn_set_tuning(ix, FP8_2K, 10, variant=variant, chunk_tiles=chunk, max_workgroups=wg)
        try:
            got = L.lnbnn_classify(ix, Q, off, 10, FP8_2K, want_neighbours=True)
        finally:
            L.lnbnn_set_tuning(ix, FP8_2K, 10)
        for x, y in zip(base, got):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("variant,k", [(0, 10), (6, 10), (11, 10), (12, 16), (16, 10), (18, 10), (21, 10)])
def test_fp8_variants_and_chunks(small, variant, k):
    cfg, R, labels, Q, off, ix, want = small
    base = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True)
    L.lnbnn_set_tuning(ix, FP8, k, variant=variant, chunk_tiles=8, max_workgroups=3)
    try:
        got = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True)
    finally:
        L.lnbnn_set_tuning(ix, FP8, k)
    for x, y in zip(base, got):
        assert np.array_equal(x, y)


def test_fp8_device_pointers(small):
    import torch
    cfg, R, labels, Q, off, ix, want = small
    host = L.lnbnn_classify(ix, Q, off, 5, FP8, want_neighbours=True)
    dq = torch.from_numpy(Q).cuda()
    for rep in range(3):
        got = L.lnbnn_classify(ix, dq, off, 5, FP8, want_neighbours=True)
        torch.cuda.synchronize()
        for x, y in zip(host, got):
            assert np.array_equal(x, y.cpu().numpy())


def _check_mechanics(Q, R, got, k):
    """Whatever the candidates, every returned neighbour carries its true
    distance (FP32 re-rank within GAMMA of FP64) and lists are in
    (distance, index) order."""
    _, _, ni, nd = got
    for i in range(ni.shape[0]):
        diff = R[ni[i]].astype(np.float64) - Q[i].astype(np.float64)[None, :]
        d64 = np.sum(diff * diff, axis=1)
        assert np.all(np.abs(nd[i] - d64) <= GAMMA * d64 + 1e-30), i
        ok = (np.diff(nd[i]) > 0) | ((np.diff(nd[i]) == 0) & (np.diff(ni[i]) > 0))
        assert np.all(ok), i


def test_fp8_edge_cases():
    """Ragged reference count, 4k == n_refs (every reference is a candidate,
    so the result must equal the oracle's), all-zero rows, empty images.
    Unstructured random vectors are nearly equidistant, the hardest case for
    an FP8 shortlist: there the neighbour sets are checked against the FP8
    model wherever it decides them."""
    rng = np.random.default_rng(3)
    for n_refs, k, exact in ((1000 + 7, 10, False), (40, 10, True), (12, 3, True), (128, 32, True), (100, 25, True)):
        R = np.maximum(rng.standard_normal((n_refs, 128)), 0).astype(np.float32)
        R[::17] = 0.0
        labels = rng.integers(0, 5, size=n_refs).astype(np.int32)
        Q = np.maximum(rng.standard_normal((150, 128)), 0).astype(np.float32)
        Q[3] = 0.0
        Q[10] = R[5]
        off = np.array([0, 0, 70, 150, 150], np.int64)
        _say(f"fp8 edge n_refs={n_refs} k={k}")
        want = oracle.classify(Q, R, labels, 6, off, k)
        ix = L.lnbnn_build_index(R, labels, 6, L.LNBNN_MODE_BIT(FP8))
        try:
            got = L.lnbnn_classify(ix, Q, off, k, FP8, want_neighbours=True)
        finally:
            ix.free()
        _check_mechanics(Q, R, got, k)
        recall, _ = _compare(got, want, labels, off, k, 6)
        if exact:
            assert recall == 1.0
        if k <= 16:
            _say(f"decided by the FP8 model and equal: {model_check(Q, R, got[2], got[3], k, FP8)}/{Q.shape[0]}")
        assert got[0][0] == 0 and np.all(got[1][0] == 0) and np.all(got[1][3] == 0)


def test_fp8_rejects():
    R = np.zeros((100, 128), np.float32)
    lab = np.zeros(100, np.int32)
    ix = L.lnbnn_build_index(R, lab, 1, L.LNBNN_MODE_BIT(FP8))
    try:
        with pytest.raises(L.LnbnnError):
            L.lnbnn_classify(ix, R[:3], np.array([0, 3], np.int64), 33, FP8)      # k > 32
        with pytest.raises(L.LnbnnError):
            L.lnbnn_classify(ix, R[:3], np.array([0, 3], np.int64), 26, FP8)      # 4k > n_refs
        with pytest.raises(L.LnbnnError):
            L.lnbnn_classify(ix, R[:3], np.array([0, 3], np.int64), 5, L.LNBNN_EXACT_F16)
        with pytest.raises(L.LnbnnError):
            L.lnbnn_classify(ix, R[:3].astype(np.uint8), np.array([0, 3], np.int64), 5, FP8)
    finally:
        ix.free()
    with pytest.raises(L.LnbnnError):
        L.lnbnn_build_index(R, lab, 1, L.LNBNN_MODE_BIT(L.LNBNN_EXACT_F16))
