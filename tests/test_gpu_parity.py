"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Exact modes must be bit-exact: neighbour indices and squared distances, the
int64 class totals and the decisions.  Sizes span several reference tiles,
several query blocks and ragged tails; the full-size case checks sampled
descriptors one by one and one whole image.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1112_0059_amd as L
import synth

pytestmark = pytest.mark.gpu

MODES = [L.LNBNN_EXACT_F16, L.LNBNN_EXACT_BF16, L.LNBNN_EXACT_I8]
BOTH = (L.LNBNN_MODE_BIT(L.LNBNN_EXACT_F16) | L.LNBNN_MODE_BIT(L.LNBNN_EXACT_BF16) |
        L.LNBNN_MODE_BIT(L.LNBNN_EXACT_I8))
# the 16-bit form and the INT8 form (different kernels, keys and packing)
FORMS = [L.LNBNN_EXACT_F16, L.LNBNN_EXACT_I8]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, BOTH)
    ref = {}
    for k in (1, 5, 10):
        ref[k] = oracle.classify(Q, R, labels, cfg.n_classes, off, k)
    yield cfg, R, labels, Q, off, ix, ref
    ix.free()


def _check_exact(got, want, k):
    cls, tot, ni, nd = got
    wt, wc, wi, wd = want
    assert np.array_equal(ni, wi), "neighbour indices differ"
    assert np.array_equal(nd.astype(np.int64), wd), "neighbour distances differ"
    assert np.all(nd == wd.astype(np.float32))
    assert np.array_equal(tot, wt), "totals differ"
    assert np.array_equal(cls, wc), "classes differ"


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k", [1, 5, 10])
def test_tiny_bit_exact(tiny, mode, k):
    cfg, R, labels, Q, off, ix, ref = tiny
    _say(f"tiny mode={mode} k={k}")
    got = L.lnbnn_classify(ix, Q, off, k, mode, want_neighbours=True)
    _check_exact(got, ref[k], k)


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("flags", [L.LNBNN_NO_GRAPH, L.LNBNN_PER_IMAGE_LAUNCH, L.LNBNN_TIMING])
def test_tiny_launch_forms(tiny, flags, mode):
    cfg, R, labels, Q, off, ix, ref = tiny
    _say(f"tiny flags={flags} mode={mode}")
    got = L.lnbnn_classify(ix, Q, off, 10, mode, flags=flags, want_neighbours=True)
    _check_exact(got, ref[10], 10)
    if flags & L.LNBNN_TIMING:
        t = L.lnbnn_last_timing(ix)
        assert t["dist_kernel_ms"] > 0 and t["total_ms"] >= t["dist_kernel_ms"]


@pytest.mark.parametrize("mode", FORMS)
def test_tiny_every_variant(tiny, mode):
    cfg, R, labels, Q, off, ix, ref = tiny
    for v in range(L.lnbnn_num_variants()):
        _say(f"variant {v} mode={mode}")
        try:
            L.lnbnn_set_variant(ix, mode, 10, v)
        except L.LnbnnError:          # not built for this operand format
            # 8, 9: 4 KB tiles only; 10, 11: 160-element rows only
            assert (mode == L.LNBNN_EXACT_F16 and v >= 8) or v >= 10
            continue
        got = L.lnbnn_classify(ix, Q, off, 10, mode, want_neighbours=True)
        _check_exact(got, ref[10], 10)
    L.lnbnn_set_variant(ix, mode, 10, -1)


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("variant", [0, 4, 6])
def test_tiny_chunked_walk(tiny, variant, mode):
    """Few resident workgroups and short chunks: every workgroup owns several
    query blocks and saves/restores their lists between chunks."""
    cfg, R, labels, Q, off, ix, ref = tiny
    _say(f"chunked walk variant {variant} mode={mode}")
    L.lnbnn_set_tuning(ix, mode, 10, variant=variant, chunk_tiles=8, max_workgroups=3)
    try:
        got = L.lnbnn_classify(ix, Q, off, 10, mode, want_neighbours=True)
        _check_exact(got, ref[10], 10)
    finally:
        L.lnbnn_set_tuning(ix, mode, 10)


@pytest.mark.parametrize("mode", MODES)
def test_tiny_16x16_blocks(tiny, mode):
    """The variants built on 16x16 MFMA blocks (four lanes, so four lists,
    per query): every list length each is built for, with the default split
    of the reference set (up to 64 partial lists per query to merge) and
    with few workgroups walking 8-tile chunks (lists parked between chunks)."""
    cfg, R, labels, Q, off, ix, ref = tiny
    shapes = [14] if mode != L.LNBNN_EXACT_I8 else [13, 15]
    assert all(L.lnbnn_variant_name(v).startswith("q16_") for v in shapes)
    ran = 0
    for v in shapes:
        for k in (1, 5, 10):
            try:
                L.lnbnn_set_tuning(ix, mode, k, variant=v)
            except L.LnbnnError:
                assert v == 15 and k == 10          # 64 queries per wave: lists up to 6
                continue
            try:
                for chunk, wg in ((0, 0), (8, 3)):
                    _say(f"16x16 variant {v} mode={mode} k={k} chunk={chunk} workgroups={wg}")
                    L.lnbnn_set_tuning(ix, mode, k, variant=v, chunk_tiles=chunk, max_workgroups=wg)
                    got = L.lnbnn_classify(ix, Q, off, k, mode, want_neighbours=True, flags=L.LNBNN_TIMING)
                    t = L.lnbnn_last_timing(ix)
                    assert t["tile_variant"] == v and (chunk or t["slices"] > 1)
                    _check_exact(got, ref[k], k)
                    ran += 1
            finally:
                L.lnbnn_set_tuning(ix, mode, k)
    assert ran >= 6


@pytest.mark.parametrize("mode", MODES)
def test_tiny_pair_lists(tiny, mode):
    """The shared-list variants (the two lanes of a query in 32x32 blocks, or
    the four in 16x16 blocks, share one list held by one of them): every
    list length, whole-slice sweeps over a split reference set and few
    workgroups walking 8-tile chunks."""
    cfg, R, labels, Q, off, ix, ref = tiny
    # 16-bit formats: also the form with next-tile prefetch (lists up to 16)
    # 16x16 blocks with shared lists: 26 (16-bit), 25 (INT8)
    shapes = [17, 20, 23, 24, 26] if mode != L.LNBNN_EXACT_I8 else [16, 21, 25]
    assert all(L.lnbnn_variant_name(v).startswith(("pl_", "plpf_", "plnp_", "plq16_")) for v in shapes)
    for k in (1, 5, 10, 20, 32):
        want = ref[k] if k in ref else oracle.classify(Q, R, labels, cfg.n_classes, off, k)
        for v in shapes:
            try:
                for chunk, wg in ((0, 0), (8, 3)):
                    _say(f"pair lists variant {v} mode={mode} k={k} chunk={chunk} workgroups={wg}")
                    try:
                        L.lnbnn_set_tuning(ix, mode, k, variant=v, chunk_tiles=chunk, max_workgroups=wg)
                    except L.LnbnnError:
                        assert v == 20 and k > 15
                        break
                    got = L.lnbnn_classify(ix, Q, off, k, mode, want_neighbours=True, flags=L.LNBNN_TIMING)
                    t = L.lnbnn_last_timing(ix)
                    assert t["tile_variant"] == v and (chunk or t["slices"] > 1)
                    _check_exact(got, want, k)
            finally:
                L.lnbnn_set_tuning(ix, mode, k)


@pytest.mark.parametrize("mode", FORMS)
def test_device_pointers_and_graph_replays(tiny, mode):
    """Device tensors on torch's stream; the captured graph is replayed with
    eager work and synchronisations in between, and every replay matches."""
    import torch
    cfg, R, labels, Q, off, ix, ref = tiny
    dq = torch.from_numpy(Q).cuda()
    out = {"class": torch.empty(cfg.n_img, dtype=torch.int32, device="cuda"),
           "totals": torch.empty((cfg.n_img, cfg.n_classes), dtype=torch.int64, device="cuda"),
           "nbr_idx": torch.empty((Q.shape[0], 11), dtype=torch.int32, device="cuda"),
           "nbr_dist": torch.empty((Q.shape[0], 11), dtype=torch.float32, device="cuda")}
    for rep in range(4):
        _say(f"replay {rep}")
        for t in out.values():
            t.fill_(-7)
        junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
        cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, 10, mode, want_neighbours=True, out=out)
        torch.cuda.synchronize()
        _check_exact((cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy()),
                     ref[10], 10)
        del junk


def test_exact_modes_agree_tiny(tiny):
    cfg, R, labels, Q, off, ix, ref = tiny
    a = L.lnbnn_classify(ix, Q, off, 5, L.LNBNN_EXACT_F16, want_neighbours=True)
    for mode in (L.LNBNN_EXACT_BF16, L.LNBNN_EXACT_I8):
        b = L.lnbnn_classify(ix, Q, off, 5, mode, want_neighbours=True)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


# ------------------------------------------------------------- edge cases
def _rand_problem(seed, n_refs, n_q, n_img, n_classes, hi=256, dup=0):
    rng = np.random.default_rng(seed)
    R = rng.integers(0, hi, size=(n_refs, 128)).astype(np.uint8)
    if dup:
        # duplicated rows with other labels: equal distances everywhere
        src = rng.integers(0, n_refs, size=dup)
        dst = rng.integers(0, n_refs, size=dup)
        R[dst] = R[src]
    Q = rng.integers(0, hi, size=(n_q, 128)).astype(np.uint8)
    m = min(4, n_q, n_refs)
    Q[:m] = R[:m]                           # exact matches (distance 0)
    labels = rng.integers(0, n_classes, size=n_refs).astype(np.int32)
    cuts = np.sort(rng.integers(0, n_q + 1, size=max(0, n_img - 1)))
    off = np.concatenate([[0], cuts, [n_q]]).astype(np.int64)
    return R, labels, Q, off


@pytest.mark.parametrize("case", [
    # (seed, n_refs, n_q, n_img, n_classes, hi, dup, k)
    (1, 1000, 300, 3, 7, 256, 0, 10),      # ragged refs (not a multiple of 32 or 256)
    (2, 33, 50, 2, 3, 256, 0, 32),         # k + 1 == n_refs (every reference retrieved)
    (3, 2, 17, 1, 2, 256, 0, 1),           # two references
    (4, 5000, 1, 1, 5, 256, 0, 5),         # a single descriptor
    (5, 3000, 700, 9, 4, 4, 200, 10),      # tiny value range: ties everywhere
    (6, 4096, 257, 5, 300, 256, 50, 20),   # more classes than neighbours, k = 20
    (7, 20000, 2048, 40, 10, 256, 0, 7),   # many query blocks, k + 1 = 8 bucket rounding
])
@pytest.mark.parametrize("mode", MODES)
def test_edge_cases(case, mode):
    seed, n_refs, n_q, n_img, n_classes, hi, dup, k = case
    _say(f"edge case {case} mode={mode}")
    R, labels, Q, off = _rand_problem(seed, n_refs, n_q, n_img, n_classes, hi, dup)
    # empty images at both ends and in the middle
    off = np.concatenate([[0], off, [off[-1]]]).astype(np.int64)
    want = oracle.classify(Q, R, labels, n_classes + 1, off, k)    # last class owns no ref
    ix = L.lnbnn_build_index(R, labels, n_classes + 1, BOTH)
    try:
        got = L.lnbnn_classify(ix, Q, off, k, mode, want_neighbours=True)
        _check_exact(got, want, k)
        got = L.lnbnn_classify(ix, Q, off, k, mode, flags=L.LNBNN_PER_IMAGE_LAUNCH, want_neighbours=True)
        _check_exact(got, want, k)
    finally:
        ix.free()


def test_no_images_and_errors(tiny):
    cfg, R, labels, Q, off, ix, ref = tiny
    cls, tot, _, _ = L.lnbnn_classify(ix, Q[:0], np.array([0], np.int64), 10, L.LNBNN_EXACT_F16)
    assert cls.shape == (0,)
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_classify(ix, Q, off, 0, L.LNBNN_EXACT_F16)
    assert e.value.code == L.LNBNN_EINVAL
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_classify(ix, Q, off, 33, L.LNBNN_EXACT_F16)
    assert e.value.code == L.LNBNN_EINVAL
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_classify(ix, Q, off[::-1].copy(), 5, L.LNBNN_EXACT_F16)
    assert e.value.code == L.LNBNN_EINVAL
    with pytest.raises(L.LnbnnError) as e:
        L.lnbnn_classify(ix, Q.astype(np.float32), off, 5, L.LNBNN_EXACT_F16)
    assert e.value.code == L.LNBNN_EINVAL


# ----------------------------------------------------- Caltech-101-sized
@pytest.fixture(scope="module")
def mid():
    cfg = synth.CONFIGS["M"]
    _say("generating M index")
    R, labels = synth.gen_index(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, BOTH)
    yield cfg, R, labels, ix
    ix.free()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", [1, 5, 10])
def test_mid_subset_bit_exact(mid, k):
    """Four whole query images of the 2.27M-reference index against the
    oracle's expanded-form route (exact for u8 data)."""
    cfg, R, labels, ix = mid
    imgs = [0, 333, 666, 999]
    Q, off = synth.gen_query_images(cfg, imgs)
    _say(f"mid k={k} oracle")
    wi, wd = oracle.knn_expanded(Q, R, k + 1)
    wt, wc = oracle.local_nbnn(wi, wd, k, labels, cfg.n_classes, off)
    for mode in MODES:
        _say(f"mid k={k} mode={mode}")
        got = L.lnbnn_classify(ix, Q, off, k, mode, want_neighbours=True)
        _check_exact(got, (wt, wc, wi, wd), k)


@pytest.mark.timeout(600)
def test_mid_all_images_exact_modes_agree(mid):
    import torch
    cfg, R, labels, ix = mid
    Q, off, true_cls = synth.gen_queries(cfg)
    dq = torch.from_numpy(Q).cuda()
    _say("mid all images")
    a = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_EXACT_F16)
    for mode in (L.LNBNN_EXACT_BF16, L.LNBNN_EXACT_I8):
        b = L.lnbnn_classify(ix, dq, off, 10, mode)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), mode
    acc = float(np.mean(a[0].cpu().numpy() == true_cls))
    _say(f"mid accuracy (statistic) {acc:.3f}")
