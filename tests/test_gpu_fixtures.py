"""Whole query images at full index size against stored oracle results.

The arrays in tests/golden/oracle_*.npz come from the oracle alone (written
by tests/golden/oracle_fixtures.py from the synthetic inputs; nothing in them
comes from the GPU path).  Here the GPU classifies the same images and every
image is compared whole: the int64 totals and class of every k, a digest of
its neighbour lists (indices and squared distances of every descriptor),
and the full lists of every 8th descriptor.

Mid size (101 classes, 2.27M references): 100 images (every 10th), k = 1,
5 and 10, in each exact mode; the original NBNN rule's totals and classes
(Algorithm 1) of the same images.
"""
import os
import sys

import numpy as np
import pytest

import paper_1112_0059_amd as L
import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import oracle_fixtures as F  # noqa: E402

pytestmark = pytest.mark.gpu
EXACT = [L.LNBNN_EXACT_I8, L.LNBNN_EXACT_F16, L.LNBNN_EXACT_BF16]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_exact(fx, off, k, cls, tot, ni, nd, what):
    """Every image's totals, class and list digest, and the sampled lists."""
    assert np.array_equal(tot, fx[f"totals_k{k}"]), f"{what}: totals differ"
    assert np.array_equal(cls, fx[f"classes_k{k}"]), f"{what}: classes differ"
    d = nd.astype(np.int64)
    assert np.array_equal(d.astype(np.float32), nd), f"{what}: distances not integers"
    bad = []
    for m in range(len(off) - 1):
        a, b = int(off[m]), int(off[m + 1])
        if F.list_digest(ni[a:b], d[a:b]) != fx[f"digest_k{k}"][m].tobytes():
            bad.append(m)
    assert not bad, f"{what}: neighbour lists of images {bad[:10]} differ"
    rows = fx["sample_rows"]
    assert np.array_equal(ni[rows], fx["sample_idx"][:, :k + 1]), f"{what}: sampled lists differ"
    assert np.array_equal(d[rows], fx["sample_dist"][:, :k + 1]), f"{what}: sampled distances differ"


@pytest.fixture(scope="module")
def mid():
    import torch
    fx = F.load("M")
    if fx is None:
        pytest.skip("oracle_M.npz has not been written")
    cfg = synth.CONFIGS["M"]
    _say("generating the 2.27M-reference index and 100 query images")
    R, labels = synth.gen_index(cfg)
    Q, off = synth.gen_query_images(cfg, fx["images"])
    assert np.array_equal(off, fx["offsets"]) and int(fx["n_refs"]) == cfg.n_refs
    mask = sum(L.LNBNN_MODE_BIT(m) for m in EXACT) | L.LNBNN_MODE_BIT(L.LNBNN_NBNN_I8)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, mask)
    dq = torch.from_numpy(Q).cuda()
    yield fx, off, ix, dq
    ix.free()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", EXACT)
def test_mid_whole_images_against_oracle(mid, mode):
    import torch
    fx, off, ix, dq = mid
    for k in (1, 5, 10):
        _say(f"mode {mode}, k {k}: 100 whole images")
        cls, tot, ni, nd = L.lnbnn_classify(ix, dq, off, k, mode, want_neighbours=True)
        torch.cuda.synchronize()
        compare_exact(fx, off, k, cls.cpu().numpy(), tot.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy(),
                      f"mode {mode} k {k}")


@pytest.mark.timeout(600)
def test_mid_nbnn_whole_images_against_oracle(mid):
    import torch
    fx, off, ix, dq = mid
    _say("original NBNN: 100 whole images")
    cls, tot, _, _ = L.lnbnn_classify(ix, dq, off, 10, L.LNBNN_NBNN_I8)
    torch.cuda.synchronize()
    assert np.array_equal(tot.cpu().numpy(), fx["nbnn_totals"])
    assert np.array_equal(cls.cpu().numpy(), fx["nbnn_classes"])
