"""The allocation-free entry point (lnbnn_classify_noalloc) against
lnbnn_classify on the same inputs: two calls in a row on one GPU's scratch
array, the second with a smaller batch, each bit-exact in the exact modes
and equal to classify in the FP8 mode; a batch too large for the array is
refused before anything runs."""
import sys

import numpy as np
import pytest

import paper_1112_0059_amd as L
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _outs(torch, n_img, n_q, kp, nc, f64):
    return {"class": torch.full((n_img,), -7, dtype=torch.int32, device="cuda"),
            "totals": torch.full((n_img, nc), -7, dtype=torch.float64 if f64 else torch.int64, device="cuda"),
            "nbr_idx": torch.full((n_q, kp), -7, dtype=torch.int32, device="cuda"),
            "nbr_dist": torch.full((n_q, kp), -7, dtype=torch.float32, device="cuda"),
            "status": torch.full((1,), 5, dtype=torch.int32, device="cuda")}


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("mode", [L.LNBNN_EXACT_I8, L.LNBNN_EXACT_F16])
def test_noalloc_equals_classify_exact(mode):
    import torch
    cfg = synth.scaled(synth.CONFIGS["T"], n_img=12, q_lo=40, q_hi=500, query_seed=2900)
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(mode))
    try:
        for imgs, k in (((0, 12), 10), ((3, 8), 5)):        # second call: a smaller batch
            s, e = int(off[imgs[0]]), int(off[imgs[1]])
            sub = (off[imgs[0]:imgs[1] + 1] - off[imgs[0]]).astype(np.int64)
            dq = torch.from_numpy(Q[s:e].copy()).cuda()
            _say(f"mode {mode}: images {imgs}, k {k}, {e - s} descriptors")
            want = L.lnbnn_classify(ix, dq, sub, k, mode, want_neighbours=True)
            out = _outs(torch, len(sub) - 1, e - s, k + 1, cfg.n_classes, False)
            L.lnbnn_classify_noalloc(ix, dq, sub, k, mode, out)
            torch.cuda.synchronize()
            got = [out[n].cpu().numpy() for n in ("class", "totals", "nbr_idx", "nbr_dist")]
            assert _same(got, [w.cpu().numpy() for w in want])
            assert int(out["status"].item()) == 0
            # without the optional outputs: class only, totals in the scratch array
            cls = torch.full((len(sub) - 1,), -7, dtype=torch.int32, device="cuda")
            L.lnbnn_classify_noalloc(ix, dq, sub, k, mode, {"class": cls})
            torch.cuda.synchronize()
            assert np.array_equal(cls.cpu().numpy(), want[0].cpu().numpy())
    finally:
        ix.free()


def test_noalloc_equals_classify_fp8():
    import torch
    FP8 = L.LNBNN_FP8_RERANK
    cfg = synth.scaled(synth.CONFIGS["P"], n_classes=6, n_train=3, n_desc=300, n_img=9, q_lo=100, q_hi=400,
                       index_seed=5200, query_seed=6200)
    R, labels = synth.gen_index(cfg)
    Q, off, _ = synth.gen_queries(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(FP8))
    try:
        for imgs in ((0, 9), (2, 5)):
            s, e = int(off[imgs[0]]), int(off[imgs[1]])
            sub = (off[imgs[0]:imgs[1] + 1] - off[imgs[0]]).astype(np.int64)
            dq = torch.from_numpy(Q[s:e].copy()).cuda()
            _say(f"fp8: images {imgs}, {e - s} descriptors")
            want = L.lnbnn_classify(ix, dq, sub, 10, FP8, flags=L.LNBNN_NO_GRAPH, want_neighbours=True)
            out = _outs(torch, len(sub) - 1, e - s, 11, cfg.n_classes, True)
            L.lnbnn_classify_noalloc(ix, dq, sub, 10, FP8, out)
            torch.cuda.synchronize()
            got = [out[n].cpu().numpy() for n in ("class", "totals", "nbr_idx", "nbr_dist")]
            assert _same(got, [w.cpu().numpy() for w in want])
    finally:
        ix.free()


def test_noalloc_refuses_oversize_batch():
    import torch
    cfg = synth.scaled(synth.CONFIGS["T"], n_img=1)
    R, labels = synth.gen_index(cfg)
    ix = L.lnbnn_build_index(R, labels, cfg.n_classes, L.LNBNN_MODE_BIT(L.LNBNN_EXACT_I8))
    try:
        # partial lists alone exceed 64 MiB: even one list of 11 entries
        # (8 bytes each) for each of 10^6 queries is 88 MB
        n = 1_000_000
        dq = torch.zeros((n, 128), dtype=torch.uint8, device="cuda")
        cls = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(L.LnbnnError) as e:
            L.lnbnn_classify_noalloc(ix, dq, np.array([0, n], np.int64), 10, L.LNBNN_EXACT_I8, {"class": cls})
        assert e.value.code == L.LNBNN_ENOMEM and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert int(cls.item()) == -7          # nothing ran
    finally:
        ix.free()
