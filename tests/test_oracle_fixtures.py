"""The stored whole-image oracle results (tests/golden/oracle_*.npz) are
what the oracle computes: one or two images of each are recomputed here
with the oracle's blocked route, Algorithm 2's scoring and Algorithm 1's
totals, and must match the file exactly (catches a stale or corrupted
fixture).  Slow-ish: each case generates its full index."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import oracle_fixtures as F  # noqa: E402

pytestmark = pytest.mark.slow


def _recompute(name, picks):
    fx = F.load(name)
    if fx is None:
        pytest.skip(f"oracle_{name}.npz has not been written")
    spec = F.SPECS[name]
    cfg = synth.CONFIGS[spec["cfg"]]
    assert fx["images"].tolist() == list(spec["images"]) and int(fx["kp"]) == spec["kp"]
    R, labels = synth.gen_index(cfg)
    off = fx["offsets"]
    for m in picks(off):
        img = int(fx["images"][m])
        Q, sub = synth.gen_query_images(cfg, [img])
        assert Q.shape[0] == off[m + 1] - off[m]
        if cfg.kind == "u8":
            idx, dist, D = oracle.knn_class_block(Q, R, labels, cfg.n_classes, spec["kp"])
            nt, nc = oracle.nbnn(D, sub)
            assert np.array_equal(nt[0], fx["nbnn_totals"][m]) and nc[0] == fx["nbnn_classes"][m]
        else:
            idx, dist = oracle.knn(Q, R, spec["kp"], route="block")
            assert np.array_equal(idx, fx["nbr_idx"][off[m]:off[m + 1]])
        for k in spec["ks"]:
            t, c = oracle.local_nbnn(idx[:, :k + 1], dist[:, :k + 1], k, labels, cfg.n_classes, sub)
            assert np.array_equal(t[0], fx[f"totals_k{k}"][m]) and c[0] == fx[f"classes_k{k}"][m]
            if cfg.kind == "u8":
                assert F.list_digest(idx[:, :k + 1], dist[:, :k + 1]) == fx[f"digest_k{k}"][m].tobytes()
        rows = fx["sample_rows"]
        sel = (rows >= off[m]) & (rows < off[m + 1])
        assert np.array_equal(dist[rows[sel] - off[m]], fx["sample_dist"][sel])


def _smallest(off):
    return [int(np.argmin(np.diff(off)))]


def test_fixture_M_is_the_oracle():
    _recompute("M", lambda off: [0, len(off) - 2])


def test_fixture_L_is_the_oracle():
    _recompute("L", _smallest)


def test_fixture_P_is_the_oracle():
    _recompute("P", _smallest)
