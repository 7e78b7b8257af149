"""Generator checks (no GPU): determinism, layout, and that the tiny config
is a sensible classification problem for the oracle."""
import numpy as np

import oracle
import synth


def test_tiny_config_shapes_and_determinism():
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    assert R.shape == (10000, 128) and R.dtype == np.uint8
    assert labels.shape == (10000,) and labels.min() == 0 and labels.max() == 9
    assert np.all(np.bincount(labels) == 1000)
    R2, _ = synth.gen_index(cfg)
    assert np.array_equal(R, R2)
    Q, off, true_cls = synth.gen_queries(cfg)
    assert Q.shape == (4000, 128) and off.tolist() == list(range(0, 4001, 200))
    assert true_cls.tolist() == [m % 10 for m in range(20)]


def test_chunking_independent_of_threads(monkeypatch):
    cfg = synth.scaled(synth.CONFIGS["T"], n_train=40)          # > 1 chunk
    a, _ = synth.gen_index(cfg)
    monkeypatch.setattr(synth, "_threads", lambda: 1)
    b, _ = synth.gen_index(cfg)
    assert np.array_equal(a, b)


def test_query_subset_matches_full():
    cfg = synth.scaled(synth.CONFIGS["L"], n_img=40)
    Q, off, _ = synth.gen_queries(cfg)
    assert off[-1] == np.diff(off).sum() and np.diff(off).min() >= 500 and np.diff(off).max() <= 4000
    sub, soff = synth.gen_query_images(cfg, [3, 17, 39])
    want = np.concatenate([Q[off[m]:off[m + 1]] for m in (3, 17, 39)])
    assert np.array_equal(sub, want)
    assert soff[-1] == want.shape[0]


def test_float_config_is_unit_norm():
    cfg = synth.scaled(synth.CONFIGS["P"], n_classes=4, n_train=2, n_desc=50, n_img=3, q_lo=20, q_hi=30)
    R, labels = synth.gen_index(cfg)
    assert R.dtype == np.float32 and R.shape == (400, 128)
    assert np.all(R >= 0)
    assert np.allclose(np.linalg.norm(R, axis=1), 1.0, atol=1e-5)


def test_tiny_config_is_classifiable():
    """Statistic, not a target: local NBNN (oracle) recovers most query
    images' classes on the tiny config."""
    cfg = synth.CONFIGS["T"]
    R, labels = synth.gen_index(cfg)
    Q, off, true_cls = synth.gen_queries(cfg)
    _, cls, _, _ = oracle.classify(Q, R, labels, cfg.n_classes, off, cfg.k)
    assert np.mean(cls == true_cls) >= 0.8


def test_request_stream():
    t, n = synth.request_stream(500, 100.0)
    assert np.all(np.diff(t) >= 0) and t[0] == 0
    assert n.min() >= 100 and n.max() <= 8000
    assert 1200 < np.median(n) < 1800


def test_location_augmented_rows():
    """Layout of the 160-byte rows and what their distance carries: the
    descriptor part equals the plain generator's, the location part holds 16
    copies of each coordinate code (at most 205), and the squared distance
    splits into the descriptor distance plus 16 times the squared code
    differences, which approximates (alpha * 512 * dcoord)^2."""
    cfg = synth.scaled(synth.CONFIGS["T"], n_classes=4, n_train=2, n_desc=100, n_img=3, q_lo=50, q_hi=50)
    R, labels = synth.gen_index(cfg)
    RL, labels2 = synth.gen_index(cfg, loc=True)
    assert RL.shape == (R.shape[0], synth.DIM_LOC) and RL.dtype == np.uint8
    assert np.array_equal(RL[:, :128], R) and np.array_equal(labels, labels2)
    assert np.all(RL[:, 128:144] == RL[:, 128:129]) and np.all(RL[:, 144:160] == RL[:, 144:145])
    assert RL[:, 128:].max() <= 205
    QL, off, _ = synth.gen_queries(cfg, loc=True)
    Q, off2, _ = synth.gen_queries(cfg)
    assert np.array_equal(QL[:, :128], Q) and np.array_equal(off, off2)
    a, b = QL[:40].astype(np.int64), RL[:40].astype(np.int64)
    d160 = np.sum((a - b) ** 2, axis=1)
    d128 = np.sum((a[:, :128] - b[:, :128]) ** 2, axis=1)
    dc = (a[:, 128] - b[:, 128]) ** 2 + (a[:, 144] - b[:, 144]) ** 2
    assert np.array_equal(d160, d128 + 16 * dc)
    # the coding: 16 dcode^2 = (alpha * 512 * dcoord)^2 up to the rounding of
    # each code (|code - 204.8 x| <= 1/2)
    xy = np.array([[0.0, 1.0], [0.25, 0.5], [1.0, 0.0]])
    codes = synth.loc_code(xy).astype(np.int64)
    assert codes.tolist() == [[0, 205], [51, 102], [205, 0]]
    dcode = codes[0] - codes[2]
    want = (1.6 * 512 * (xy[0] - xy[2])) ** 2
    assert np.all(np.abs(16 * dcode ** 2 - want) <= 16 * (2 * np.abs(dcode) + 1))
    # prototype descriptors sit near their class's location centres
    cen = synth.loc_centres(cfg)
    assert cen.shape == (4, cfg.n_proto, 2) and cen.min() >= 0.15 and cen.max() <= 0.85
