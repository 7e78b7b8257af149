"""Pins for the FP8 candidate model (oracle/fp8.py), no GPU: the e4m3
rounding against the format's own table of values (decoded bit by bit from
the code definition, independent of the rounding formula), the scale rule
by brute force, and the candidate keys against exact arithmetic."""
import numpy as np
import pytest

from oracle import fp8


def _table():
    """Every finite non-negative OCP e4m3 value, in code order: code bits
    eeee.mmm (bias 7), exponent field 0 is subnormal, code 0x7f is NaN."""
    vals = []
    for code in range(0x7F):
        e, m = code >> 3, code & 7
        vals.append(m * 2.0 ** -9 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


def test_table_is_the_e4m3_range():
    t = _table()
    assert np.all(np.diff(t) > 0)
    assert t[0] == 0.0 and t[1] == 2.0 ** -9 and t[-1] == 448.0 and len(t) == 127


def test_representable_values_are_fixed_points():
    t = _table()
    assert np.array_equal(fp8.e4m3_round(t), t)
    assert np.array_equal(fp8.e4m3_round(-t), -t)


def test_ties_go_to_the_even_code():
    t = _table()
    mid = (t[:-1] + t[1:]) / 2                    # exact in float64
    got = fp8.e4m3_round(mid)
    want = np.where(np.arange(len(mid)) % 2 == 0, t[:-1], t[1:])   # even code wins
    assert np.array_equal(got, want)
    assert np.array_equal(fp8.e4m3_round(-mid), -want)


def test_nearest_value_brute_force():
    t = _table()
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(0, 450, 5000), np.exp(rng.uniform(np.log(1e-4), np.log(400), 5000))])
    got = fp8.e4m3_round(x)
    d = np.abs(x[:, None] - t[None, :])
    best = t[np.argmin(d, axis=1)]               # no exact ties among random draws
    assert np.array_equal(got, best)


def test_saturation():
    assert np.array_equal(fp8.e4m3_round([448.0, 460.0, 464.0, 1e6, -1e6]), [448.0, 448.0, 448.0, 448.0, -448.0])


def test_scale_exponent_brute_force():
    rng = np.random.default_rng(1)
    m = np.concatenate([np.exp(rng.uniform(-20, 20, 300)), [448.0, 224.0, 1.0, 0.875, 1.75, 2.0 ** -30]])
    e = fp8.scale_exponent(m)
    for v, ev in zip(m, e):
        cands = [k for k in range(-130, 131) if np.ldexp(v, k) <= 448.0]
        assert ev == max(-120, min(120, max(cands)))
    assert fp8.scale_exponent(np.array([0.0]))[0] == 0


def test_keys_exact_for_representable_data():
    """Rows whose scaled values are e4m3 values already: the keys are the
    exact expanded form ||r||^2 - 2 q.r of the original data."""
    rng = np.random.default_rng(2)
    t = _table()[:96]                            # values up to 15
    R = rng.choice(t, size=(40, 16)) * 2.0 ** -5
    Q = rng.choice(t, size=(7, 16)) * 2.0 ** -3
    R[:, 0] = t[95] * 2.0 ** -5                  # a fixed row maximum: scaling stays exact
    Q[:, 0] = t[95] * 2.0 ** -3
    K = fp8.keys(Q, R)
    want = np.sum(R * R, axis=1)[None, :] - 2.0 * Q @ R.T
    assert np.array_equal(K, want)


def test_keys_against_per_pair_definition():
    rng = np.random.default_rng(3)
    R = np.maximum(rng.standard_normal((30, 128)), 0).astype(np.float32)
    Q = np.maximum(rng.standard_normal((5, 128)), 0).astype(np.float32)
    t = _table()
    K = fp8.keys(Q, R)

    def deq(row):
        e = fp8.scale_exponent(np.array([np.abs(row).max()]))[0]
        s = np.abs(row.astype(np.float64)) * 2.0 ** e
        near = t[np.argmin(np.abs(s[:, None] - t[None, :]), axis=1)]
        return np.sign(row) * near * 2.0 ** -e

    for i in range(5):
        q = deq(Q[i])
        for j in range(30):
            r = deq(R[j])
            assert abs(K[i, j] - (r @ r - 2 * q @ r)) <= 1e-12
    idx, _ = fp8.candidates(Q, R, 6)
    for i in range(5):
        assert idx[i].tolist() == np.lexsort((np.arange(30), K[i]))[:6].tolist()
