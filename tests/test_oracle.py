"""Pins for the CPU oracle (no GPU).

Every check here ties the oracle to something other than itself: a
hand-worked example, a second route to the same definition, the closed form
of Algorithm 2's totals, the NBNN equivalence theorem, exact rescaling
between the integer and float routes, and invariances that hold for any
correct implementation.
"""
import json
import os

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def hw(golden_dir):
    with open(os.path.join(golden_dir, "handworked_d2.json")) as f:
        return json.load(f)


def _u8(a):
    return np.asarray(a, dtype=np.uint8)


# ------------------------------------------------------------ hand-worked
def test_handworked_distances(hw):
    R, Q = _u8(hw["refs"]), _u8(hw["queries"])
    want = {0: [0, 1, 4, 18, 1, 50], 1: [2, 1, 2, 8, 1, 32], 2: [41, 32, 29, 5, 32, 1]}
    for i, row in want.items():
        got = [oracle.sqdist_u8(Q[i], R[j]) for j in range(R.shape[0])]
        assert got == row
        got = [oracle.sqdist_u8_expanded(Q[i], R[j]) for j in range(R.shape[0])]
        assert got == row


@pytest.mark.parametrize("route", ["sort", "scan", "block", "expanded"])
def test_handworked_neighbours(hw, route):
    R, Q = _u8(hw["refs"]), _u8(hw["queries"])
    for case in hw["cases"]:
        kp = case["k"] + 1
        if route == "expanded":
            idx, dist = oracle.knn_expanded(Q, R, kp)
        else:
            idx, dist = oracle.knn(Q, R, kp, route=route)
        assert idx.tolist() == case["nbr_idx"]
        assert dist.tolist() == case["nbr_dist"]


def test_handworked_local_nbnn(hw):
    R, Q = _u8(hw["refs"]), _u8(hw["queries"])
    labels = np.asarray(hw["labels"], np.int32)
    off = np.asarray(hw["offsets"], np.int64)
    for case in hw["cases"]:
        totals, cls, _, _ = oracle.classify(Q, R, labels, hw["n_classes"], off, case["k"])
        assert totals.tolist() == case["totals"]
        assert cls.tolist() == case["classes"]
        D, kth = oracle.class_nn(Q, R, labels, hw["n_classes"], case["k"])
        ct, cc = oracle.closed_form(D, kth, off)
        assert ct.tolist() == case["totals"]
        assert cc.tolist() == case["classes"]


def test_handworked_nbnn(hw):
    R, Q = _u8(hw["refs"]), _u8(hw["queries"])
    labels = np.asarray(hw["labels"], np.int32)
    off = np.asarray(hw["offsets"], np.int64)
    D, _ = oracle.class_nn(Q, R, labels, hw["nbnn_n_classes"], 1)
    totals, cls = oracle.nbnn(D, off)
    assert totals.tolist() == hw["nbnn_totals"]
    assert cls.tolist() == hw["nbnn_classes"]


# ------------------------------------------------------------ random cases
def _case(seed, n_refs=60, n_q=25, dim=8, n_classes=4, hi=4, n_img=3):
    """Small integer data with a tiny value range, so equal distances (ties)
    are frequent."""
    rng = np.random.default_rng(seed)
    R = rng.integers(0, hi, size=(n_refs, dim)).astype(np.uint8)
    Q = rng.integers(0, hi, size=(n_q, dim)).astype(np.uint8)
    labels = rng.integers(0, n_classes, size=n_refs).astype(np.int32)
    cuts = np.sort(rng.integers(0, n_q + 1, size=n_img - 1))
    off = np.concatenate([[0], cuts, [n_q]]).astype(np.int64)
    return Q, R, labels, off


def test_distance_routes_agree():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = rng.integers(0, 256, size=128).astype(np.uint8)
        b = rng.integers(0, 256, size=128).astype(np.uint8)
        assert oracle.sqdist_u8(a, b) == oracle.sqdist_u8_expanded(a, b)
    a = np.zeros(128, np.uint8)
    b = np.full(128, 255, np.uint8)
    assert oracle.sqdist_u8(a, b) == 128 * 255 * 255


@pytest.mark.parametrize("seed", range(6))
def test_knn_routes_agree(seed):
    Q, R, _, _ = _case(seed)
    for kp in (1, 2, 6, R.shape[0]):
        i1, d1 = oracle.knn(Q, R, kp, route="sort")
        i2, d2 = oracle.knn(Q, R, kp, route="scan")
        i3, d3 = oracle.knn_expanded(Q, R, kp, chunk=17)
        i4, d4 = oracle.knn(Q, R, kp, route="block")
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
        assert np.array_equal(i1, i3) and np.array_equal(d1, d3)
        assert np.array_equal(i1, i4) and np.array_equal(d1, d4)
        # lexicographic (distance, index) order within each list
        assert np.all((np.diff(d1, axis=1) > 0) | ((np.diff(d1, axis=1) == 0) & (np.diff(i1, axis=1) > 0)))


def test_knn_against_full_enumeration():
    """The kp-list equals the first kp entries of every (distance, index)
    pair listed and sorted in numpy (no oracle code involved)."""
    Q, R, _, _ = _case(11, n_refs=40, n_q=10)
    diff = Q[:, None, :].astype(np.int64) - R[None, :, :].astype(np.int64)
    full = np.sum(diff * diff, axis=2)
    for route in ("scan", "block"):
        idx, dist = oracle.knn(Q, R, 7, route=route)
        for i in range(Q.shape[0]):
            order = np.lexsort((np.arange(R.shape[0]), full[i]))[:7]
            assert idx[i].tolist() == order.tolist()
            assert dist[i].tolist() == full[i][order].tolist()


@pytest.mark.parametrize("n,N", [(1, 1), (3, 15), (4, 16), (65, 17), (130, 47), (64, 200)])
def test_block_route_ragged(n, N):
    """The blocked route's query blocks (64), query groups (4) and reference
    groups (16) end raggedly: every size still gives the scan route's
    lists, for u8 and for float data, and the per-class minima of the same
    pass are Algorithm 1's D_C(d) (numpy enumeration)."""
    rng = np.random.default_rng(n * 1000 + N)
    R = rng.integers(0, 6, size=(N, 40)).astype(np.uint8)
    Q = rng.integers(0, 6, size=(n, 40)).astype(np.uint8)
    labels = rng.integers(0, 3, size=N).astype(np.int32)
    for kp in sorted({1, min(5, N), N}):
        i1, d1 = oracle.knn(Q, R, kp, route="scan")
        i2, d2, D = oracle.knn_class_block(Q, R, labels, 4, kp)      # class 3 is empty
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
        full = np.sum((Q[:, None, :].astype(np.int64) - R[None, :, :].astype(np.int64)) ** 2, axis=2)
        for c in range(4):
            have = labels == c
            want = full[:, have].min(axis=1) if have.any() else np.full(n, np.iinfo(np.int64).max)
            assert np.array_equal(D[:, c], want)
        Rf = rng.standard_normal((N, 40)).astype(np.float32)
        Qf = rng.standard_normal((n, 40)).astype(np.float32)
        Rf[N // 2] = Rf[0]                                             # a duplicate row
        i1, d1 = oracle.knn(Qf, Rf, kp, route="scan")
        i2, d2 = oracle.knn(Qf, Rf, kp, route="block")
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


@pytest.mark.parametrize("seed", range(8))
def test_algorithm2_equals_closed_form(seed):
    Q, R, labels, off = _case(seed, n_classes=5)
    N = R.shape[0]
    for k in (1, 2, 5, N - 1):
        totals, cls, _, _ = oracle.classify(Q, R, labels, 6, off, k)   # class 5 empty
        D, kth = oracle.class_nn(Q, R, labels, 6, k)
        ct, cc = oracle.closed_form(D, kth, off)
        assert np.array_equal(totals, ct)
        assert np.array_equal(cls, cc)
        assert np.all(totals <= 0)           # every update is <= 0
        assert np.all(totals[:, 5] == 0)     # a class with no reference


@pytest.mark.parametrize("seed", range(5))
def test_nbnn_equivalence_k_full(seed):
    """k = N-1: the (k+1)-th neighbour is the farthest reference, every class
    is within it, so T_local = T_NBNN - sum_d delta_max(d) and the argmins
    of local NBNN and Algorithm 1 coincide."""
    Q, R, labels, off = _case(seed, n_classes=4)
    labels[:4] = np.arange(4)                # every class owns a reference
    N = R.shape[0]
    totals, cls, _, dist = oracle.classify(Q, R, labels, 4, off, N - 1)
    D, _ = oracle.class_nn(Q, R, labels, 4, 1)
    nt, ncls = oracle.nbnn(D, off)
    dmax = dist[:, -1]
    shift = np.array([dmax[off[m]:off[m + 1]].sum() for m in range(len(off) - 1)])
    assert np.array_equal(totals, nt - shift[:, None])
    assert np.array_equal(cls, ncls)


def test_nbnn_equivalence_under_coverage():
    """Whenever every class has a reference within the (k+1)-th distance of
    every descriptor, local NBNN and NBNN agree (Sec. 5: discounting by the
    background distance does not change the minimum)."""
    hits = 0
    for seed in range(40):
        Q, R, labels, off = _case(100 + seed, n_refs=30, n_classes=2, hi=6)
        labels[:2] = [0, 1]
        k = 6
        D, kth = oracle.class_nn(Q, R, labels, 2, k)
        if not np.all(D <= kth[:, None]):
            continue
        hits += 1
        totals, cls, _, _ = oracle.classify(Q, R, labels, 2, off, k)
        nt, ncls = oracle.nbnn(D, off)
        shift = np.array([kth[off[m]:off[m + 1]].sum() for m in range(len(off) - 1)])
        assert np.array_equal(totals, nt - shift[:, None])
        assert np.array_equal(cls, ncls)
    assert hits >= 5


def test_k1_special_case():
    """k = 1: only the nearest reference's class moves, by delta_1 - delta_2."""
    Q, R, labels, off = _case(7)
    totals, _, idx, dist = oracle.classify(Q, R, labels, 4, off, 1)
    want = np.zeros_like(totals)
    for m in range(len(off) - 1):
        for i in range(off[m], off[m + 1]):
            want[m, labels[idx[i, 0]]] += dist[i, 0] - dist[i, 1]
    assert np.array_equal(totals, want)


def test_single_class_and_empty_image():
    Q, R, _, _ = _case(3)
    labels = np.zeros(R.shape[0], np.int32)
    off = np.array([0, 0, 10, Q.shape[0]], np.int64)   # first image is empty
    totals, cls, _, _ = oracle.classify(Q, R, labels, 1, off, 3)
    assert cls.tolist() == [0, 0, 0]
    assert totals[0, 0] == 0


@pytest.mark.parametrize("seed", range(4))
def test_invariances(seed):
    Q, R, labels, off = _case(seed, n_classes=4, hi=256, dim=16)
    k = 5
    base, bcls, bidx, bdist = oracle.classify(Q, R, labels, 4, off, k)
    rng = np.random.default_rng(seed)
    # reference permutation: totals identical
    perm = rng.permutation(R.shape[0])
    t, c, _, _ = oracle.classify(Q, R[perm], labels[perm], 4, off, k)
    assert np.array_equal(t, base) and np.array_equal(c, bcls)
    # label permutation: totals permuted the same way
    pi = rng.permutation(4).astype(np.int32)
    t, _, _, _ = oracle.classify(Q, R, pi[labels], 4, off, k)
    assert np.array_equal(t[:, pi], base)
    # shift of every descriptor by one integer vector (kept in range)
    Qs, Rs = Q.astype(np.int64), R.astype(np.int64)
    lo = np.minimum(Qs.min(0), Rs.min(0))
    hi = np.maximum(Qs.max(0), Rs.max(0))
    v = rng.integers(-lo, 255 - hi + 1)
    t, c, i2, d2 = oracle.classify((Qs + v).astype(np.uint8), (Rs + v).astype(np.uint8),
                                   labels, 4, off, k)
    assert np.array_equal(t, base) and np.array_equal(i2, bidx) and np.array_equal(d2, bdist)
    # additivity: merging images sums their totals
    merged = np.array([0, Q.shape[0]], np.int64)
    t, _, _, _ = oracle.classify(Q, R, labels, 4, merged, k)
    assert np.array_equal(t[0], base.sum(0))


def test_float_routes_match_integer_routes_exactly():
    """Float descriptors that are u8 values / 8 are exact in float32 and all
    their distance arithmetic is exact in double, so the float route must
    give the same neighbours and exactly 1/64 of the integer distances and
    totals."""
    Q, R, labels, off = _case(5, n_classes=4, hi=256, dim=32)
    k = 4
    ti, ci, ii, di = oracle.classify(Q, R, labels, 4, off, k)
    Qf, Rf = Q.astype(np.float32) / 8, R.astype(np.float32) / 8
    for route in ("sort", "scan", "block"):
        tf, cf, idf, dfl = oracle.classify(Qf, Rf, labels, 4, off, k, route=route)
        assert np.array_equal(idf, ii)
        assert np.array_equal(dfl * 64, di.astype(np.float64))
        assert np.array_equal(tf * 64, ti.astype(np.float64))
        assert np.array_equal(cf, ci)
    i3, d3 = oracle.knn_expanded(Qf, Rf, k + 1, chunk=13, margin=3)
    assert np.array_equal(i3, ii) and np.array_equal(d3 * 64, di.astype(np.float64))
    a, b = Qf[0], Rf[0]
    assert oracle.sqdist_f32(a, b) * 64 == oracle.sqdist_u8(Q[0], R[0])


def test_float_routes_agree_random():
    rng = np.random.default_rng(9)
    R = rng.random((300, 128), dtype=np.float32)
    Q = rng.random((20, 128), dtype=np.float32)
    i1, d1 = oracle.knn(Q, R, 11, route="sort")
    i2, d2 = oracle.knn(Q, R, 11, route="scan")
    i3, d3 = oracle.knn_expanded(Q, R, 11, chunk=64)
    i4, d4 = oracle.knn(Q, R, 11, route="block")
    assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
    assert np.array_equal(i1, i3) and np.array_equal(d1, d3)
    assert np.array_equal(i1, i4) and np.array_equal(d1, d4)
    # the block route's distance is the direct form summed in dimension order
    for i in range(3):
        assert d4[i, 0] == oracle.sqdist_f32(Q[i], R[i4[i, 0]])


def test_expanded_route_larger():
    """The numpy route used for sampled checks at full size agrees with the
    C scan on a few thousand references of the generator's kind."""
    rng = np.random.default_rng(4)
    R = rng.integers(0, 256, size=(5000, 128)).astype(np.uint8)
    R[4000:4010] = R[10:20]                       # duplicated rows -> ties
    Q = np.concatenate([rng.integers(0, 256, size=(30, 128)).astype(np.uint8), R[10:14]])
    labels = (np.arange(5000) % 7).astype(np.int32)
    for kp in (1, 11, 33):
        i1, d1 = oracle.knn(Q, R, kp, route="scan")
        i2, d2 = oracle.knn_expanded(Q, R, kp, chunk=777)
        i3, d3, D = oracle.knn_class_block(Q, R, labels, 7, kp)
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
        assert np.array_equal(i1, i3) and np.array_equal(d1, d3)
        D2, kth = oracle.class_nn(Q, R, labels, 7, kp - 1)
        assert np.array_equal(D, D2) and np.array_equal(d3[:, -1], kth)


def test_rejects_bad_arguments():
    Q, R, labels, off = _case(0)
    with pytest.raises(ValueError):
        oracle.knn(Q, R, R.shape[0] + 1)
    with pytest.raises(ValueError):
        oracle.local_nbnn(np.zeros((Q.shape[0], 3), np.int32), np.zeros((Q.shape[0], 3), np.int64),
                          2, labels, 4, np.array([1, Q.shape[0]], np.int64))


def test_knn_160_against_full_enumeration():
    """Location-augmented width (160 elements, full u8 range): every oracle
    route equals numpy's sorted enumeration of all (distance, index) pairs."""
    rng = np.random.default_rng(21)
    R = rng.integers(0, 256, size=(50, 160)).astype(np.uint8)
    Q = rng.integers(0, 256, size=(9, 160)).astype(np.uint8)
    R[7] = R[3]                        # a duplicate reference: tie by index
    Q[2] = R[11]                       # an exact match
    diff = Q[:, None, :].astype(np.int64) - R[None, :, :].astype(np.int64)
    full = np.sum(diff * diff, axis=2)
    for route in ("scan", "sort", "block", "expanded"):
        if route == "expanded":
            idx, dist = oracle.knn_expanded(Q, R, 12, chunk=13)
        else:
            idx, dist = oracle.knn(Q, R, 12, route=route)
        for i in range(Q.shape[0]):
            order = np.lexsort((np.arange(R.shape[0]), full[i]))[:12]
            assert idx[i].tolist() == order.tolist(), route
            assert dist[i].tolist() == full[i][order].tolist(), route
