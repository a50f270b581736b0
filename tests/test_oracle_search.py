"""Pins of the oracle's clutter-resistant distance (Sec. 3.2, Eq. 6-7) and of
the rank of the true match (Sec. 4.1 step 6c, tie rule of Sec. 4.2)."""

import os

import numpy as np
import pytest

import oracle

NB = 64
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "crd_worked_examples.txt")


def _load_golden():
    cases, cur = [], None
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = dict(name=tok[1], needle=np.zeros((NB, NB), np.uint32), haystack=np.zeros((NB, NB), np.uint32))
                cases.append(cur)
            elif tok[0] in ("needle", "haystack"):
                r, c0, c1, v = map(int, tok[1:])
                cur[tok[0]][r, c0:c1] = v
            elif tok[0] == "expect":
                cur["expect"] = (int(tok[1]), int(tok[2]))
    return cases


@pytest.mark.parametrize("case", _load_golden(), ids=lambda c: c["name"])
def test_worked_examples(case):
    n, h = case["needle"], case["haystack"]
    assert oracle.crd(n, h) == case["expect"][0]
    assert oracle.crd(h, n) == case["expect"][1]


def _split_identity(n, h):
    """CRD = |D_n|^2 - 2 <D_n, D_h> + <[D_n != 0], D_h^2> (the masked square
    expanded; exact because the mask times D_n is D_n)."""
    dn = np.diff(n.astype(np.int64), axis=-1)
    dh = np.diff(h.astype(np.int64), axis=-1)
    m = (dn != 0).astype(np.int64)
    return int((dn * dn).sum() - 2 * (dn * dh).sum() + (m * dh * dh).sum())


def _random_images(rng, k, hi=6, density=0.3):
    base = rng.integers(0, hi, size=(k, NB, NB)).astype(np.uint32)
    keep = rng.random((k, NB, NB)) < density
    return np.where(keep, base, np.roll(base, 1, axis=-1)).astype(np.uint32)


def test_listing_equals_split_identity():
    rng = np.random.default_rng(0)
    a = _random_images(rng, 20)
    b = _random_images(rng, 20)
    for i in range(20):
        assert oracle.crd(a[i], b[i]) == _split_identity(a[i], b[i])
    # large counts: still exact in int64 while |D| < 2^24 (Eq. 6 in signed arithmetic)
    big = rng.integers(0, 2 ** 24, size=(2, NB, NB)).astype(np.uint32)
    assert oracle.crd(big[0], big[1]) == _split_identity(big[0], big[1])


def test_distance_properties():
    rng = np.random.default_rng(1)
    a = _random_images(rng, 10)
    for i in range(10):
        assert oracle.crd(a[i], a[i]) == 0
        j = (i + 1) % 10
        assert oracle.crd(a[i], a[j]) >= 0
        # a constant added to a whole haystack row leaves every delta unchanged
        shift = rng.integers(0, 50, size=(NB, 1)).astype(np.uint32)
        assert oracle.crd(a[i], a[j] + shift) == oracle.crd(a[i], a[j])
    assert any(oracle.crd(a[i], a[i + 1]) != oracle.crd(a[i + 1], a[i]) for i in range(9))
    flat = np.full((NB, NB), 3, np.uint32)
    assert oracle.crd(flat, a[0]) == 0


def test_distance_matrix_matches_pairs():
    rng = np.random.default_rng(2)
    n = _random_images(rng, 5)
    h = _random_images(rng, 7)
    M = oracle.distance_matrix(n, h, nthreads=3)
    for i in range(5):
        for j in range(7):
            assert M[i, j] == _split_identity(n[i], h[j])


@pytest.mark.parametrize("seed", range(5))
def test_rank_matches_sorted_list(seed):
    """Rank = position of the true match in the ascending list of distances,
    where equal distances give the best (lowest) position."""
    rng = np.random.default_rng(seed)
    nn, nh = 12, 40
    h = _random_images(rng, nh, hi=3, density=0.1)
    h[5] = h[6]          # duplicate haystack images make ties
    h[7] = h[6]
    true = rng.integers(0, nh, nn).astype(np.uint32)
    true[0] = 6
    n = h[true].copy()
    n[1::2] = _random_images(rng, n[1::2].shape[0], hi=3, density=0.1)
    rk, ds = oracle.rank(n, h, true, nthreads=4)
    for i in range(nn):
        d = np.array([_split_identity(n[i], h[j]) for j in range(nh)])
        order = np.argsort(d, kind="stable")
        pos = int(np.nonzero(d[order] == d[true[i]])[0][0])
        assert rk[i] == pos
        assert ds[i] == d[true[i]]
        assert 0 <= rk[i] <= nh - 1
    assert rk[0] == 0


def test_needle_equal_to_haystack_has_rank_zero():
    rng = np.random.default_rng(4)
    h = _random_images(rng, 30)
    rk, ds = oracle.rank(h, h, np.arange(30, dtype=np.uint32))
    assert (rk == 0).all() and (ds == 0).all()


def test_rank_rejects_bad_index():
    h = np.zeros((3, NB, NB), np.uint32)
    with pytest.raises(ValueError):
        oracle.rank(h[:1], h, np.array([3], np.uint32))
