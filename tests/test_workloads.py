"""Pins of the input generators (codes, DEMs, observables) against the paper's tables."""
import os

import numpy as np
import pytest

from paper_2607_27644_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "zsz_lp_tables.txt")


def _table():
    rows = {}
    for ln in open(GOLD):
        if ln.startswith("#") or not ln.strip():
            continue
        f = ln.split()
        rows[f[0]] = [None if x == "-" else int(x) for x in f[1:]]
    return rows


TABLE = _table()


def cycles_4_6(H: np.ndarray):
    """Exact counts of simple 4- and 6-cycles of a Tanner graph (check-pair
    overlaps; inclusion-exclusion over triples of checks)."""
    A = H.astype(np.int64)
    P = A @ A.T
    m = A.shape[0]
    iu = np.triu_indices(m, 1)
    c4 = int((P[iu] * (P[iu] - 1) // 2).sum())
    total = 0
    for c1 in range(m):
        nb = np.flatnonzero(A[c1])
        S = A[:, nb]
        T = S @ S.T  # |N(c1) & N(c2) & N(c3)|
        p1 = P[c1]
        cnt = np.outer(p1, p1) * P - T * (P + p1[:, None] + p1[None, :]) + 2 * T
        mask = np.ones(m, bool)
        mask[c1] = False
        sub = cnt[np.ix_(mask, mask)]
        total += int(sub.sum() - np.trace(sub))
    return c4, total // 6


def center_size(G: W.ZSZGroup) -> int:
    gens = [(1, 0), (0, 1)]
    return sum(all(G.mul(G.element(i), g) == G.mul(g, G.element(i)) for g in gens) for i in range(G.order))


def order_counts(G: W.ZSZGroup):
    cnt = {2: 0, 3: 0}
    for i in range(G.order):
        g = G.element(i)
        h, o = g, 1
        while h != (0, 0):
            h, o = G.mul(h, g), o + 1
        if o in cnt:
            cnt[o] += 1
    return cnt[2], cnt[3]


@pytest.mark.parametrize("name", list(W.ZSZ_LP_CODES))
def test_code_dimension_and_weights(name):
    c = W.zsz_lp(name)
    n, k = TABLE[name][:2]
    assert c.n == n
    assert not ((c.HX.astype(int) @ c.HZ.T.astype(int)) % 2).any()
    assert c.k() == k
    assert set(c.HX.sum(1)) == {9} and set(c.HZ.sum(1)) == {9}
    assert set(c.HX.sum(0)) <= {3, 6} and set(c.HZ.sum(0)) <= {3, 6}


@pytest.mark.parametrize("name", ["ZSZ-LP-160", "ZSZ-LP-240", "ZSZ-LP-320", "ZSZ-LP-390", "ZSZ-LP-550",
                                  "ZSZ-LP-775"])
def test_group_and_cycle_tables(name):
    l1, l2, q = W.ZSZ_LP_CODES[name][:3]
    G = W.ZSZGroup(l1, l2, q)
    _, _, c4, c6, cen, nu2, nu3 = TABLE[name]
    assert center_size(G) == cen
    assert order_counts(G) == (nu2, nu3)
    c = W.zsz_lp(name)
    x4, x6 = cycles_4_6(c.HX)
    z4, z6 = cycles_4_6(c.HZ)
    assert (x4 + z4, x6 + z6) == (c4, c6)


def test_cycle_counter_on_known_graphs():
    # K_{3,3} as a Tanner graph has 9 four-cycles and 6 six-cycles
    assert cycles_4_6(np.ones((3, 3), np.uint8)) == (9, 6)
    # a single 6-cycle
    H = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 1]], np.uint8)
    assert cycles_4_6(H) == (0, 1)


def test_regular_representations_commute():
    G = W.ZSZGroup(16, 2, 9)
    a, b, c, d = W.ZSZ_LP_CODES["ZSZ-LP-160"][3:]
    for p in (a, b):
        for r in (c, d):
            Lp, Rr = G.L(p).astype(int), G.R(r).astype(int)
            assert np.array_equal(Lp @ Rr % 2, Rr @ Lp % 2)
    x = [(1, 0)]
    y = [(0, 1)]
    # L[xy] = L[x] L[y]; R[g] R[h] = R[hg]
    Lxy = G.L([G.mul((1, 0), (0, 1))]).astype(int)
    assert np.array_equal(Lxy, G.L(x).astype(int) @ G.L(y).astype(int) % 2)
    Ryx = G.R([G.mul((0, 1), (1, 0))]).astype(int)
    assert np.array_equal(Ryx, G.R(x).astype(int) @ G.R(y).astype(int) % 2)


def test_gf2_tools():
    rng = np.random.default_rng(0)
    A = (rng.random((30, 50)) < 0.3).astype(np.uint8)
    R, piv = W.gf2_rref(A)
    # rank agrees with elimination on the transpose
    assert len(piv) == W.gf2_rank(A.T)
    K = W.gf2_nullspace(A)
    assert K.shape[0] == 50 - len(piv)
    assert not ((A.astype(int) @ K.T.astype(int)) % 2).any()


@pytest.mark.parametrize("name", ["ZSZ-LP-60", "ZSZ-LP-160", "ZSZ-LP-320"])
def test_logical_basis(name):
    c = W.zsz_lp(name)
    O = W.logical_basis(c.HX, c.HZ)
    k = c.k()
    assert O.shape == (k, c.n)
    assert not ((O.astype(int) @ c.HZ.T.astype(int)) % 2).any()
    assert W.gf2_rank(np.vstack([c.HX, O])) == W.gf2_rank(c.HX) + k


def test_phenomenological_dem_structure():
    c = W.zsz_lp("ZSZ-LP-160")
    d1 = W.phenomenological_dem(c, 1, 1e-3)
    assert np.array_equal(d1.H, c.HX)
    T = 9
    d = W.phenomenological_dem(c, T, 1e-3)
    m, n = c.HX.shape
    assert d.H.shape == (T * m, T * n + (T - 1) * m)
    assert d.nnz == 6208
    cw = d.H.sum(0)
    assert set(cw[: T * n]) == {3, 6} and set(cw[T * n:]) == {2}
    rw = d.H.sum(1)
    assert set(rw[:m]) == {10} and set(rw[-m:]) == {10} and set(rw[m:-m]) == {11}
    assert not d.O[:, T * n:].any()
    # an error repeated on one qubit in every round is seen only in round 0,
    # and flips the observables T times
    e = np.zeros(d.N, np.uint8)
    e[0] = 1
    assert ((d.H.astype(int) @ e) % 2)[:m].any() and not ((d.H.astype(int) @ e) % 2)[m:].any()


def test_named_workload_sizes():
    assert W.workload("cc160").H.shape == (64, 160)
    d = W.workload("phen160")
    assert d.H.shape == (576, 1952) and d.k == 32
    d = W.workload("phen840")
    assert d.H.shape == (4032, 13776) and d.nnz == 43680 and d.k == 168


def test_seeded_hgp():
    H1 = W.configuration_model_36(16, seed=3)
    assert set(H1.sum(0)) == {3} and set(H1.sum(1)) == {6}
    c = W.build_hgp(H1)
    assert set(c.HX.sum(1)) == {9}
    assert not ((c.HX.astype(int) @ c.HZ.T.astype(int)) % 2).any()
    r = W.gf2_rank(H1)
    assert c.k() == (16 - r) ** 2 + (8 - r) ** 2


def test_bit_packing_roundtrip():
    rng = np.random.default_rng(1)
    b = (rng.random((5, 77)) < 0.5).astype(np.uint8)
    w = W.pack_bits(b)
    assert w.shape == (5, 3) and w.dtype == np.uint32
    assert np.array_equal(W.unpack_bits(w, 77), b)
    assert int(w[0, 0]) & 1 == b[0, 0]
