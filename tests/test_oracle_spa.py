"""Pins of the sum-product / AWGN oracle (classical channel coding of the
ZSZ-2BGA codes, numerics appendix) and of the classical code tables.

The oracle is pinned to things it does not compute itself:
  * phi equals -ln tanh(x/2) (float64 numpy) and is an involution;
  * on a single check, one iteration equals the tanh rule
    2 atanh(prod tanh(L/2)) (float64), a different formula for the same update;
  * on tree-shaped Tanner graphs, sum-product is exact: after enough
    iterations the marginals equal the bitwise posterior log-ratios obtained by
    enumerating every codeword (textbook belief propagation on trees);
  * the stop rule and the codeword property of converged outputs;
  * the Box-Muller channel has the LLR mean 2/sigma^2 and variance 4/sigma^2 of
    the BPSK-AWGN model, passes a normality test and has uncorrelated bits;
  * the ZSZ-2BGA tables: (3,6)-regular, full rank (k = n/2) and the Tanner
    girths of the paper's table, for the left and right codes;
  * the BPSK-AWGN Shannon limit at rate 1/2 is about 0.19 dB (0.187 dB).
"""
import itertools

import numpy as np
import pytest
from scipy import stats as sst

import oracle
from paper_2607_27644_amd import stats, workloads as W


def test_phi_definition_and_involution():
    for x in [1e-4, 1e-2, 0.3, 1.0, 2.5, 7.0, 15.0]:
        ref = -np.log(np.tanh(x / 2.0))
        assert abs(oracle.spa_phi(x) - ref) <= 2e-6 * max(ref, 1e-30) + 1e-12, x
        assert abs(oracle.spa_phi(oracle.spa_phi(x)) - x) <= 1e-4 * x + 1e-6, x
    assert oracle.spa_phi(0.0) == np.inf
    assert oracle.spa_phi(np.inf) == 0.0


@pytest.mark.parametrize("D", [2, 3, 6, 9])
def test_single_check_matches_tanh_rule(D):
    rng = np.random.default_rng(D)
    H = np.ones((1, D), dtype=np.uint8)
    L = rng.uniform(-4, 4, size=(50, D)).astype(np.float32)
    r = oracle.spa_decode(H, L, max_iterations=1, llr_max=20.0, stop=False, marginals=True, nthreads=2)
    Ld = L.astype(np.float64)
    th = np.tanh(Ld / 2.0)
    for j in range(D):
        others = np.prod(np.delete(th, j, axis=1), axis=1)
        mu = 2.0 * np.arctanh(others)
        np.testing.assert_allclose(r["marginals"][:, j], Ld[:, j] + mu, rtol=2e-5, atol=2e-5)


def random_tree(n_checks, seed):
    """A random tree-shaped Tanner graph: each new check joins one existing
    variable and 1-3 new ones."""
    rng = np.random.default_rng(seed)
    rows, n = [], 1
    for _ in range(n_checks):
        old = int(rng.integers(0, n))
        k = int(rng.integers(1, 4))
        rows.append([old] + list(range(n, n + k)))
        n += k
    H = np.zeros((n_checks, n), dtype=np.uint8)
    for i, r in enumerate(rows):
        H[i, r] = 1
    return H


def exact_posteriors(H, L):
    """log P(c_j = 0 | y) / P(c_j = 1 | y) by enumerating all codewords."""
    M, N = H.shape
    words = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.uint8)
    code = words[((words @ H.T) % 2 == 0).all(axis=1)]
    out = np.zeros((L.shape[0], N))
    for s in range(L.shape[0]):
        lw = -(code @ L[s].astype(np.float64))  # log prob up to a constant: P(c) ~ exp(-sum c_j L_j)
        for j in range(N):
            a = np.logaddexp.reduce(lw[code[:, j] == 0])
            b = np.logaddexp.reduce(lw[code[:, j] == 1])
            out[s, j] = a - b
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tree_marginals_are_exact(seed):
    H = random_tree(5, seed)
    N = H.shape[1]
    assert N <= 16
    rng = np.random.default_rng(100 + seed)
    L = rng.uniform(-2.0, 2.0, size=(20, N)).astype(np.float32)
    r = oracle.spa_decode(H, L, max_iterations=2 * N, llr_max=20.0, stop=False, marginals=True, nthreads=2)
    ref = exact_posteriors(H, L)
    np.testing.assert_allclose(r["marginals"], ref, rtol=2e-4, atol=2e-4)


def test_stop_rule_and_codewords():
    H = W.zsz_2bga("ZSZ-2BGA-64")
    N = H.shape[1]
    L = np.full((3, N), 2.0, dtype=np.float32)
    r = oracle.spa_decode(H, L, max_iterations=100, nthreads=1)
    assert (r["iters"] == 1).all() and (r["converged"] == 1).all() and not r["bits"].any()
    sigma = W.awgn_sigma(2.0, 0.5)
    L = W.awgn_llrs(N, 400, sigma, seed=5)
    r = oracle.spa_decode(H, L, max_iterations=100, nthreads=4)
    conv = r["converged"] == 1
    assert 0.5 < conv.mean() < 1.0
    assert not ((r["bits"][conv].astype(np.int64) @ H.T.astype(np.int64)) % 2).any()
    # without stopping, every shot runs the full budget
    r2 = oracle.spa_decode(H, L[:20], max_iterations=7, stop=False, nthreads=2)
    assert (r2["iters"] == 7).all()


def test_awgn_channel_statistics():
    sigma = 0.8
    llr = oracle.awgn(101, 4000, sigma, seed=9)
    x = llr.reshape(-1)
    mu, var = 2.0 / sigma ** 2, 4.0 / sigma ** 2
    n = x.size
    assert abs(x.mean() - mu) < 5 * np.sqrt(var / n)
    assert abs(x.var() / var - 1.0) < 5 * np.sqrt(2.0 / n)
    assert sst.kstest((x - mu) / np.sqrt(var), "norm").pvalue > 1e-3
    # adjacent bits (same and different Philox words) and adjacent shots are uncorrelated
    assert abs(np.corrcoef(llr[:, :-1].reshape(-1), llr[:, 1:].reshape(-1))[0, 1]) < 0.01
    assert abs(np.corrcoef(llr[:-1].reshape(-1), llr[1:].reshape(-1))[0, 1]) < 0.01
    # shot offsets address the same stream
    np.testing.assert_array_equal(oracle.awgn(101, 10, sigma, 9, shot_offset=5), llr[5:15])


def tanner_girth(H):
    """Shortest cycle of the bipartite Tanner graph by BFS from every node."""
    M, N = H.shape
    adj = [[] for _ in range(M + N)]
    for i, j in zip(*np.nonzero(H)):
        adj[N + i].append(j)
        adj[j].append(N + i)
    best = np.inf
    for s in range(M + N):
        dist = {s: 0}
        par = {s: -1}
        q = [s]
        for u in q:
            for v in adj[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    par[v] = u
                    q.append(v)
                elif par[u] != v:
                    best = min(best, dist[u] + dist[v] + 1)
    return int(best)


@pytest.mark.parametrize("name", list(W.ZSZ_2BGA))
def test_classical_code_tables(name):
    lp, n, k, d, girth = W.ZSZ_2BGA[name]
    for side in ("left", "right"):
        H = W.zsz_2bga(name, side)
        assert H.shape == (n // 2, n)
        assert set(H.sum(axis=0).tolist()) == {3} and set(H.sum(axis=1).tolist()) == {6}
        assert n - W.gf2_rank(H) == k
        assert tanner_girth(H) == girth, (name, side)


def test_shannon_limit():
    lim = stats.shannon_limit_db(0.5)
    assert abs(lim - 0.187) < 0.002 and abs(lim - 0.19) < 0.01
    # the capacity by Monte Carlo on independent samples of the LLR law
    rng = np.random.default_rng(4)
    for sigma in (0.6, 0.97, 1.5):
        L = 2.0 / sigma ** 2 + (2.0 / sigma) * rng.standard_normal(2_000_000)
        mc = 1.0 - np.mean(np.logaddexp(0.0, -L)) / np.log(2.0)
        assert abs(stats.bpsk_awgn_capacity(sigma) - mc) < 2e-3
    caps = [stats.bpsk_awgn_capacity(s) for s in (0.3, 0.6, 1.0, 2.0, 4.0)]
    assert all(a > b for a, b in zip(caps, caps[1:])) and caps[0] > 0.99
    # E_b/N_0 = 1 / (2 R sigma^2)
    s = W.awgn_sigma(3.0, 0.5)
    assert abs(10 * np.log10(1.0 / (2 * 0.5 * s * s)) - 3.0) < 1e-12
