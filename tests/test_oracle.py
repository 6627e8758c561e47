"""Pins of the CPU oracle against definitions, closed forms, brute force and invariants.

Each test fixes something the oracle must reproduce that does not come from
the oracle itself: published known-answer vectors, exact min-marginals by
exhaustive enumeration, minimum-weight solutions by enumeration, the GF(2)
syndrome map as a dense matrix product, binomial closed forms.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import stats as ostats
from paper_2607_27644_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _graph(dem):
    return oracle.Graph(dem.H, dem.O)


# ---------------------------------------------------------------- Philox
def test_philox_known_answers():
    for ln in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        v = [int(x, 16) for x in ln.split()]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# ---------------------------------------------------------------- thresholds, LLRs, gammas
def test_sampler_tables_closed_form():
    # T_k = floor((1 - pmax)^k 2^32): powers of two for pmax = 1/2 (up to one unit
    # of rounding in exp), and floor(0.999 * 2^32) for pmax = 1e-3
    T = oracle.gap_table(0.5, 40)
    for k in range(1, 41):
        assert int(T[k - 1]) in (2 ** (32 - k), 2 ** (32 - k) - 1) or (k > 32 and int(T[k - 1]) == 0)
    assert int(oracle.gap_table(1e-3, 1)[0]) == math.floor(0.999 * 2 ** 32)
    t = oracle.gap_table(1e-3, 2000).astype(np.int64)
    assert (np.diff(t) <= 0).all()
    assert abs(t[1999] / 2 ** 32 - 0.999 ** 2000) < 1e-9
    # acceptance: p_j / pmax in 32-bit fixed point; p_j = pmax is marked
    A = oracle.accept_table(np.array([1e-3, 5e-4, 2.5e-4, 1e-3]), 1e-3)
    assert list(A) == [0xFFFFFFFF, 2 ** 31, 2 ** 30, 0xFFFFFFFF]


def test_llr_closed_form():
    x = np.array([0.5, 2.0, 6.9, 13.0])
    p = 1.0 / (1.0 + np.exp(x))
    lam = oracle.llr(p)
    assert np.allclose(lam, x, rtol=1e-6)
    assert lam.dtype == np.float32


def test_gamma_table_definition():
    N, R, lo, hi, seed = 10, 3, -0.24, 0.66, 99
    tab = oracle.gamma_table(N, R, lo, hi, seed)
    assert tab.shape == (R, N)
    assert (tab >= np.float32(lo)).all() and (tab <= np.float32(hi)).all()
    # entry (r, j) uses counter (j/4, r, 0, 1) and word j % 4
    for r, j in [(1, 0), (2, 5), (3, 9)]:
        o = oracle.philox4x32_10([j // 4, r, 0, 1], [seed & 0xFFFFFFFF, seed >> 32])
        u = np.float32(int(o[j % 4]) >> 8) * np.float32(2.0 ** -24)
        span = np.float32(np.float32(hi) - np.float32(lo))
        exact = float(u) * float(span) + float(np.float32(lo))
        assert abs(float(tab[r - 1, j]) - exact) <= 1e-7


def test_gamma_table_spread():
    tab = oracle.gamma_table(1000, 20, -0.24, 0.66, 5)
    assert abs(tab.mean() - 0.21) < 0.01
    assert tab.min() < -0.23 and tab.max() > 0.65


# ---------------------------------------------------------------- sampling and syndromes
def test_sampler_frequency_and_syndrome_map():
    dem = W.workload("cc160")
    g = _graph(dem)
    shots = 4000
    syn, obs, err = oracle.sample(g, dem.priors, shots, seed=11, want_errors=True)
    e = W.unpack_bits(err, dem.N)
    # flips ~ Binomial(shots * N, p): 5-sigma window
    n, p = shots * dem.N, 0.01
    assert abs(e.sum() - n * p) < 5 * math.sqrt(n * p * (1 - p))
    # per-mechanism counts are consistent with the same p (chi-square, N-1 dof)
    cnt = e.sum(0)
    chi2 = ((cnt - shots * p) ** 2 / (shots * p * (1 - p))).sum()
    assert chi2 < dem.N + 6 * math.sqrt(2 * dem.N)
    # sigma = H e and o = O e as dense GF(2) products
    s_dense = (e.astype(np.int64) @ dem.H.T.astype(np.int64)) % 2
    o_dense = (e.astype(np.int64) @ dem.O.T.astype(np.int64)) % 2
    assert np.array_equal(W.unpack_bits(syn, dem.M), s_dense)
    assert np.array_equal(W.unpack_bits(obs, dem.k), o_dense)
    assert np.array_equal(oracle.syndrome(g, err), syn)


def test_sampler_adjacent_pairs_uncorrelated():
    dem = W.workload("cc160")
    pri = np.full(dem.N, 0.3)
    _, _, err = oracle.sample(_graph(dem), pri, 3000, seed=2, want_errors=True)
    e = W.unpack_bits(err, dem.N).astype(float)
    c = np.corrcoef(e[:, 0:80].ravel(), e[:, 1:81].ravel())[0, 1]
    assert abs(c) < 0.01
    c2 = np.corrcoef(e[:-1].ravel(), e[1:].ravel())[0, 1]
    assert abs(c2) < 0.01


def test_sampler_thinning_nonuniform_priors():
    # per-mechanism frequencies follow p_j when the priors differ (geometric gaps
    # at the largest prior, candidates kept with probability p_j / pmax)
    dem = W.workload("cc160")
    pri = W.random_priors(dem.N, 2e-3, 5e-2, seed=4)
    shots = 20000
    _, _, err = oracle.sample(_graph(dem), pri, shots, seed=21, want_errors=True)
    cnt = W.unpack_bits(err, dem.N).sum(0)
    z = (cnt - shots * pri) / np.sqrt(shots * pri * (1 - pri))
    assert (z ** 2).sum() < dem.N + 6 * math.sqrt(2 * dem.N)
    assert np.abs(z).max() < 5.0


def test_sampler_segment_law():
    # no fault in a segment of length len with probability (1 - p)^len; segments of
    # one shot are independent (64 segments of ceil(N / 64) mechanisms)
    dem = W.workload("phen160")
    p = 2e-3
    shots = 20000
    _, _, err = oracle.sample(_graph(dem), np.full(dem.N, p), shots, seed=8, want_errors=True)
    e = W.unpack_bits(err, dem.N)
    L = (dem.N + 63) // 64
    seg = np.add.reduceat(e, np.arange(0, dem.N, L), axis=1) > 0
    q = (1 - p) ** L
    n0 = (~seg[:, :-1]).sum()
    n = seg[:, :-1].size
    assert abs(n0 - n * q) < 5 * math.sqrt(n * q * (1 - q))
    c = np.corrcoef(seg[:, 0].astype(float), seg[:, 1].astype(float))[0, 1]
    assert abs(c) < 0.03


def test_sampler_offsets_are_resumable():
    dem = W.workload("phen160")
    g = _graph(dem)
    full = oracle.sample(g, dem.priors, 300, seed=5)[0]
    part = oracle.sample(g, dem.priors, 100, seed=5, shot_offset=150)[0]
    assert np.array_equal(full[150:250], part)
    other = oracle.sample(g, dem.priors, 300, seed=6)[0]
    assert not np.array_equal(full, other)


# ---------------------------------------------------------------- min-sum on trees
def _random_tree(rng, n_checks):
    """Tanner graph that is a tree: each new check joins one existing
    variable and 1-3 new ones."""
    edges = []
    nv = 1
    for c in range(n_checks):
        old = int(rng.integers(nv))
        new = list(range(nv, nv + int(rng.integers(1, 4))))
        nv += len(new)
        for v in [old] + new:
            edges.append((c, v))
    H = np.zeros((n_checks, nv), np.uint8)
    for c, v in edges:
        H[c, v] = 1
    return H


def _exact_min_marginals(H, lam, sigma):
    N = H.shape[1]
    best = {0: np.full(N, np.inf), 1: np.full(N, np.inf)}
    for bits in itertools.product((0, 1), repeat=N):
        e = np.array(bits)
        if np.array_equal((H.astype(int) @ e) % 2, sigma):
            w = float(e @ lam)
            for b in (0, 1):
                sel = e == b
                best[b][sel] = np.minimum(best[b][sel], w)
    return best[1] - best[0]


@pytest.mark.parametrize("seed", range(6))
def test_min_sum_is_exact_on_trees(seed):
    rng = np.random.default_rng(seed)
    H = _random_tree(rng, int(rng.integers(3, 6)))
    N = H.shape[1]
    if N > 16:
        pytest.skip("tree too large for enumeration")
    p = rng.uniform(0.02, 0.3, N)
    lam64 = oracle.llr(p).astype(np.float64)
    g = oracle.Graph(H, np.zeros((0, N), np.uint8))
    for trial in range(3):
        sigma = rng.integers(0, 2, H.shape[0]).astype(np.uint8)
        Mx = oracle.bp_marginals(g, p, W.pack_bits(sigma[None, :])[0], gamma=0.0, T=3 * H.shape[0] + 2)
        exact = _exact_min_marginals(H, lam64, sigma)
        assert np.allclose(Mx, exact, rtol=1e-5, atol=1e-4), (Mx, exact)


def test_min_sum_single_check_closed_form():
    # one check on three variables, sigma = 1: M_j = Lambda_j + (-1) * min of the others
    H = np.ones((1, 3), np.uint8)
    p = np.array([0.1, 0.2, 0.3])
    lam = oracle.llr(p)
    g = oracle.Graph(H, np.zeros((0, 3), np.uint8))
    Mx = oracle.bp_marginals(g, p, np.array([1], np.uint32), gamma=0.0, T=1)
    for j in range(3):
        others = [lam[i] for i in range(3) if i != j]
        assert Mx[j] == np.float32(lam[j] - min(others))


def test_memory_term_closed_form():
    # degree-2 check (sigma = 0) between a variable and a much more reliable one:
    # mu into variable 0 equals |nu_1| = Lambda_1 at t = 1, so
    # M_0(1) = fmaf(g, M_0(0) - L0, L0) + L1 = L0 + L1 (M_0(0) = L0); at t = 2
    # nu_1 = M_1(1) - mu_{->1}(1) = L1 + L0 - L0 = L1 again and
    # M_0(2) = L0 + g*(M_0(1) - L0) + L1 = L0 + g*L1 + L1.
    H = np.array([[1, 1]], np.uint8)
    p = np.array([0.2, 0.01])
    lam = oracle.llr(p).astype(np.float64)
    g = oracle.Graph(H, np.zeros((0, 2), np.uint8))
    for gam in (0.0, 0.125, 0.5, -0.2):
        m1 = oracle.bp_marginals(g, p, np.array([0], np.uint32), gamma=gam, T=1)
        m2 = oracle.bp_marginals(g, p, np.array([0], np.uint32), gamma=gam, T=2)
        assert abs(m1[0] - (lam[0] + lam[1])) < 1e-5
        assert abs(m2[0] - (lam[0] + gam * lam[1] + lam[1])) < 1e-5


# ---------------------------------------------------------------- Relay-BP decode flow
def _params(**kw):
    return oracle.RelayParams(**kw)


def test_zero_syndrome_shortcut():
    dem = W.workload("phen160")
    g = _graph(dem)
    syn = np.zeros((3, (dem.M + 31) // 32), np.uint32)
    r = oracle.decode(g, dem.priors, syn, _params(), nthreads=2)
    assert not r["corrections"].any() and (r["converged"] == 1).all() and (r["path"] == 3).all()
    assert (r["legs"] == 0).all()


def test_textbook_min_sum_reduction():
    """gamma0 = 0 and no relay legs is flooding min-sum that stops at the first
    iteration whose hard decision reproduces the syndrome."""
    dem = W.workload("cc160")
    g = _graph(dem)
    syn, _, _ = oracle.sample(g, dem.priors, 60, seed=3)
    T = 12
    r = oracle.decode(g, dem.priors, syn, _params(gamma0=0.0, num_sets=0, pre_iter=T), nthreads=4)
    for s in range(syn.shape[0]):
        sigma = W.unpack_bits(syn[s:s + 1], dem.M)[0]
        if not sigma.any():
            continue
        want = None
        for t in range(1, T + 1):
            Mx = oracle.bp_marginals(g, dem.priors, syn[s], 0.0, t)
            e = (Mx < 0).astype(np.uint8)
            if np.array_equal((dem.H.astype(int) @ e) % 2, sigma):
                want = (e, t)
                break
        got = W.unpack_bits(r["corrections"][s:s + 1], dem.N)[0]
        if want is None:
            assert r["converged"][s] == 0 and r["iters"][s] == T
            assert np.array_equal(got, (Mx < 0).astype(np.uint8))
        else:
            assert r["converged"][s] == 1 and r["iters"][s] == want[1]
            assert np.array_equal(got, want[0])


def test_relay_legs_with_zero_memory_repeat_leg0():
    dem = W.workload("cc160")
    g = _graph(dem)
    syn, _, _ = oracle.sample(g, dem.priors, 40, seed=4)
    one = oracle.decode(g, dem.priors, syn, _params(gamma0=0.0, num_sets=0), nthreads=4)
    rel = oracle.decode(g, dem.priors, syn, _params(gamma0=0.0, gamma_min=0.0, gamma_max=0.0, num_sets=10),
                        nthreads=4)
    nz = one["path"] != 3
    ok = nz & (one["converged"] == 1)
    assert np.array_equal(one["corrections"][ok], rel["corrections"][ok])
    assert (rel["nconv"][ok] == 5).all() and (rel["legs"][ok] == 5).all()
    assert np.array_equal(rel["iters"][ok], 5 * one["iters"][ok])


def _bruteforce_min_weight(H, max_w):
    """syndrome (as int) -> minimum Hamming weight of an error with that syndrome."""
    m, n = H.shape
    colint = np.array([int("".join(str(b) for b in H[::-1, j]), 2) for j in range(n)], dtype=np.int64)
    best = {0: 0}
    for w in range(1, max_w + 1):
        for comb in itertools.combinations(range(n), w):
            s = 0
            for j in comb:
                s ^= int(colint[j])
            if s not in best:
                best[s] = w
    return best


@pytest.mark.slow
def test_relay_bp_against_minimum_weight_on_60_qubit_code():
    c = W.zsz_lp("ZSZ-LP-60")
    dem = W.code_capacity_dem(c, 0.02)
    g = _graph(dem)
    best = _bruteforce_min_weight(dem.H, 3)
    rng = np.random.default_rng(7)
    errs = []
    for _ in range(150):
        w = int(rng.integers(1, 3))
        e = np.zeros(dem.N, np.uint8)
        e[rng.choice(dem.N, w, replace=False)] = 1
        errs.append(e)
    errs = np.array(errs)
    sig = (errs.astype(int) @ dem.H.T.astype(int)) % 2
    syn = W.pack_bits(sig)
    r = oracle.decode(g, dem.priors, syn, _params(), nthreads=4)
    ehat = W.unpack_bits(r["corrections"], dem.N)
    conv = r["converged"] == 1
    assert conv.mean() > 0.95
    resyn = (ehat.astype(int) @ dem.H.T.astype(int)) % 2
    assert np.array_equal(resyn[conv], sig[conv])
    equal = 0
    for s in range(len(errs)):
        if not conv[s]:
            continue
        key = int("".join(str(b) for b in sig[s][::-1]), 2)
        wmin = best.get(key, 4)
        assert ehat[s].sum() >= wmin
        equal += ehat[s].sum() == wmin
    assert equal >= 0.9 * conv.sum()


@pytest.mark.parametrize("name", ["cc160", "phen160"])
def test_converged_corrections_reproduce_syndrome(name):
    dem = W.workload(name)
    g = _graph(dem)
    syn, _, _ = oracle.sample(g, dem.priors, 400, seed=12)
    r = oracle.decode(g, dem.priors, syn, _params(), nthreads=8)
    e = W.unpack_bits(r["corrections"], dem.N)
    s = (e.astype(np.int64) @ dem.H.T.astype(np.int64)) % 2
    conv = r["converged"] == 1
    assert conv.mean() > 0.99
    assert np.array_equal(s[conv], W.unpack_bits(syn, dem.M)[conv])
    # predicted observables are O applied to the correction
    o = (e.astype(np.int64) @ dem.O.T.astype(np.int64)) % 2
    assert np.array_equal(W.unpack_bits(r["obs_pred"], dem.k), o)


def test_determinism_across_threads():
    dem = W.workload("phen160")
    g = _graph(dem)
    syn, _, _ = oracle.sample(g, dem.priors, 200, seed=13)
    a = oracle.decode(g, dem.priors, syn, _params(), nthreads=1)
    b = oracle.decode(g, dem.priors, syn, _params(), nthreads=7)
    for key in ("corrections", "obs_pred", "converged", "legs", "iters", "nconv"):
        assert np.array_equal(a[key], b[key])


def test_all_criterion_runs_every_leg_and_never_loses():
    dem = W.workload("cc160")
    g = _graph(dem)
    syn, _, _ = oracle.sample(g, dem.priors, 60, seed=14)
    R = 12
    nc = oracle.decode(g, dem.priors, syn, _params(num_sets=R), nthreads=4)
    al = oracle.decode(g, dem.priors, syn, _params(num_sets=R, stopping_criterion=1), nthreads=4)
    lam = oracle.llr(dem.priors).astype(np.float64)
    nz = nc["path"] != 3
    assert (al["legs"][nz] == R + 1).all()
    wn = W.unpack_bits(nc["corrections"], dem.N) @ lam
    wa = W.unpack_bits(al["corrections"], dem.N) @ lam
    ok = (nc["converged"] == 1) & nz
    assert (wa[ok] <= wn[ok] + 1e-9).all()


def test_learned_proposal_paths():
    dem = W.workload("cc160")
    g = _graph(dem)
    syn, _, err = oracle.sample(g, dem.priors, 80, seed=15, want_errors=True)
    e = W.unpack_bits(err, dem.N)
    lam = oracle.llr(dem.priors)
    # delta = 0: the proposal leg is leg 0, accepted when it converges
    zero = np.zeros((80, dem.N), np.float32)
    rp = oracle.decode(g, dem.priors, syn, _params(), delta=zero, nthreads=4)
    r1 = oracle.decode(g, dem.priors, syn, _params(stop_nconv=1), nthreads=4)
    nz = rp["path"] != 3
    acc = rp["path"] == 1
    assert acc[nz].mean() > 0.9
    assert np.array_equal(rp["corrections"][acc], r1["corrections"][acc])
    # an oracle proposal pointing at the true error is accepted and returns it
    d = np.where(e == 1, -2.0 * lam - 10.0, 10.0).astype(np.float32)
    ro = oracle.decode(g, dem.priors, syn, _params(), delta=d, nthreads=4)
    assert (ro["path"][nz] == 1).all()
    assert np.array_equal(W.unpack_bits(ro["corrections"], dem.N)[nz], e[nz])
    # a noise proposal does not converge; plain Relay-BP then runs from scratch
    bad = np.random.default_rng(0).normal(0.0, 20.0, (80, dem.N)).astype(np.float32)
    rb = oracle.decode(g, dem.priors, syn, _params(), delta=bad, nthreads=4)
    full = oracle.decode(g, dem.priors, syn, _params(), nthreads=4)
    fb = rb["path"] == 2
    assert fb[nz].all()
    assert np.array_equal(rb["corrections"], full["corrections"])
    assert (rb["legs"][nz] == full["legs"][nz] + 1).all()
    # a proposal leg that converges is accepted even when its solution is heavier
    mis = np.where(e == 1, 30.0, -30.0).astype(np.float32)
    rm = oracle.decode(g, dem.priors, syn, _params(), delta=mis, nthreads=4)
    assert (rm["path"][nz] == 1).all()
    em = W.unpack_bits(rm["corrections"], dem.N)
    assert np.array_equal((em.astype(int) @ dem.H.T.astype(int)) % 2, W.unpack_bits(syn, dem.M))


def test_trace_matches_marginal_iteration():
    dem = W.workload("cc160")
    g = _graph(dem)
    syn, _, _ = oracle.sample(g, dem.priors, 30, seed=16)
    prm = _params(gamma0=0.125)
    for s in range(30):
        for t in (1, 2, 3):
            tr = oracle.trace(g, dem.priors, syn[s], prm, leg=0, t=t)
            if tr is None:
                continue
            ref = oracle.bp_marginals(g, dem.priors, syn[s], 0.125, t)
            assert np.array_equal(tr[0], ref)


# ---------------------------------------------------------------- statistics
def test_clopper_pearson_closed_forms():
    n = 1000
    lo, hi = ostats.clopper_pearson(0, n)
    assert lo == 0.0 and abs(hi - (1 - 0.025 ** (1 / n))) < 1e-12
    lo, hi = ostats.clopper_pearson(n, n)
    assert hi == 1.0 and abs(lo - 0.025 ** (1 / n)) < 1e-12
    a = ostats.clopper_pearson(7, 100)
    b = ostats.clopper_pearson(93, 100)
    assert abs(a[0] - (1 - b[1])) < 1e-10 and abs(a[1] - (1 - b[0])) < 1e-10


def test_clopper_pearson_matches_beta_quantiles():
    from scipy.stats import beta
    for x, n in [(1, 50), (5, 1000), (37, 100000), (500, 1000)]:
        lo, hi = ostats.clopper_pearson(x, n)
        assert abs(lo - beta.ppf(0.025, x, n - x + 1)) < 1e-9
        assert abs(hi - beta.ppf(0.975, x + 1, n - x)) < 1e-9


def test_per_round_rate():
    assert abs(ostats.per_round(1 - 0.9 ** 9, 9) - 0.1) < 1e-12
    assert ostats.per_round(0.0, 5) == 0.0
