"""More pins of the CPU oracle: the relay step across leg boundaries, and the
fault law of the gap sampler against the plain per-mechanism definition.

Relay-BP (Sec. 6.1): every relay leg restarts its messages, starts from the
marginals the previous leg ended with, and uses that leg's own row of memory
strengths.  The closed forms below are derived by hand on a single check of
three variables, where each leg converges at its first iteration, so every
marginal is a short FP32 expression of the LLRs and the strengths.

Sampling: each mechanism faults independently with probability p_j.  The
oracle's main sampler draws by geometric gaps over 64 segments (the layout the
GPU sampler reproduces bit for bit); here its law is checked against the plain
definition (one word per mechanism, e_j = [word < floor(p_j 2^32)]) and
against the exact Poisson-binomial law of the number of faults per shot, with
checks shown to reject a law that is off by a few percent or correlated.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2607_27644_amd import workloads as W


# ---------------------------------------------------------------- relay legs
def _three_var_check():
    H = np.ones((1, 3), np.uint8)
    p = np.array([0.2, 0.05, 0.01])
    g = oracle.Graph(H, np.zeros((0, 3), np.uint8))
    syn = np.array([1], np.uint32)  # sigma = 1
    return g, p, syn


def test_relay_step_closed_form_across_legs():
    # One check on three variables with sigma = 1, Lambda_0 < Lambda_1 < Lambda_2.
    # Leg 0 (nu(0) = Lambda, M(0) = Lambda): mu = -(least other |nu|) =
    # (-L1, -L0, -L0); M_j = fmaf(g0, 0, L_j) + mu_j = L_j + mu_j; only variable 0
    # turns negative, the check is satisfied: converged at t = 1.
    # Leg r >= 1 restarts nu(0) = Lambda, so mu is again (-L1, -L0, -L0), and
    # M_j = fmaf(gamma^(r)_j, M_j(end of leg r-1) - L_j, L_j) + mu_j with the
    # strengths of row r - 1 of the relay table; again converged at t = 1.
    g, p, syn = _three_var_check()
    L = oracle.llr(p)
    R, seed, lo, hi = 3, 11, -0.24, 0.66
    prm = oracle.RelayParams(gamma0=0.125, gamma_min=lo, gamma_max=hi, pre_iter=4, max_iterations=4,
                             num_sets=R, stop_nconv=5, stopping_criterion=1, gamma_seed=seed)
    gam = oracle.gamma_table(3, R, lo, hi, seed)
    mu0 = np.array([-L[1], -L[0], -L[0]], np.float32)
    M = (L + mu0).astype(np.float32)  # leg 0, t = 1 (one FP32 add each)
    tr = oracle.trace(g, p, syn, prm, leg=0, t=1)
    assert tr is not None
    assert np.array_equal(tr[0], M)
    assert np.array_equal(tr[1], mu0)
    assert oracle.trace(g, p, syn, prm, leg=0, t=2) is None  # leg 0 ended at t = 1
    for r in range(1, R + 1):
        tr = oracle.trace(g, p, syn, prm, leg=r, t=1)
        assert tr is not None, r
        # restart: the first messages of every leg are leg 0's
        assert np.array_equal(tr[1], mu0), r
        want = np.array([float(gam[r - 1, j]) * float(M[j] - L[j]) + float(L[j]) + float(mu0[j])
                         for j in range(3)])
        assert np.allclose(tr[0], want, rtol=1e-6, atol=1e-6), (r, tr[0], want)
        # the alternatives a wrong carry or a wrong row would produce are far off
        reset = (L + mu0).astype(np.float64)  # marginals reset to Lambda each leg
        assert np.abs(tr[0] - reset).max() > 1e-2, r
        other = gam[r % R] if R > 1 else gam[0]
        wrong_row = np.array([float(other[j]) * float(M[j] - L[j]) + float(L[j]) + float(mu0[j]) for j in range(3)])
        assert np.abs(tr[0] - wrong_row).max() > 1e-3, r
        M = tr[0]
    # every leg converges to e = (1, 0, 0) of weight Lambda_0: 1 + R solutions
    r = oracle.decode(g, p, syn[None, :], prm, nthreads=1)
    assert r["nconv"][0] == 1 + R and r["legs"][0] == 1 + R and r["iters"][0] == 1 + R
    assert r["corrections"][0, 0] == 1 and r["converged"][0] == 1


def test_relay_carry_keeps_non_converged_marginals():
    # A leg that does not converge still hands its final marginals on.  Four
    # checks on a cycle of four variables with an odd-weight syndrome have no
    # solution, so no leg converges: the marginals at (leg r, t = 1) must be the
    # memory update of the marginals at (leg r - 1, last iteration).
    H = np.array([[1, 1, 0, 0], [0, 1, 1, 0], [0, 0, 1, 1], [1, 0, 0, 1]], np.uint8)
    g = oracle.Graph(H, np.zeros((0, 4), np.uint8))
    p = np.array([0.1, 0.03, 0.2, 0.05])
    syn = np.array([0b0001], np.uint32)  # one unsatisfied check: odd parity, unsolvable
    L = oracle.llr(p).astype(np.float64)
    R, T0, Tr = 2, 3, 2
    prm = oracle.RelayParams(gamma0=0.125, gamma_min=-0.24, gamma_max=0.66, pre_iter=T0, max_iterations=Tr,
                             num_sets=R, stop_nconv=5, stopping_criterion=0, gamma_seed=3)
    gam = oracle.gamma_table(4, R, -0.24, 0.66, 3)
    r = oracle.decode(g, p, syn[None, :], prm, nthreads=1)
    assert r["converged"][0] == 0 and r["nconv"][0] == 0
    assert r["legs"][0] == 1 + R and r["iters"][0] == T0 + R * Tr
    last = oracle.trace(g, p, syn, prm, leg=0, t=T0)[0].astype(np.float64)
    first_mu = oracle.trace(g, p, syn, prm, leg=0, t=1)[1]
    for leg in range(1, R + 1):
        M, mu = oracle.trace(g, p, syn, prm, leg=leg, t=1)
        assert np.array_equal(mu, first_mu)  # messages restart from nu(0) = Lambda
        # M_j = Lt_j + sum of the mu into j (CSC edge order: per column, ascending rows)
        cp, ri = g.cp, g.ri
        musum = np.array([mu[cp[j]:cp[j + 1]].astype(np.float64).sum() for j in range(4)])
        want = gam[leg - 1].astype(np.float64) * (last - L) + L + musum
        assert np.allclose(M, want, rtol=1e-6, atol=1e-6), (leg, M, want)
        last = oracle.trace(g, p, syn, prm, leg=leg, t=Tr)[0].astype(np.float64)


# ---------------------------------------------------------------- sampler law
def _poisson_binomial(p):
    """Exact pmf of the number of successes of independent Bernoulli(p_j)."""
    f = np.zeros(len(p) + 1)
    f[0] = 1.0
    for q in p:
        f[1:] = f[1:] * (1 - q) + f[:-1] * q
        f[0] *= 1 - q
    return f


def _chi2_pooled(counts, expect, min_expect=20.0):
    """Pearson chi-square with the tail bins pooled until each expects min_expect."""
    c, e = [], []
    ac = ae = 0.0
    for k in range(len(expect)):
        ac += counts[k]
        ae += expect[k]
        if ae >= min_expect:
            c.append(ac)
            e.append(ae)
            ac = ae = 0.0
    if ae > 0:
        c[-1] += ac
        e[-1] += ae
    c, e = np.array(c), np.array(e)
    return float(((c - e) ** 2 / e).sum()), len(c) - 1


def _chi2_ok(chi2, dof, z=5.0):
    return chi2 < dof + z * math.sqrt(2 * dof)


def _freq_chi2(cnt, shots, p):
    z = (cnt - shots * p) / np.sqrt(shots * p * (1 - p))
    return float((z ** 2).sum()), len(p)


def test_plain_sampler_is_the_definition():
    # e_j = [word_j < floor(p_j 2^32)], word_j = Philox(seed; j/4, shot, 0)_{j mod 4}
    N, shots, seed = 13, 5, 99
    p = np.linspace(0.05, 0.5, N)
    err = oracle.sample_plain(N, p, shots, seed, shot_offset=2 ** 32 + 7)
    e = W.unpack_bits(err, N)
    for s in range(shots):
        sid = 2 ** 32 + 7 + s
        for j in range(N):
            w = oracle.philox4x32_10([j // 4, sid & 0xFFFFFFFF, sid >> 32, 0], [seed, 0])[j % 4]
            assert e[s, j] == int(int(w) < math.floor(p[j] * 2 ** 32))
    # frequencies follow p_j
    p = W.random_priors(300, 1e-3, 0.2, seed=2)
    cnt = W.unpack_bits(oracle.sample_plain(300, p, 20000, seed=4), 300).sum(0)
    assert _chi2_ok(*_freq_chi2(cnt, 20000, p))


def _law_checks(b, p):
    """Checks of a fault sample b (shots x N, 0/1) against independent
    Bernoulli(p_j) faults; name -> passed."""
    shots, N = b.shape
    out = {}
    cnt = b.sum(0).astype(np.float64)
    out["frequency"] = _chi2_ok(*_freq_chi2(cnt, shots, p))
    hist = np.bincount(b.sum(1), minlength=N + 1)[: N + 1]
    out["count_law"] = _chi2_ok(*_chi2_pooled(hist, shots * _poisson_binomial(p)))
    # co-occurrence of neighbours, inside a segment and across the 64-segment
    # boundaries of the gap sampler: joint counts ~ Poisson(shots p_i p_j)
    L = (N + 63) // 64
    for name, sel in (("neighbours", [(j, j + 1) for j in range(N - 1)]),
                      ("segment_boundaries", [(k * L - 1, k * L) for k in range(1, 64) if k * L < N])):
        a = np.array([i for i, _ in sel])
        c = np.array([j for _, j in sel])
        obs = float((b[:, a] & b[:, c]).sum())
        exp = float((shots * p[a] * p[c]).sum())
        out[name] = abs(obs - exp) < 5 * math.sqrt(exp) + 3
    # the same mechanism in consecutive shots
    obs = float((b[1:] & b[:-1]).sum())
    exp = float((shots - 1) * (p * p).sum())
    out["consecutive_shots"] = abs(obs - exp) < 5 * math.sqrt(exp) + 3
    return out


@pytest.mark.parametrize("name,lo,hi", [("phen160", 1e-3, 1e-3), ("phen160", 5e-4, 2e-2), ("cc160", 0.01, 0.01)])
def test_gap_sampler_law_matches_plain_definition(name, lo, hi):
    dem = W.workload(name)
    N = dem.N
    p = np.full(N, lo) if lo == hi else W.random_priors(N, lo, hi, seed=6)
    shots = 40000 if N > 1000 else 60000
    g = oracle.Graph(dem.H, dem.O)
    _, _, eg = oracle.sample(g, p, shots, seed=31, want_errors=True)
    ep = oracle.sample_plain(N, p, shots, seed=32)
    bg, bp = W.unpack_bits(eg, N), W.unpack_bits(ep, N)
    for b in (bg, bp):
        res = _law_checks(b, p)
        assert all(res.values()), res
    # the two samplers' per-mechanism counts against each other
    cg, cpl = bg.sum(0).astype(np.float64), bp.sum(0).astype(np.float64)
    z2 = ((cg - cpl) ** 2 / (2 * shots * p * (1 - p))).sum()
    assert _chi2_ok(z2, N)
    # and their fault-count histograms (two-sample chi-square over pooled bins)
    hg = np.bincount(bg.sum(1), minlength=N + 1)[: N + 1].astype(np.float64)
    hp = np.bincount(bp.sum(1), minlength=N + 1)[: N + 1].astype(np.float64)
    tot = hg + hp
    keep = tot >= 20
    chi = float((((hg - hp)[keep]) ** 2 / tot[keep]).sum())
    assert _chi2_ok(chi, int(keep.sum()) - 1)


def test_sampler_law_checks_reject_a_biased_or_correlated_law():
    # The checks above have power: the gap sampler's faults thinned by 4 %, or
    # one segment of every even shot copied into the next shot, fail them.
    dem = W.workload("phen160")
    N = dem.N
    p = np.full(N, 1e-3)
    shots = 40000
    g = oracle.Graph(dem.H, dem.O)
    _, _, eg = oracle.sample(g, p, shots, seed=41, want_errors=True)
    b = W.unpack_bits(eg, N)
    assert all(_law_checks(b, p).values())
    rng = np.random.default_rng(0)
    thinned = b & (rng.random(b.shape) >= 0.04).astype(b.dtype)
    assert not all(_law_checks(thinned, p).values())
    L = (N + 63) // 64
    corr = b.copy()
    corr[1::2, :L] = corr[0::2, :L]
    res = _law_checks(corr, p)
    assert not res["consecutive_shots"], res


def test_marginals_saturate_and_stay_finite():
    """Min-sum with memory grows messages geometrically on shots that never
    converge (phen160 at p = 1 %, gamma in [0, 0.66]: |M| about 4e10 after leg
    0 and 6e18 after leg 1).  The marginals saturate at 2^90, so every marginal
    and message stays finite, the bound is attained, and no check message
    exceeds the one-iteration growth bound (|mu| <= max |nu| <= 2^90 + max |mu|
    of the previous iteration, at most T 2^90 within a leg of T iterations)."""
    dem = W.workload("phen160")
    g = oracle.Graph(dem.H, dem.O)
    pr = np.full(dem.N, 1e-2)
    syn, _ = oracle.sample(g, pr, 379, 17)[:2]
    prm = oracle.RelayParams(gamma_min=0.0, gamma_max=0.66, num_sets=10)
    sat = float(np.float32(2.0 ** 90))
    for leg, t in [(0, 80), (1, 60), (5, 60), (10, 60)]:
        M, mu = oracle.trace(g, pr, syn[378], prm, leg=leg, t=t)
        assert np.isfinite(M).all() and np.isfinite(mu).all(), (leg, t)
        assert np.abs(M).max() <= sat
        assert np.abs(mu).max() <= t * sat
        if leg >= 5:
            assert np.abs(M).max() == sat  # the bound is reached, and held
    out = oracle.decode(g, pr, syn[378:379], prm, nthreads=1)
    assert out["converged"][0] == 0 and out["legs"][0] == 11
