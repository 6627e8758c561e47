"""Monte-Carlo statistics of the memory experiment (paper Sec. 6.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* block failure: any logical observable wrong, or the decoder did not converge
* 95% Clopper-Pearson interval, from its definition: the lower end is the p at
  which P[X >= x | p] = alpha/2, the upper end the p at which
  P[X <= x | p] = alpha/2, X ~ Binomial(n, p); found by bisection on binomial
  tail sums evaluated term by term in log space.
* per-round rate p_round = 1 - (1 - p)^(1/T).
"""
from __future__ import annotations

import math


def _log_pmf(n: int, i: int, p: float) -> float:
    return (math.lgamma(n + 1) - math.lgamma(i + 1) - math.lgamma(n - i + 1)
            + i * math.log(p) + (n - i) * math.log1p(-p))


def binom_cdf(x: int, n: int, p: float) -> float:
    """P[X <= x]."""
    if x < 0:
        return 0.0
    if x >= n or p <= 0.0:
        return 1.0
    if p >= 1.0:
        return 0.0
    logs = [_log_pmf(n, i, p) for i in range(0, x + 1)]
    m = max(logs)
    return min(1.0, math.exp(m) * sum(math.exp(v - m) for v in logs))


def binom_sf(x: int, n: int, p: float) -> float:
    """P[X >= x]."""
    if x <= 0:
        return 1.0
    return 1.0 - binom_cdf(x - 1, n, p) if x - 1 < n else _tail_top(x, n, p)


def _tail_top(x: int, n: int, p: float) -> float:
    logs = [_log_pmf(n, i, p) for i in range(x, n + 1)]
    m = max(logs)
    return math.exp(m) * sum(math.exp(v - m) for v in logs)


def _bisect(f, lo: float, hi: float, iters: int = 200) -> float:
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if f(mid):
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def clopper_pearson(x: int, n: int, alpha: float = 0.05):
    if n <= 0:
        return 0.0, 1.0
    a2 = alpha / 2
    lo = 0.0 if x == 0 else _bisect(lambda p: _upper_tail(x, n, p) >= a2, 0.0, 1.0)
    hi = 1.0 if x == n else _bisect(lambda p: binom_cdf(x, n, p) <= a2, 0.0, 1.0)
    return lo, hi


def _upper_tail(x: int, n: int, p: float) -> float:
    # P[X >= x] summed directly over the top terms when x is large
    if x > n // 2:
        return _tail_top(x, n, p)
    return 1.0 - binom_cdf(x - 1, n, p)


def per_round(p_block: float, rounds: int) -> float:
    return 1.0 - (1.0 - p_block) ** (1.0 / rounds)


def block_failures(obs_pred_words, obs_words, converged):
    import numpy as np
    wrong = (np.asarray(obs_pred_words) != np.asarray(obs_words)).any(axis=1)
    return wrong | (np.asarray(converged) == 0)
