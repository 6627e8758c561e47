"""Monte-Carlo statistics for the memory experiment (paper Sec. 6.1).

Block failure = any observable predicted wrong or no converged solution.
Intervals are 95 % Clopper-Pearson (beta quantiles); the per-round rate is
1 - (1 - p)^(1/T) and the per-qubit-round rate uses T*k.
"""
from __future__ import annotations

import numpy as np
from scipy.stats import beta


def clopper_pearson(x: int, n: int, alpha: float = 0.05):
    if n <= 0:
        return 0.0, 1.0
    lo = 0.0 if x == 0 else float(beta.ppf(alpha / 2, x, n - x + 1))
    hi = 1.0 if x == n else float(beta.ppf(1 - alpha / 2, x + 1, n - x))
    return lo, hi


def per_round(p: float, rounds: int) -> float:
    return 1.0 - (1.0 - p) ** (1.0 / rounds)


def block_failures(obs_pred: np.ndarray, obs: np.ndarray, converged: np.ndarray) -> np.ndarray:
    return (np.asarray(obs_pred) != np.asarray(obs)).any(axis=1) | (np.asarray(converged) == 0)


def ler_summary(failures: int, shots: int, rounds: int, k: int) -> dict:
    p = failures / shots if shots else 0.0
    lo, hi = clopper_pearson(failures, shots)
    return {"failures": int(failures), "shots": int(shots), "ler": p, "ci95": [lo, hi],
            "per_round": per_round(p, rounds), "per_qubit_round": per_round(p, rounds * k)}


def percentiles(x: np.ndarray, qs=(50, 99, 99.9)) -> dict:
    x = np.asarray(x, dtype=np.float64)
    out = {f"p{q:g}": float(np.percentile(x, q)) for q in qs}
    out["mean"] = float(x.mean())
    out["max"] = float(x.max())
    return out
