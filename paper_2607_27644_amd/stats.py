"""Monte-Carlo statistics for the memory experiment (paper Sec. 6.1).

Block failure = any observable predicted wrong or no converged solution.
Intervals are 95 % Clopper-Pearson (beta quantiles); the per-round rate is
1 - (1 - p)^(1/T) and the per-qubit-round rate uses T*k.  Low-p extrapolation
uses the phenomenological form p^(d_circ/2) exp(c0 + c1 p + c2 p^2) that the
paper fits to its sub-threshold points (Sec. 6.1, Fig. "LER vs kd^2/n").
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq
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


def fit_ler(p, pbar, d_circ: float, failures=None):
    """Fit pbar = p^(d_circ/2) * exp(c0 + c1 p + c2 p^2) (Sec. 6.1).

    In logs the model is linear in (c0, c1, c2):
        log pbar - (d_circ/2) log p = c0 + c1 p + c2 p^2,
    so the fit is a weighted linear least-squares problem.  With failure counts
    given, each point is weighted by its count (the inverse of the binomial
    variance of log pbar, 1/failures, to first order); otherwise all weights are
    1.  Points with pbar <= 0 (no failures) carry no information in logs and
    are dropped.  Returns (c0, c1, c2); needs at least three usable points.
    """
    p = np.asarray(p, dtype=np.float64)
    pbar = np.asarray(pbar, dtype=np.float64)
    w = np.ones_like(p) if failures is None else np.asarray(failures, dtype=np.float64)
    keep = (pbar > 0) & (p > 0) & (w > 0)
    if int(keep.sum()) < 3:
        raise ValueError("the LER fit needs at least three points with failures")
    p, pbar, w = p[keep], pbar[keep], w[keep]
    y = np.log(pbar) - 0.5 * d_circ * np.log(p)
    A = np.stack([np.ones_like(p), p, p * p], axis=1)
    sw = np.sqrt(w)
    c, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    return float(c[0]), float(c[1]), float(c[2])


def ler_model(p, c, d_circ: float):
    """pbar(p) = p^(d_circ/2) exp(c0 + c1 p + c2 p^2) for fitted c = (c0, c1, c2)."""
    p = np.asarray(p, dtype=np.float64)
    return p ** (0.5 * d_circ) * np.exp(c[0] + c[1] * p + c[2] * p * p)


def bpsk_awgn_capacity(sigma: float, nodes: int = 200) -> float:
    """Capacity (bits per channel use) of BPSK over AWGN with noise sigma:
    1 - E[log2(1 + exp(-L))], L ~ N(2/sigma^2, 4/sigma^2) the LLR of a received
    +1 (App. "classical channel coding", eq. "bpsk awgn capacity"), by
    Gauss-Hermite quadrature."""
    x, w = np.polynomial.hermite_e.hermegauss(nodes)
    mu, sd = 2.0 / sigma ** 2, 2.0 / sigma
    L = mu + sd * x
    return float(1.0 - np.sum(w * np.logaddexp(0.0, -L)) / np.sqrt(2.0 * np.pi) / np.log(2.0))


def shannon_limit_db(rate: float) -> float:
    """E_b/N_0 (dB) at which the BPSK-AWGN capacity equals the code rate."""
    def gap(db):
        sigma = np.sqrt(1.0 / (2.0 * rate * 10.0 ** (db / 10.0)))
        return bpsk_awgn_capacity(sigma) - rate
    return float(brentq(gap, -10.0, 20.0, xtol=1e-10))
