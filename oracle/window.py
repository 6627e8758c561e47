"""Sliding-window decoding, oracle version (TEST INFRASTRUCTURE ONLY).

The paper argues that its Relay-BP configuration is fast enough for
sliding-window decoding with a commit region of one round (Sec. 6.1, latency
discussion).  The windowing written out here, for a detector error model whose
detectors come in rounds of m (round-major rows):

  * window k starts at round s = k c and covers rounds [s, min(s + w, T));
    the last window is the first one that reaches round T;
  * its mechanisms are the columns whose first detector lies in the window
    (columns touching an earlier round were committed before); a column that
    also touches later rounds enters with its in-window rows only;
  * its syndrome is the current syndrome on the window's rows; it is decoded
    with Relay-BP (``oracle.decode``) on the window's matrix and priors;
  * it commits the decoded mechanisms whose first detector lies in rounds
    [s, s + c) (the last window commits all of its mechanisms): each committed
    mechanism is set in the correction, and its full column of H and of O is
    XORed into the syndrome and the predicted observables;
  * a shot is converged when every window converged.

Plain numpy loops and the oracle decoder; shares nothing with the product.
"""
from __future__ import annotations

import numpy as np

from . import Graph, RelayParams, decode


def _unpack(words: np.ndarray, nbits: int) -> np.ndarray:
    b = np.unpackbits(np.ascontiguousarray(words, dtype=np.uint32).view(np.uint8), axis=1, bitorder="little")
    return b[:, :nbits].astype(np.uint8)


def _pack(bits: np.ndarray) -> np.ndarray:
    r, c = bits.shape
    W = max((c + 31) // 32, 1)
    pad = np.zeros((r, W * 32), dtype=np.uint8)
    pad[:, :c] = bits
    return np.packbits(pad, axis=1, bitorder="little").view(np.uint32).reshape(r, W).copy()


def windows(H: np.ndarray, m: int, window: int, commit: int):
    """[(first round, rounds, columns, commit mask)] of the sliding windows."""
    M, N = H.shape
    assert M % m == 0 and 1 <= commit <= window
    T = M // m
    first_row = np.full(N, -1)
    for j in range(N):
        nz = np.flatnonzero(H[:, j])
        if nz.size:
            first_row[j] = nz[0]
    out = []
    s = 0
    while True:
        last = s + window >= T
        r = min(window, T - s)
        cols = [j for j in range(N) if s * m <= first_row[j] < (s + r) * m]
        cm = [True if last else first_row[j] < (s + commit) * m for j in cols]
        out.append((s, r, np.array(cols, dtype=np.int64), np.array(cm, dtype=bool)))
        if last:
            return out
        s += commit


def decode_windowed(H: np.ndarray, O: np.ndarray, priors: np.ndarray, syndromes: np.ndarray, m: int, window: int,
                    commit: int, params: RelayParams, nthreads: int | None = None) -> dict:
    """Windowed Relay-BP of packed syndromes uint32[shots][ceil(M/32)]: packed
    corrections and predicted observables, converged flags, total iterations."""
    H = np.asarray(H, dtype=np.uint8)
    O = np.asarray(O, dtype=np.uint8)
    M, N = H.shape
    shots = syndromes.shape[0]
    syn = _unpack(syndromes, M)
    corr = np.zeros((shots, N), dtype=np.uint8)
    obs = np.zeros((shots, O.shape[0]), dtype=np.uint8)
    conv = np.ones(shots, dtype=bool)
    iters = np.zeros(shots, dtype=np.int64)
    for s, r, cols, cm in windows(H, m, window, commit):
        rows = slice(s * m, (s + r) * m)
        Hw = H[rows][:, cols]
        g = Graph(Hw, np.zeros((0, cols.size), dtype=np.uint8))
        res = decode(g, priors[cols], _pack(syn[:, rows]), params, nthreads=nthreads)
        ew = _unpack(res["corrections"], cols.size)
        conv &= res["converged"] == 1
        iters += res["iters"]
        for t, j in enumerate(cols):
            if not cm[t]:
                continue
            hit = ew[:, t] == 1
            if hit.any():
                corr[hit, j] = 1
                syn[hit] ^= H[:, j]
                obs[hit] ^= O[:, j]
    return {"corrections": _pack(corr), "obs_pred": _pack(obs), "converged": conv.astype(np.uint8),
            "iters": iters, "residual": _pack(syn)}
