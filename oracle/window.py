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


# ---------------------------------------------------------------------------
# Parallel-window decoding (the paper points to it for the rare shots whose
# decoding outlasts the syndrome stream, Sec. 6.1 latency discussion), in two
# layers over the detector layers 0..L-1 (L = M / m):
#
#   * layer A: window k has a core of `core` layers starting at k P
#     (P = core + gap) and `buffer` layers on each side; its mechanisms are all
#     columns with a detector in the window, cut to the window's rows (open
#     boundaries on both sides); it commits those whose first detector lies in
#     its core;
#   * layer B: window k covers the gap [k P + core, (k+1) P); its mechanisms
#     are the columns whose first detector lies in the gap.  A row above the
#     gap (in the next core, already decoded) that meets exactly one of them
#     fixes that column: it is committed with the row's current syndrome bit
#     before the gap is decoded (a parity check on one unknown determines it),
#     and leaves the window.  The window's rows are the gap's rows and the
#     rows above it that meet two or more of the remaining columns; it commits
#     all remaining columns;
#   * all windows of a layer decode the syndrome as it stood before that
#     layer's commits (they are independent); then the layer commits.
# Every column with a detector is committed once: cores and gaps tile the
# layers.  A shot is converged when every window converged and the syndrome
# left after both layers is zero.
# ---------------------------------------------------------------------------
def parallel_windows(H: np.ndarray, m: int, core: int, buffer: int, gap: int):
    """[layer A, layer B]: A windows (rows, columns, commit mask); B windows
    (rows, columns, commit mask, fixed [(row, column)])."""
    M, N = H.shape
    assert M % m == 0 and core >= 1 and buffer >= 0 and gap >= 1
    L = M // m
    first = np.full(N, -1)
    last = np.full(N, -1)
    for j in range(N):
        nz = np.flatnonzero(H[:, j])
        if nz.size:
            first[j] = nz[0] // m
            last[j] = nz[-1] // m
    P = core + gap
    A, B = [], []
    k = 0
    while k * P < L:
        c0, c1 = k * P, min(k * P + core, L)
        r0, r1 = max(0, c0 - buffer), min(L, c1 + buffer)
        cols = [j for j in range(N) if first[j] >= 0 and first[j] < r1 and last[j] >= r0]
        A.append((np.arange(r0 * m, r1 * m), np.array(cols, dtype=np.int64),
                  np.array([c0 <= first[j] < c1 for j in cols], dtype=bool)))
        g0, g1 = c1, min((k + 1) * P, L)
        if g0 < g1:
            cols = [j for j in range(N) if first[j] >= 0 and g0 <= first[j] < g1]
            fixed = []
            above = [i for i in range(g1 * m, M) if H[i, cols].any()]
            for i in above:
                hit = [j for j in cols if H[i, j]]
                if len(hit) == 1 and hit[0] not in [f[1] for f in fixed]:
                    fixed.append((i, hit[0]))
            fixed_cols = set(f[1] for f in fixed)
            cols = [j for j in cols if j not in fixed_cols]
            keep = [i for i in above if int(H[i, cols].sum()) >= 2]
            rows = np.concatenate([np.arange(g0 * m, g1 * m), np.array(keep, dtype=np.int64)])
            B.append((rows, np.array(cols, dtype=np.int64), np.ones(len(cols), dtype=bool), fixed))
        k += 1
    return [A, B]


def decode_parallel(H: np.ndarray, O: np.ndarray, priors: np.ndarray, syndromes: np.ndarray, m: int, core: int,
                    buffer: int, gap: int, params: RelayParams, nthreads: int | None = None) -> dict:
    """Two-layer parallel-window Relay-BP of packed syndromes; the result keys
    of ``decode_windowed``."""
    H = np.asarray(H, dtype=np.uint8)
    O = np.asarray(O, dtype=np.uint8)
    M, N = H.shape
    shots = syndromes.shape[0]
    syn = _unpack(syndromes, M)
    corr = np.zeros((shots, N), dtype=np.uint8)
    obs = np.zeros((shots, O.shape[0]), dtype=np.uint8)
    conv = np.ones(shots, dtype=bool)
    iters = np.zeros(shots, dtype=np.int64)
    def commit(hit, j):
        if hit.any():
            corr[hit, j] = 1
            syn[hit] ^= H[:, j]
            obs[hit] ^= O[:, j]

    for layer in parallel_windows(H, m, core, buffer, gap):
        # columns fixed by a single-column row above a gap, from the current syndrome
        for w in layer:
            if len(w) == 4:
                bits = [(syn[:, i] == 1, j) for i, j in w[3]]
                for hit, j in bits:
                    commit(hit, j)
        decoded = []
        for w in layer:  # every window reads the same syndrome
            rows, cols, cm = w[0], w[1], w[2]
            g = Graph(H[rows][:, cols], np.zeros((0, cols.size), dtype=np.uint8))
            res = decode(g, priors[cols], _pack(syn[:, rows]), params, nthreads=nthreads)
            decoded.append((cols, cm, _unpack(res["corrections"], cols.size)))
            conv &= res["converged"] == 1
            iters += res["iters"]
        for cols, cm, ew in decoded:
            for t, j in enumerate(cols):
                if cm[t]:
                    commit(ew[:, t] == 1, j)
    conv &= ~syn.any(axis=1)
    return {"corrections": _pack(corr), "obs_pred": _pack(obs), "converged": conv.astype(np.uint8),
            "iters": iters, "residual": _pack(syn)}
