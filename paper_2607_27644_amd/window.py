"""Sliding-window decoding on the GPU (paper Sec. 6.1, latency discussion:
sliding-window decoding with a commit region of c rounds).

For a detector error model whose rows come in rounds of m detectors
(round-major), window k covers rounds [k c, min(k c + w, T)); its mechanisms
are the columns whose first detector lies in the window (a column reaching
past the window keeps only its in-window rows), it is decoded with Relay-BP on
the current syndrome of its rows, and it commits the decoded mechanisms whose
first detector lies in its first c rounds (the last window commits everything).
A committed mechanism enters the correction and its columns of H and O are
XORed into the running syndrome and the predicted observables.  A shot is
converged when every window converged.

Every window decode is ``rbp_decode`` on a handle of the window matrix; the
syndrome slices and commits are ``rbp_bits_extract`` and ``rbp_window_commit``.

Parallel-window decoding (``ParallelWindowDecoder``; the paper points to it
for shots whose decoding outlasts the syndrome stream) works in two layers of
independent windows over the detector layers (rounds of m rows).  Layer A:
window k has a core of `core` layers from k P (P = core + gap) and `buffer`
layers on each side, takes every column with a detector in it (cut to its
rows: open on both sides) and commits the columns that start in its core.
Layer B: window k covers the gap [k P + core, (k+1) P) with the columns that
start there; a row above the gap that meets exactly one of them fixes that
column to the row's syndrome bit (committed first, via ``rbp_bits_gather``),
and rows above that meet two or more stay in the window; it commits all its
columns.  The windows of a layer all read the syndrome as it was before the
layer's commits; windows with the same matrix and priors (the interior ones
of a repetitive model) are decoded together in one launch, one shot per
(window, shot) pair.  A shot is converged when every window converged and no
syndrome is left (``rbp_window_residual``).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from . import rbp


@dataclasses.dataclass
class Window:
    start: int              # first round
    rounds: int
    cols: np.ndarray        # full-model columns of the window, in window order
    commit: np.ndarray      # bool per window column
    code: rbp.Code
    cmap: torch.Tensor      # int32 [n]: full column if committed, else -1


class SlidingWindowDecoder:
    def __init__(self, H: np.ndarray, O: np.ndarray, m: int, window: int, commit: int):
        H = np.asarray(H, dtype=np.uint8)
        O = np.asarray(O, dtype=np.uint8)
        M, N = H.shape
        if M % m:
            raise ValueError("the detector count must be a multiple of the detectors per round")
        if not 1 <= commit <= window:
            raise ValueError("need 1 <= commit <= window")
        self.M, self.N, self.m, self.T = M, N, m, M // m
        self.window, self.commit = window, commit
        self.full = rbp.Code(H, O)
        self.k = O.shape[0]
        any_row = H.any(axis=0)
        first = np.where(any_row, H.argmax(axis=0), -1)  # first detector of each column
        self.windows: List[Window] = []
        s = 0
        while True:
            last = s + window >= self.T
            r = min(window, self.T - s)
            cols = np.flatnonzero((first >= s * m) & (first < (s + r) * m))
            cm = np.ones(cols.size, dtype=bool) if last else first[cols] < (s + commit) * m
            Hw = H[s * m:(s + r) * m][:, cols]
            code = rbp.Code(Hw, np.zeros((0, cols.size), dtype=np.uint8))
            cmap = torch.from_numpy(np.where(cm, cols, -1).astype(np.int32)).cuda()
            self.windows.append(Window(s, r, cols, cm, code, cmap))
            if last:
                break
            s += commit

    def decode(self, priors: np.ndarray, syndromes: torch.Tensor, params: rbp.RelayParams, stream=None):
        """Windowed decode of syndromes int32 [shots][ceil(M/32)] -> (corrections,
        predicted observables, accumulated per-shot statistics)."""
        priors = np.asarray(priors, dtype=np.float64)
        shots = syndromes.shape[0]
        dev = syndromes.device
        syn = syndromes.clone()
        corr = torch.zeros((shots, rbp.words(self.N)), dtype=torch.int32, device=dev)
        obs = torch.zeros((shots, max(rbp.words(self.k), 1)), dtype=torch.int32, device=dev)
        acc = torch.empty((shots, 32), dtype=torch.uint8, device=dev)
        bufs = {}
        for i, w in enumerate(self.windows):
            nb = w.rounds * self.m
            n = w.cols.size
            key = (nb, n)
            if key not in bufs:
                bufs[key] = (torch.empty((shots, rbp.words(nb)), dtype=torch.int32, device=dev),
                             torch.empty((shots, rbp.words(n)), dtype=torch.int32, device=dev),
                             torch.empty((shots, 1), dtype=torch.int32, device=dev),
                             torch.empty((shots, 32), dtype=torch.uint8, device=dev))
            syn_w, cw, ow, st = bufs[key]
            rbp.bits_extract(syn, w.start * self.m, nb, syn_w, stream=stream)
            w.code.decode(priors[w.cols], syn_w, params, stream=stream, out=(cw, ow, st))
            rbp.window_commit(self.full, cw, w.cmap, n, syn, obs, corr, st, acc, first=(i == 0), stream=stream)
        return corr, obs, acc

    def close(self):
        for w in self.windows:
            w.code.close()
        self.full.close()


@dataclasses.dataclass
class PWindow:
    rows: np.ndarray        # full-model rows of the window, in window order
    cols: np.ndarray        # full-model columns of the window, in window order
    cmap: torch.Tensor      # int32 [n]: full column if committed, else -1
    key: bytes              # the window matrix (windows with equal keys share a handle)
    fix_rows: torch.Tensor  # int32: rows that fix single columns (layer B), may be empty
    fix_map: torch.Tensor   # int32: the column each of them fixes


def parallel_layout(H: np.ndarray, m: int, core: int, buffer: int, gap: int):
    """The two layers of parallel windows (host only): [layer A, layer B], each
    a list of (rows, columns, commit mask, fixing rows, fixed columns) as numpy
    arrays, rows and columns ascending within their parts."""
    H = np.asarray(H, dtype=np.uint8)
    M, N = H.shape
    if M % m:
        raise ValueError("the detector count must be a multiple of the detectors per round")
    if core < 1 or buffer < 0 or gap < 1:
        raise ValueError("need core >= 1, buffer >= 0, gap >= 1")
    has = H.any(axis=0)
    first = np.where(has, H.argmax(axis=0) // m, -1)
    last = np.where(has, (M - 1 - H[::-1].argmax(axis=0)) // m, -1)
    L, P = M // m, core + gap
    none = np.zeros(0, dtype=np.int64)
    A, B = [], []
    for c0 in range(0, L, P):
        c1 = min(c0 + core, L)
        r0, r1 = max(0, c0 - buffer), min(L, c1 + buffer)
        cols = np.flatnonzero(has & (first < r1) & (last >= r0))
        commit = (first[cols] >= c0) & (first[cols] < c1)
        A.append((np.arange(r0 * m, r1 * m), cols, commit, none, none))
        g0, g1 = c1, min(c0 + P, L)
        if g0 >= g1:
            continue
        cols = np.flatnonzero(has & (first >= g0) & (first < g1))
        arows = np.flatnonzero(H[g1 * m:, cols].any(axis=1)) + g1 * m
        fixed_r, fixed_c = [], []
        for i in arows:
            hit = cols[H[i, cols] == 1]
            if hit.size == 1 and hit[0] not in fixed_c:
                fixed_r.append(i)
                fixed_c.append(hit[0])
        cols = np.setdiff1d(cols, np.array(fixed_c, dtype=np.int64))
        keep = [i for i in arows if int(H[i, cols].sum()) >= 2]
        rows = np.concatenate([np.arange(g0 * m, g1 * m), np.array(keep, dtype=np.int64)])
        B.append((rows, cols, np.ones(cols.size, dtype=bool), np.array(fixed_r, dtype=np.int64),
                  np.array(fixed_c, dtype=np.int64)))
    return [A, B]


class ParallelWindowDecoder:
    def __init__(self, H: np.ndarray, O: np.ndarray, m: int, core: int, buffer: int, gap: int):
        H = np.asarray(H, dtype=np.uint8)
        O = np.asarray(O, dtype=np.uint8)
        M, N = H.shape
        layout = parallel_layout(H, m, core, buffer, gap)
        self.H, self.M, self.N, self.m, self.k = H, M, N, m, O.shape[0]
        self.full = rbp.Code(H, O)
        self.codes = {}
        self.layers: List[List[PWindow]] = [[], []]
        dev = torch.device("cuda")
        for li, layer in enumerate(layout):
            for rows, cols, commit, fixed_r, fixed_c in layer:
                fr = torch.from_numpy(fixed_r.astype(np.int32)).to(dev)
                fc = torch.from_numpy(fixed_c.astype(np.int32)).to(dev)
                self.layers[li].append(self._window(rows, cols, commit, fr, fc))

    def _window(self, rows, cols, commit, fix_rows, fix_map) -> PWindow:
        Hw = np.ascontiguousarray(self.H[rows][:, cols])
        key = np.asarray(Hw.shape, np.int64).tobytes() + np.packbits(Hw, axis=1).tobytes()
        if key not in self.codes:
            self.codes[key] = rbp.Code(Hw, np.zeros((0, cols.size), dtype=np.uint8))
        cmap = torch.from_numpy(np.where(commit, cols, -1).astype(np.int32)).cuda()
        return PWindow(np.asarray(rows, np.int32), cols, cmap, key, fix_rows, fix_map)

    def decode(self, priors: np.ndarray, syndromes: torch.Tensor, params: rbp.RelayParams, stream=None):
        """Parallel-window decode of syndromes int32 [shots][ceil(M/32)] ->
        (corrections, predicted observables, accumulated per-shot statistics)."""
        priors = np.asarray(priors, dtype=np.float64)
        shots = syndromes.shape[0]
        dev = syndromes.device
        syn = syndromes.clone()
        corr = torch.zeros((shots, rbp.words(self.N)), dtype=torch.int32, device=dev)
        obs = torch.zeros((shots, max(rbp.words(self.k), 1)), dtype=torch.int32, device=dev)
        acc = torch.empty((shots, 32), dtype=torch.uint8, device=dev)
        first = True
        for layer in self.layers:
            for w in layer:
                n = w.fix_rows.numel()
                if n:
                    bits = torch.empty((shots, rbp.words(n)), dtype=torch.int32, device=dev)
                    rbp.bits_gather(syn, w.fix_rows, bits, stream=stream)
                    rbp.window_commit(self.full, bits, w.fix_map, n, syn, obs, corr, stream=stream)
            groups = {}
            for w in layer:
                groups.setdefault((w.key, priors[w.cols].tobytes()), []).append(w)
            decoded = []
            for (key, _), ws in groups.items():
                nb = int(ws[0].rows.size)
                stack = torch.empty((len(ws) * shots, rbp.words(nb)), dtype=torch.int32, device=dev)
                for i, w in enumerate(ws):
                    part = stack[i * shots:(i + 1) * shots]
                    r0 = int(w.rows[0])
                    if np.array_equal(w.rows, np.arange(r0, r0 + nb)):
                        rbp.bits_extract(syn, r0, nb, part, stream=stream)
                    else:
                        rbp.bits_gather(syn, torch.from_numpy(w.rows).to(dev), part, stream=stream)
                out = self.codes[key].decode(priors[ws[0].cols], stack, params, stream=stream)
                decoded.append((ws, out))
            for ws, (cw, ow, st) in decoded:
                for i, w in enumerate(ws):
                    sl = slice(i * shots, (i + 1) * shots)
                    rbp.window_commit(self.full, cw[sl], w.cmap, w.cols.size, syn, obs, corr, st[sl], acc,
                                      first=first, stream=stream)
                    first = False
        rbp.window_residual(syn, acc, stream=stream)
        return corr, obs, acc

    def close(self):
        for c in self.codes.values():
            c.close()
        self.full.close()
