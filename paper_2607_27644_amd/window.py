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
