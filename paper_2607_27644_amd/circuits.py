"""Circuit-level detector error models of the paper's memory experiments.

Input generator (like ``workloads``): it builds the matrices H, O and the
priors the decoder is given, and holds none of the sampling or decoding
arithmetic.

Circuit (Sec. 6.1, quantum circuit-level memory; App. "greedy AOD" scheduling,
Table "greedy-aod-gate-schedule"):

* qubits: five data blocks Q_1..Q_5 and the check blocks C^X_1, C^X_2,
  C^Z_1, C^Z_2, each of |G| qubits indexed by the group elements;
* a memory experiment in basis B (X or Z) prepares every data qubit in |+>
  (B = X) or |0> (B = Z), runs T rounds (T = d by default), then measures every
  data qubit in basis B;
* one round: the X part (C^X prepared in |+>, the X-check CNOT layers
  C^X -> Q in table order, C^X measured in X), then the Z part (C^Z prepared in
  |0>, the Z-check layers Q -> C^Z, C^Z measured in Z);
* a table entry (check block, data block, monomial) is one CNOT per group
  element: the permutation matrix of that monomial inside the (check, data)
  block of H_X = [[A,0,B,0,C^T],[0,A,0,B,D^T]] or H_Z = [[C,D,0,0,A^T],
  [0,0,C,D,B^T]] (A = L[a], B = L[b], C = R[c], D = R[d]).  Every block is a
  sum of the disjoint permutations of its three monomials, so the table's
  layers cover H_X and H_Z edge for edge (checked when the layers are built).

Noise (Sec. 6.1): two-qubit depolarizing with probability p after every CNOT,
preparations flipped with probability p, measurement results flipped with
probability p; no single-qubit or idle noise.

Detectors: the basis-B checks.  Layer 0 is the first round's measurement
(deterministic after the data preparation), layer t in 1..T-1 compares rounds
t and t-1, layer T compares the parity of the final data measurements on each
check with round T-1; detector (t, i) is row t*m + i.  Observables: a basis of
the basis-B logical operators (ker H_other modulo the row space of H_B),
read from the final data measurements.

Mechanisms: every fault component with the set of detectors and observables
it flips.  Components with identical sets merge into one mechanism whose
probability is that of an odd number of them firing, 1/2 (1 - prod (1 - 2 p_i));
components that flip nothing are dropped.  Depolarizing noise enters as its 15
Pauli components applied independently with probability q each, where
(1 - 2q)^8 = 1 - 16p/15: every non-identity two-qubit Pauli anticommutes with
8 of the 15, so both channels scale each Pauli's expectation by the same
factor.  Only one error type matters for a memory in basis B (Z errors for
B = X, X errors for B = Z), and the Paulis of a CNOT fall into three classes of
four by the part of that type they carry (control, target, both).

Sets are found by propagating sensitivities backwards through the circuit: for
each qubit, the detectors and observables an error of the tracked type at the
current time would flip.  A CNOT carries Z from target to control and X from
control to target, so going backwards the control's set (Z) or the target's
set (X) is XORed into the other.

Columns are ordered by their first detector (then by the rest of the set), so
a column's first detector layer is its round, as the sliding-window decoder
expects.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import workloads as W

# Table "greedy-aod-gate-schedule": layers of (check block, data block, monomial
# term).  A term "a2" is the second monomial of a as written in Table "ZSZ-LP
# polynomials"; the Z-check table's inverse monomials name the same terms of
# the transposed blocks.
_X_LAYERS: Dict[str, List[str]] = {
    "ZSZ-LP-160": ["1,1,a1 2,2,a1", "1,3,b1 2,4,b1", "1,5,c1", "1,1,a2 2,5,d1", "2,2,a2", "1,5,c2 2,2,a3",
                   "1,5,c3 2,4,b2", "2,4,b3", "1,1,a3", "1,3,b2 2,5,d2", "1,3,b3 2,5,d3"],
    "ZSZ-LP-240": ["1,1,a1 2,2,a1", "1,3,b1 2,4,b1", "1,3,b2 2,4,b2", "1,3,b3 2,4,b3", "1,1,a3 2,2,a3",
                   "1,1,a2 2,2,a2", "1,5,c1", "1,5,c2", "1,5,c3", "2,5,d1", "2,5,d3", "2,5,d2"],
    "ZSZ-LP-320": ["1,1,a1 2,2,a1", "1,3,b1 2,4,b1", "1,5,c1", "1,1,a3 2,5,d1", "1,3,b2 2,2,a3",
                   "1,1,a2 2,4,b2", "1,3,b3 2,2,a2", "2,4,b3", "1,5,c2", "1,5,c3", "2,5,d2", "2,5,d3"],
    "ZSZ-LP-390": ["1,1,a1 2,2,a1", "1,3,b1 2,4,b1", "1,5,c1", "1,3,b3 2,5,d1", "1,1,a2 2,4,b3",
                   "1,1,a3 2,2,a2", "1,3,b2 2,2,a3", "2,4,b2", "1,5,c2", "1,5,c3", "2,5,d2", "2,5,d3"],
    "ZSZ-LP-550": ["1,1,a1 2,2,a1", "1,3,b1 2,4,b1", "1,5,c1", "1,1,a3 2,5,d1", "1,3,b3 2,2,a3",
                   "1,1,a2 2,4,b3", "1,3,b2 2,2,a2", "2,4,b2", "1,5,c3", "1,5,c2", "2,5,d3", "2,5,d2"],
}
_Z_LAYERS: Dict[str, List[str]] = {
    "ZSZ-LP-160": ["1,1,c1 2,3,c1", "1,2,d1 2,4,d1", "1,5,a1", "1,1,c2 2,5,b1", "1,1,c3 2,3,c2",
                   "1,2,d3 2,3,c3", "1,2,d2 2,4,d3", "2,4,d2", "1,5,a2", "1,5,a3", "2,5,b2", "2,5,b3"],
    "ZSZ-LP-240": ["1,1,c1 2,3,c1", "1,2,d1 2,4,d1", "1,5,a1", "1,2,d3 2,5,b1", "1,1,c2 2,4,d3",
                   "1,1,c3 2,3,c2", "1,2,d2 2,3,c3", "2,4,d2", "1,5,a3", "1,5,a2", "2,5,b2", "2,5,b3"],
    "ZSZ-LP-320": ["1,1,c1 2,3,c1", "1,2,d1 2,4,d1", "1,5,a1", "1,5,a3", "2,5,b1", "1,2,d2 2,5,b2", "1,1,c3",
                   "1,1,c2 2,4,d2", "1,2,d3 2,3,c3", "2,3,c2", "1,5,a2 2,4,d3", "2,5,b3"],
    "ZSZ-LP-390": ["1,1,c1 2,3,c1", "1,2,d1 2,4,d1", "1,5,a1", "1,2,d2 2,5,b1", "1,1,c3 2,4,d2", "1,2,d3",
                   "1,1,c2 2,5,b3", "2,5,b2", "1,5,a2", "1,5,a3 2,3,c2", "2,4,d3", "2,3,c3"],
    "ZSZ-LP-550": ["1,1,c1 2,3,c1", "1,2,d1 2,4,d1", "1,5,a1", "1,5,a3", "1,5,a2", "2,5,b1", "1,1,c3 2,5,b3",
                   "1,2,d3 2,5,b2", "1,1,c2", "1,2,d2 2,3,c3", "2,4,d3", "2,3,c2", "2,4,d2"],
}

# code distances (Table 1): the memory experiments run d rounds
DISTANCE = {"ZSZ-LP-160": 10, "ZSZ-LP-240": 12, "ZSZ-LP-320": 14, "ZSZ-LP-390": 16, "ZSZ-LP-550": 18}

# DEM sizes (N_det, N_loc) printed in Table "decoding latency" (d rounds)
PAPER_DEM_SIZES = {"ZSZ-LP-320": (1920, 28992), "ZSZ-LP-390": (2652, 40326), "ZSZ-LP-550": (4180, 63910)}

# (check block, data block) -> transposed block?  Left blocks A, B hold L[a],
# L[b]; right blocks C, D hold R[c], R[d].
_X_BLOCKS = {(1, 1): False, (1, 3): False, (1, 5): True, (2, 2): False, (2, 4): False, (2, 5): True}
_Z_BLOCKS = {(1, 1): False, (1, 2): False, (1, 5): True, (2, 3): False, (2, 4): False, (2, 5): True}

Layer = List[Tuple[np.ndarray, np.ndarray]]  # [(check qubits, data qubits)] of one time step


def layer_pairs(name: str) -> Tuple[int, List[Layer], List[Layer]]:
    """(|G|, X-check layers, Z-check layers).  Each layer is a list of gates,
    each gate a pair of int arrays (check index in 0..2|G|-1, data index in
    0..5|G|-1) of one CNOT per group element."""
    l1, l2, q, a, b, c, d = W.ZSZ_LP_CODES[name]
    G = W.ZSZGroup(l1, l2, q)
    polys = {"a": a, "b": b, "c": c, "d": d}
    g = G.order

    def build(tab, blocks) -> List[Layer]:
        out = []
        for row in tab:
            gates = []
            used_c, used_q = set(), set()
            for ent in row.split():
                cb, qb, term = ent.split(",")
                cb, qb = int(cb), int(qb)
                letter, idx = term[0], int(term[1:]) - 1
                mono = [polys[letter][idx]]
                Mx = G.L(mono) if letter in "ab" else G.R(mono)
                if blocks[(cb, qb)]:
                    Mx = Mx.T
                r, col = np.nonzero(Mx)
                if cb in used_c or qb in used_q:
                    raise ValueError("a layer uses a block twice")
                used_c.add(cb)
                used_q.add(qb)
                gates.append(((cb - 1) * g + r, (qb - 1) * g + col))
            out.append(gates)
        return out

    return g, build(_X_LAYERS[name], _X_BLOCKS), build(_Z_LAYERS[name], _Z_BLOCKS)


def _check_cover(layers: Sequence[Layer], H: np.ndarray):
    A = np.zeros_like(H)
    for layer in layers:
        for ci, qi in layer:
            A[ci, qi] ^= 1
    if not np.array_equal(A, H):
        raise AssertionError("the schedule does not cover the check matrix edge for edge")


def _pack_rows(D: np.ndarray, words: int) -> np.ndarray:
    """uint8 bit rows -> uint64 words, bit b at word b // 64, bit b % 64."""
    P = np.packbits(D, axis=1, bitorder="little")
    out = np.zeros((D.shape[0], words * 8), dtype=np.uint8)
    out[:, : P.shape[1]] = P
    return out.view(np.uint64)


def memory_dem(name: str, basis: str = "X", p: float = 1e-3, rounds: int | None = None) -> W.DEM:
    """Circuit-level DEM of a basis-B memory experiment of ZSZ-LP code `name`."""
    if basis not in ("X", "Z"):
        raise ValueError("basis must be 'X' or 'Z'")
    code = W.zsz_lp(name)
    HX, HZ = code.HX, code.HZ
    g, XL, ZL = layer_pairs(name)
    _check_cover(XL, HX)
    _check_cover(ZL, HZ)
    n, m = 5 * g, 2 * g
    T = DISTANCE[name] if rounds is None else int(rounds)
    if T < 1:
        raise ValueError("rounds must be >= 1")
    Hdet = HX if basis == "X" else HZ
    O1 = W.logical_basis(HX, HZ) if basis == "X" else W.logical_basis(HZ, HX)
    k = O1.shape[0]
    M = m * (T + 1)
    nb = M + k
    words = (nb + 63) // 64
    xa, za = n, n + m                     # first X-check and Z-check ancilla
    track_z = basis == "X"                # the error type that flips the detectors

    S = np.zeros((n + 2 * m, words), dtype=np.uint64)
    rows: List[np.ndarray] = []
    logs: List[float] = []

    def record(v: np.ndarray, log1m2p: float):
        rows.append(np.atleast_2d(v).copy())
        logs.append((log1m2p, rows[-1].shape[0]))

    lp = math.log1p(-2.0 * p)                       # one flip of probability p
    ldep = 4.0 * math.log1p(-16.0 * p / 15.0) / 8.0  # four Pauli components of probability q

    def meas_sets(t: int) -> np.ndarray:
        """sets of the detector-basis check measurements of round t."""
        D = np.zeros((m, nb), dtype=np.uint8)
        D[np.arange(m), t * m + np.arange(m)] = 1
        D[np.arange(m), (t + 1) * m + np.arange(m)] = 1
        return _pack_rows(D, words)

    # final data measurement in basis B: flips the last detector layer of its
    # checks and the observables on it
    D = np.zeros((n, nb), dtype=np.uint8)
    D[:, T * m:(T + 1) * m] = Hdet.T
    D[:, M:] = O1.T
    S[:n] = _pack_rows(D, words)
    record(S[:n], lp)                               # final measurement flips

    for t in range(T - 1, -1, -1):
        # ---- Z part, backwards: measurement, CNOT layers, preparation
        if track_z:
            S[za:za + m] = 0                        # Z errors do not flip Z measurements
        else:
            S[za:za + m] = meas_sets(t)
            record(S[za:za + m], lp)                # measurement flips
        for layer in reversed(ZL):
            for ci, qi in layer:
                anc, dat = za + ci, qi              # CNOT dat -> anc
                sc, st = S[dat], S[anc]
                record(sc, ldep)
                record(st, ldep)
                record(sc ^ st, ldep)
                if track_z:
                    S[anc] ^= S[dat]                # Z on the target reaches the control
                else:
                    S[dat] ^= S[anc]                # X on the control reaches the target
        if not track_z:
            record(S[za:za + m], lp)                # |0> prepared as |1>
        S[za:za + m] = 0
        # ---- X part, backwards
        if track_z:
            S[xa:xa + m] = meas_sets(t)
            record(S[xa:xa + m], lp)
        else:
            S[xa:xa + m] = 0
        for layer in reversed(XL):
            for ci, qi in layer:
                anc, dat = xa + ci, qi              # CNOT anc -> dat
                sc, st = S[anc], S[dat]
                record(sc, ldep)
                record(st, ldep)
                record(sc ^ st, ldep)
                if track_z:
                    S[dat] ^= S[anc]                # Z on the target reaches the control
                else:
                    S[anc] ^= S[dat]                # X on the control reaches the target
        if track_z:
            record(S[xa:xa + m], lp)                # |+> prepared as |->
        S[xa:xa + m] = 0
    record(S[:n], lp)                               # data preparation flips

    R = np.vstack(rows)
    L = np.concatenate([np.full(cnt, v) for v, cnt in logs])
    keep = R.any(axis=1)
    R, L = R[keep], L[keep]
    uniq, inv = np.unique(R, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    tot = np.bincount(inv, weights=L, minlength=uniq.shape[0])
    priors = -np.expm1(tot) / 2.0

    bits = np.unpackbits(uniq.view(np.uint8), axis=1, bitorder="little")[:, :nb]
    det = bits[:, :M]
    first = np.where(det.any(axis=1), det.argmax(axis=1), M)
    order = np.lexsort((np.arange(uniq.shape[0]), first))
    H = np.ascontiguousarray(det[order].T)
    O = np.ascontiguousarray(bits[order, M:].T)
    dem = W.DEM(f"{name}/circuit-{basis}/T={T}/p={p:g}", H, O, priors[order], rounds=T)
    return dem
