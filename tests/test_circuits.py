"""Pins of the circuit-level detector error models.

* The DEM sizes (N_det, N_loc) of the d-round memory circuits equal the ones
  the paper prints in Table "decoding latency" for ZSZ-LP-320, -390 and -550,
  in both memory bases.
* A forward Pauli-frame simulation of the same circuit, written here
  independently of the builder's backward propagation, injects every fault
  component (all 15 Paulis after each CNOT, both X and Z frames tracked,
  preparation and measurement flips) one at a time; the set of non-empty
  (detector, observable) flip patterns must be exactly the DEM's columns, and
  the probabilities combined per pattern must equal the DEM's priors.
* Structure: the schedule covers H_X and H_Z edge for edge; every column's
  first detector layer is its round or the next (a fault acts on the
  detectors of the round it happens in or later).
"""
import itertools
import math

import numpy as np
import pytest

from paper_2607_27644_amd import circuits as C
from paper_2607_27644_amd import workloads as W


@pytest.mark.parametrize("name", ["ZSZ-LP-320", "ZSZ-LP-390", "ZSZ-LP-550"])
@pytest.mark.parametrize("basis", ["X", "Z"])
def test_dem_sizes_match_the_paper(name, basis):
    dem = C.memory_dem(name, basis, 1e-3)
    assert (dem.M, dem.N) == C.PAPER_DEM_SIZES[name]
    assert dem.k == W.ZSZ_LP_NK[name][1]


def test_schedule_covers_the_checks():
    for name in C.DISTANCE:
        code = W.zsz_lp(name)
        g, XL, ZL = C.layer_pairs(name)
        for layers, H in ((XL, code.HX), (ZL, code.HZ)):
            A = np.zeros_like(H)
            for layer in layers:
                qubits = np.concatenate([np.concatenate([c + 10 ** 6, q]) for c, q in layer])
                assert len(np.unique(qubits)) == len(qubits)  # a layer touches each qubit once
                for c, q in layer:
                    A[c, q] ^= 1
            assert np.array_equal(A, H)


def forward_patterns(name, basis, T, p):
    """Every fault component of the circuit propagated forward on its own.
    Returns (patterns uint8 [R, M + k], probabilities [R])."""
    code = W.zsz_lp(name)
    g, XL, ZL = C.layer_pairs(name)
    n, m = 5 * g, 2 * g
    xa, za = n, n + m
    nq = n + 2 * m
    # circuit in time order
    ops = [("prep", np.arange(n), "X" if basis == "X" else "Z", None)]
    for t in range(T):
        ops.append(("prep", xa + np.arange(m), "X", None))
        for layer in XL:
            for c, q in layer:
                ops.append(("cnot", xa + c, q, None))
        ops.append(("meas", xa + np.arange(m), "X", ("X", t)))
        ops.append(("prep", za + np.arange(m), "Z", None))
        for layer in ZL:
            for c, q in layer:
                ops.append(("cnot", q, za + c, None))
        ops.append(("meas", za + np.arange(m), "Z", ("Z", t)))
    ops.append(("meas", np.arange(n), basis, ("D", 0)))
    qdep = 0.5 - 0.5 * (1.0 - 16.0 * p / 15.0) ** 0.125
    paulis = [pq for pq in itertools.product(range(4), repeat=2) if pq != (0, 0)]  # 0 I, 1 X, 2 Y, 3 Z
    # fault rows: (op index, kind, payload, probability)
    faults = []
    for oi, op in enumerate(ops):
        if op[0] == "prep":
            for qb in op[1]:
                faults.append((oi, "flip", qb, p))
        elif op[0] == "cnot":
            for c, tq in zip(op[1], op[2]):
                for pc, pt in paulis:
                    faults.append((oi, "pauli", (c, tq, pc, pt), qdep))
        else:
            for j in range(len(op[1])):
                faults.append((oi, "mflip", j, p))
    R = len(faults)
    by_op = {}
    for r, f in enumerate(faults):
        by_op.setdefault(f[0], []).append((r, f))
    fx = np.zeros((R, nq), dtype=np.uint8)
    fz = np.zeros((R, nq), dtype=np.uint8)
    rec = {}
    for oi, op in enumerate(ops):
        kind = op[0]
        if kind == "prep":
            fx[:, op[1]] = 0
            fz[:, op[1]] = 0
        elif kind == "cnot":
            c, tq = op[1], op[2]
            fx[:, tq] ^= fx[:, c]
            fz[:, c] ^= fz[:, tq]
        else:
            flips = (fz if op[2] == "X" else fx)[:, op[1]].copy()
        for r, f in by_op.get(oi, []):
            if f[1] == "flip":
                (fz if op[2] == "X" else fx)[r, f[2]] ^= 1
            elif f[1] == "pauli":
                c, tq, pc, pt = f[2]
                fx[r, c] ^= pc in (1, 2)
                fz[r, c] ^= pc in (2, 3)
                fx[r, tq] ^= pt in (1, 2)
                fz[r, tq] ^= pt in (2, 3)
            else:
                flips[r, f[2]] ^= 1
        if kind == "meas":
            rec[op[3]] = flips
    Hd = code.HX if basis == "X" else code.HZ
    O1 = W.logical_basis(code.HX, code.HZ) if basis == "X" else W.logical_basis(code.HZ, code.HX)
    det = [rec[(basis, 0)]]
    for t in range(1, T):
        det.append(rec[(basis, t)] ^ rec[(basis, t - 1)])
    data = rec[("D", 0)].astype(np.int64)
    det.append(((data @ Hd.T.astype(np.int64)) % 2).astype(np.uint8) ^ rec[(basis, T - 1)])
    obs = ((data @ O1.T.astype(np.int64)) % 2).astype(np.uint8)
    return np.concatenate(det + [obs], axis=1), np.array([f[3] for f in faults])


@pytest.mark.parametrize("basis", ["X", "Z"])
@pytest.mark.parametrize("T", [1, 3])
def test_forward_frame_simulation_gives_the_dem(basis, T):
    name, p = "ZSZ-LP-160", 2e-3
    dem = C.memory_dem(name, basis, p, rounds=T)
    pat, pr = forward_patterns(name, basis, T, p)
    nz = pat.any(axis=1)
    pat, pr = pat[nz], pr[nz]
    uniq, inv = np.unique(pat, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    comb = -np.expm1(np.bincount(inv, weights=np.log1p(-2.0 * pr), minlength=uniq.shape[0])) / 2.0
    cols = np.concatenate([dem.H, dem.O], axis=0).T
    assert cols.shape == uniq.shape
    # match columns to patterns
    key = {bytes(np.packbits(r)): i for i, r in enumerate(uniq)}
    idx = np.array([key[bytes(np.packbits(c))] for c in cols])
    assert len(set(idx.tolist())) == len(idx)
    np.testing.assert_allclose(dem.priors, comb[idx], rtol=1e-12, atol=0)


def test_column_order_and_rounds():
    dem = C.memory_dem("ZSZ-LP-160", "X", 1e-3)
    m = 64
    first = dem.H.argmax(axis=0)
    assert dem.H.any(axis=0).all()
    assert np.all(np.diff(first) >= 0)
    assert dem.M == m * (C.DISTANCE["ZSZ-LP-160"] + 1)
    # every column spans at most two consecutive detector layers
    last = dem.H.shape[0] - 1 - dem.H[::-1].argmax(axis=0)
    assert np.all(last // m - first // m <= 1)
    # every mechanism holds at least one class of four Pauli components, of
    # combined probability 1/2 (1 - (1 - 16p/15)^(1/2)), or a flip of probability p
    p = 1e-3
    q4 = 0.5 * (1.0 - math.sqrt(1.0 - 16.0 * p / 15.0))
    assert dem.priors.min() >= q4 * (1 - 1e-12) and dem.priors.max() < 0.5
