"""Seeded input generators: codes, detector error models, observables and priors.

This module builds the *inputs* of the Monte-Carlo decoding path; it holds none of
the sampling or decoding arithmetic.  Both the HIP path and the CPU oracle take
their matrices from here, so it imports nothing else from this package except
``circuits`` (circuit-level models, built on this module) for the named
circuit workloads.

Contents
--------
* ZSZ group law and regular representations (paper Sec. 2.2, eqs. "ZSZ
  presentation", "push-through relations"; App. B eq. "regular representation";
  element indexing x^a y^b -> a*l2 + b from App. C.4).
* The 5-block CSS matrices H_X, H_Z of a ZSZ-LP code (Sec. 2.1 eq. "5-block
  H_X,H_Z", Sec. 2.4 with A=L[a], B=L[b], C=R[c], D=R[d]) for every code of
  Table "ZSZ-LP polynomials" and Table "more ZSZ-LP codes".
* A seeded hypergraph-product code from a (3,6)-regular configuration-model seed
  code (Sec. 2.3 describes the configuration model), used for large instances.
* GF(2) rank / kernel / logical basis (k = n - rk H_X - rk H_Z, Sec. 2.1).
* Code-capacity and phenomenological detector error models over T rounds
  (the DEM notion of Sec. 6.1, Table "decoding latency").
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Dict, List, Sequence, Tuple

import numpy as np

Mono = Tuple[int, int]  # x^i y^j

# ---------------------------------------------------------------------------
# Code tables.  Table "ZSZ-LP polynomials" (Sec. 2.4) and Table "more ZSZ-LP
# codes" (App. A): (l1, l2, q, a, b, c, d), each polynomial a list of monomials.
# ---------------------------------------------------------------------------
ZSZ_LP_CODES: Dict[str, Tuple[int, int, int, List[Mono], List[Mono], List[Mono], List[Mono]]] = {
    # candidate codes (Table 1 / Table "ZSZ-LP polynomials")
    "ZSZ-LP-160": (16, 2, 9, [(0, 0), (13, 0), (14, 1)], [(0, 0), (3, 1), (13, 1)],
                   [(0, 0), (14, 0), (12, 1)], [(0, 0), (7, 0), (11, 0)]),
    "ZSZ-LP-240": (12, 4, 7, [(0, 0), (8, 1), (7, 2)], [(0, 0), (2, 0), (5, 1)],
                   [(0, 0), (4, 1), (2, 3)], [(0, 0), (4, 0), (9, 0)]),
    "ZSZ-LP-320": (16, 4, 3, [(0, 0), (1, 0), (0, 1)], [(0, 0), (2, 0), (13, 3)],
                   [(0, 0), (12, 1), (2, 3)], [(0, 0), (12, 0), (11, 2)]),
    "ZSZ-LP-390": (26, 3, 3, [(0, 0), (17, 1), (14, 2)], [(0, 0), (16, 0), (3, 1)],
                   [(0, 0), (24, 0), (8, 1)], [(0, 0), (21, 0), (0, 1)]),
    "ZSZ-LP-550": (22, 5, 3, [(0, 0), (10, 0), (5, 2)], [(0, 0), (8, 0), (2, 3)],
                   [(0, 0), (7, 0), (16, 1)], [(0, 0), (1, 0), (6, 4)]),
    "ZSZ-LP-775": (31, 5, 2, [(0, 0), (26, 2), (18, 3)], [(0, 0), (13, 2), (7, 4)],
                   [(0, 0), (1, 1), (28, 4)], [(0, 0), (0, 1), (22, 2)]),
    # additional codes (Table "more ZSZ-LP codes")
    "ZSZ-LP-60": (3, 4, 2, [(0, 0), (0, 3), (2, 3)], [(0, 0), (1, 0), (1, 2)],
                  [(0, 0), (0, 1), (1, 3)], [(0, 0), (0, 2), (0, 3)]),
    "ZSZ-LP-100": (5, 4, 4, [(0, 0), (2, 1), (0, 3)], [(0, 0), (2, 0), (1, 3)],
                   [(0, 0), (0, 3), (4, 3)], [(0, 0), (4, 2), (1, 3)]),
    "ZSZ-LP-150": (15, 2, 11, [(0, 0), (11, 0), (12, 1)], [(0, 0), (0, 1), (6, 1)],
                   [(0, 0), (3, 0), (11, 0)], [(0, 0), (6, 0), (14, 1)]),
    "ZSZ-LP-210": (21, 2, 8, [(0, 0), (1, 1), (3, 1)], [(0, 0), (12, 0), (17, 0)],
                   [(0, 0), (4, 1), (15, 1)], [(0, 0), (9, 1), (18, 1)]),
    "ZSZ-LP-525": (35, 3, 11, [(0, 0), (22, 0), (1, 2)], [(0, 0), (4, 0), (16, 2)],
                   [(0, 0), (34, 0), (12, 1)], [(0, 0), (28, 1), (31, 1)]),
    "ZSZ-LP-625": (25, 5, 6, [(0, 0), (6, 0), (1, 1)], [(0, 0), (24, 1), (21, 3)],
                   [(0, 0), (3, 2), (11, 3)], [(0, 0), (4, 0), (6, 2)]),
    "ZSZ-LP-700": (35, 4, 8, [(0, 0), (29, 1), (2, 2)], [(0, 0), (7, 1), (9, 1)],
                   [(0, 0), (19, 0), (16, 1)], [(0, 0), (32, 2), (23, 3)]),
    "ZSZ-LP-840": (28, 6, 11, [(0, 0), (0, 1), (5, 2)], [(0, 0), (2, 3), (19, 3)],
                   [(0, 0), (24, 1), (2, 2)], [(0, 0), (26, 2), (27, 3)]),
}

# n, k from Table 1 (Sec. 1) and Table "more ZSZ-LP codes" (App. A).
ZSZ_LP_NK: Dict[str, Tuple[int, int]] = {
    "ZSZ-LP-160": (160, 32), "ZSZ-LP-240": (240, 48), "ZSZ-LP-320": (320, 64),
    "ZSZ-LP-390": (390, 78), "ZSZ-LP-550": (550, 110), "ZSZ-LP-775": (775, 155),
    "ZSZ-LP-60": (60, 12), "ZSZ-LP-100": (100, 20), "ZSZ-LP-150": (150, 30),
    "ZSZ-LP-210": (210, 42), "ZSZ-LP-525": (525, 105), "ZSZ-LP-625": (625, 125),
    "ZSZ-LP-700": (700, 140), "ZSZ-LP-840": (840, 168),
}


# Classical seed codes H_left = (L[a] L[b]), H_right = (R[c] R[d]) of each
# candidate (Sec. 2.3, eq. "H_left, H_right"; Table "classical ZSZ code
# params"): name -> (ZSZ-LP code, n, k, d or its upper bound, Tanner girth).
ZSZ_2BGA: Dict[str, Tuple[str, int, int, int, int]] = {
    "ZSZ-2BGA-64": ("ZSZ-LP-160", 64, 32, 10, 6), "ZSZ-2BGA-96": ("ZSZ-LP-240", 96, 48, 12, 6),
    "ZSZ-2BGA-128": ("ZSZ-LP-320", 128, 64, 14, 6), "ZSZ-2BGA-156": ("ZSZ-LP-390", 156, 78, 16, 6),
    "ZSZ-2BGA-220": ("ZSZ-LP-550", 220, 110, 18, 8), "ZSZ-2BGA-310": ("ZSZ-LP-775", 310, 155, 22, 8),
}


# ---------------------------------------------------------------------------
# ZSZ group (Sec. 2.2)
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class ZSZGroup:
    l1: int
    l2: int
    q: int

    def __post_init__(self):
        if pow(self.q, self.l2, self.l1) != 1 % self.l1:
            raise ValueError("q^l2 must be 1 mod l1 for a ZSZ group")

    @property
    def order(self) -> int:
        return self.l1 * self.l2

    def index(self, g: Mono) -> int:
        """x^a y^b -> a*l2 + b (App. C.4)."""
        a, b = g
        return (a % self.l1) * self.l2 + (b % self.l2)

    def element(self, idx: int) -> Mono:
        return divmod(idx, self.l2)

    def mul(self, g: Mono, h: Mono) -> Mono:
        """(x^a y^b)(x^c y^d) = x^(a + q^b c) y^(b + d): the push-through relation."""
        a, b = g
        c, d = h
        return ((a + pow(self.q, b % self.l2, self.l1) * c) % self.l1, (b + d) % self.l2)

    def mul_table(self) -> np.ndarray:
        """T[g, h] = index(g h)."""
        n = self.order
        T = np.empty((n, n), dtype=np.int64)
        for gi in range(n):
            g = self.element(gi)
            for hi in range(n):
                T[gi, hi] = self.index(self.mul(g, self.element(hi)))
        return T

    def L(self, poly: Sequence[Mono]) -> np.ndarray:
        """Left-regular representation L[p] = sum_g L[g], L[g]|h> = |gh> (App. B)."""
        n = self.order
        T = self.mul_table()
        Mx = np.zeros((n, n), dtype=np.uint8)
        cols = np.arange(n)
        for g in poly:
            Mx[T[self.index(g), cols], cols] ^= 1
        return Mx

    def R(self, poly: Sequence[Mono]) -> np.ndarray:
        """Right-regular representation R[p] = sum_g R[g], R[g]|h> = |hg> (App. B)."""
        n = self.order
        T = self.mul_table()
        Mx = np.zeros((n, n), dtype=np.uint8)
        cols = np.arange(n)
        for g in poly:
            Mx[T[cols, self.index(g)], cols] ^= 1
        return Mx


# ---------------------------------------------------------------------------
# GF(2) linear algebra on bit-packed rows
# ---------------------------------------------------------------------------
def _pack(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.uint8) & 1
    r, c = A.shape
    W = max(1, (c + 63) // 64)
    pad = np.zeros((r, W * 64), dtype=np.uint8)
    pad[:, :c] = A
    return np.packbits(pad, axis=1, bitorder="little").view(np.uint64).copy()


def _unpack(P: np.ndarray, c: int) -> np.ndarray:
    bits = np.unpackbits(P.view(np.uint8), axis=1, bitorder="little")
    return bits[:, :c].astype(np.uint8)


def gf2_rref(A: np.ndarray) -> Tuple[np.ndarray, List[int]]:
    """Reduced row echelon form over GF(2).  Returns (R, pivots), R dense uint8."""
    A = np.asarray(A)
    r, c = A.shape
    P = _pack(A)
    pivots: List[int] = []
    row = 0
    for col in range(c):
        if row == r:
            break
        w, b = divmod(col, 64)
        bit = np.uint64(b)
        colbits = (P[row:, w] >> bit) & np.uint64(1)
        nz = np.flatnonzero(colbits)
        if nz.size == 0:
            continue
        p = row + int(nz[0])
        if p != row:
            P[[row, p]] = P[[p, row]]
        mask = ((P[:, w] >> bit) & np.uint64(1)).astype(bool)
        mask[row] = False
        if mask.any():
            P[mask] ^= P[row]
        pivots.append(col)
        row += 1
    return _unpack(P[:row], c), pivots


def gf2_rank(A: np.ndarray) -> int:
    return len(gf2_rref(A)[1])


def gf2_nullspace(A: np.ndarray) -> np.ndarray:
    """Basis (rows) of {x : A x = 0} over GF(2)."""
    A = np.asarray(A, dtype=np.uint8)
    c = A.shape[1]
    R, piv = gf2_rref(A)
    free = [j for j in range(c) if j not in set(piv)]
    K = np.zeros((len(free), c), dtype=np.uint8)
    for t, f in enumerate(free):
        K[t, f] = 1
        for row, p in enumerate(piv):
            K[t, p] = R[row, f]
    return K


def logical_basis(HX: np.ndarray, HZ: np.ndarray) -> np.ndarray:
    """Rows: a basis of ker H_Z modulo the row space of H_X (the X-type logicals).

    A residual error r with H_X r = 0 is a nontrivial logical exactly when some
    row of this basis has odd overlap with r, so these rows are the observables
    of a decoder working on H_X.
    """
    K = gf2_nullspace(HZ)
    RX, pivX = gf2_rref(HX)
    PK = _pack(K)
    PX = _pack(RX)
    for row, col in enumerate(pivX):
        w, b = divmod(col, 64)
        mask = ((PK[:, w] >> np.uint64(b)) & np.uint64(1)).astype(bool)
        if mask.any():
            PK[mask] ^= PX[row]
    Kred = _unpack(PK, HX.shape[1])
    Lr, piv = gf2_rref(Kred)
    return Lr[: len(piv)]


# ---------------------------------------------------------------------------
# Codes
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class CSSCode:
    name: str
    HX: np.ndarray
    HZ: np.ndarray

    @property
    def n(self) -> int:
        return self.HX.shape[1]

    def k(self) -> int:
        return self.n - gf2_rank(self.HX) - gf2_rank(self.HZ)


def build_zsz_lp(l1: int, l2: int, q: int, a, b, c, d, name: str = "") -> CSSCode:
    """5-block H_X, H_Z with A=L[a], B=L[b], C=R[c], D=R[d] (Sec. 2.1, 2.4)."""
    G = ZSZGroup(l1, l2, q)
    A, B, C, D = G.L(a), G.L(b), G.R(c), G.R(d)
    Z = np.zeros_like(A)
    HX = np.block([[A, Z, B, Z, C.T], [Z, A, Z, B, D.T]]).astype(np.uint8)
    HZ = np.block([[C, D, Z, Z, A.T], [Z, Z, C, D, B.T]]).astype(np.uint8)
    return CSSCode(name or f"ZSZ-LP({l1},{l2},{q})", HX, HZ)


def zsz_lp(name: str) -> CSSCode:
    l1, l2, q, a, b, c, d = ZSZ_LP_CODES[name]
    return build_zsz_lp(l1, l2, q, a, b, c, d, name)


def configuration_model_36(n1: int, seed: int, max_tries: int = 10000) -> np.ndarray:
    """Seeded (3,6)-regular Tanner graph by the configuration model.

    Variable sockets (3 per bit) are paired with check sockets (6 per check) by a
    uniformly random permutation; a draw with a repeated edge is rejected and
    redrawn.  n1 must be even; the result is (n1/2) x n1.
    """
    if n1 % 2:
        raise ValueError("n1 must be even")
    m1 = n1 // 2
    rng = np.random.default_rng(seed)
    vs = np.repeat(np.arange(n1), 3)
    cs = np.repeat(np.arange(m1), 6)
    for _ in range(max_tries):
        perm = rng.permutation(cs.size)
        pairs = cs[perm] * n1 + vs
        if np.unique(pairs).size == pairs.size:
            H = np.zeros((m1, n1), dtype=np.uint8)
            H[cs[perm], vs] = 1
            return H
    raise RuntimeError("configuration model: no simple graph found")


def build_hgp(H1: np.ndarray, name: str = "") -> CSSCode:
    """Hypergraph product with H_X = [H1 (x) I_n1 | I_m1 (x) H1^T],
    H_Z = [I_n1 (x) H1 | H1^T (x) I_m1]  (check weight 6 + 3 = 9 for a (3,6) seed)."""
    m1, n1 = H1.shape
    HX = np.hstack([np.kron(H1, np.eye(n1, dtype=np.uint8)),
                    np.kron(np.eye(m1, dtype=np.uint8), H1.T)]).astype(np.uint8)
    HZ = np.hstack([np.kron(np.eye(n1, dtype=np.uint8), H1),
                    np.kron(H1.T, np.eye(m1, dtype=np.uint8))]).astype(np.uint8)
    return CSSCode(name or f"HGP-{n1}", HX, HZ)


def seeded_hgp(n1: int, seed: int) -> CSSCode:
    return build_hgp(configuration_model_36(n1, seed), f"HGP(3,6)-n1={n1}-seed={seed}")


# ---------------------------------------------------------------------------
# Detector error models
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DEM:
    """Detector error model: H (M detectors x N mechanisms), observables O (k x N),
    per-mechanism probabilities."""
    name: str
    H: np.ndarray          # uint8 (M, N)
    O: np.ndarray          # uint8 (k, N)
    priors: np.ndarray     # float64 (N,)
    rounds: int = 1

    @property
    def M(self) -> int:
        return self.H.shape[0]

    @property
    def N(self) -> int:
        return self.H.shape[1]

    @property
    def k(self) -> int:
        return self.O.shape[0]

    @property
    def nnz(self) -> int:
        return int(self.H.sum())

    def csc(self):
        """(col_ptr[N+1], row_idx[nnz]) int32, rows ascending within a column."""
        return dense_to_csc(self.H)

    def obs_csc(self):
        return dense_to_csc(self.O)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.H, self.O):
            h.update(np.packbits(a, axis=1).tobytes())
            h.update(np.asarray(a.shape, np.int64).tobytes())
        h.update(np.asarray(self.priors, np.float64).tobytes())
        return h.hexdigest()[:16]


def dense_to_csc(A: np.ndarray):
    A = np.asarray(A, dtype=np.uint8)
    rows, cols = np.nonzero(A.T)  # iterate column-major: (col, row) pairs sorted
    col_ptr = np.zeros(A.shape[1] + 1, dtype=np.int32)
    np.add.at(col_ptr, rows + 1, 1)
    col_ptr = np.cumsum(col_ptr).astype(np.int32)
    return col_ptr, cols.astype(np.int32)


def code_capacity_dem(code: CSSCode, p: float, obs: np.ndarray | None = None) -> DEM:
    """Code capacity: H = H_X, O = L_X, all priors p."""
    O = logical_basis(code.HX, code.HZ) if obs is None else obs
    return DEM(f"{code.name}/cc/p={p:g}", code.HX.copy(), O.astype(np.uint8),
               np.full(code.n, float(p)), rounds=1)


def phenomenological_dem(code: CSSCode, rounds: int, p: float, q_meas: float | None = None,
                         obs: np.ndarray | None = None) -> DEM:
    """Phenomenological noise over T rounds of X-check measurements.

    Detector (t, i) compares round t with round t-1 and sits at row t*m + i.
    Columns: data mechanisms (t, j) at t*n + j flip detectors {(t, i): H_X[i, j]=1}
    and the observables O[:, j]; measurement mechanisms (t, i), t < T-1, at
    T*n + t*m + i flip (t, i) and (t+1, i) and no observable.  The last round is
    noiseless, so H = [I_T (x) H_X | B_T (x) I_m] with B_T the T x (T-1)
    bidiagonal matrix.  T = 1 is code capacity.
    """
    HX = code.HX
    m, n = HX.shape
    T = int(rounds)
    O1 = logical_basis(code.HX, code.HZ) if obs is None else obs.astype(np.uint8)
    k = O1.shape[0]
    Nd, Nm = T * n, (T - 1) * m
    H = np.zeros((T * m, Nd + Nm), dtype=np.uint8)
    for t in range(T):
        H[t * m:(t + 1) * m, t * n:(t + 1) * n] = HX
    eye = np.eye(m, dtype=np.uint8)
    for t in range(T - 1):
        c0 = Nd + t * m
        H[t * m:(t + 1) * m, c0:c0 + m] = eye
        H[(t + 1) * m:(t + 2) * m, c0:c0 + m] = eye
    O = np.zeros((k, Nd + Nm), dtype=np.uint8)
    for t in range(T):
        O[:, t * n:(t + 1) * n] = O1
    pr = np.full(Nd + Nm, float(p))
    if q_meas is not None:
        pr[Nd:] = float(q_meas)
    return DEM(f"{code.name}/phen/T={T}/p={p:g}", H, O, pr, rounds=T)


# ---------------------------------------------------------------------------
# Named workloads (sizes follow the configurations the benchmarks run)
# ---------------------------------------------------------------------------
def zsz_2bga(name: str, side: str = "left") -> np.ndarray:
    """Parity-check matrix (l x 2l, uint8) of a classical ZSZ-2BGA code:
    (L[a] L[b]) for the left code, (R[c] R[d]) for the right one (Sec. 2.3)."""
    lp = ZSZ_2BGA[name][0]
    l1, l2, q, a, b, c, d = ZSZ_LP_CODES[lp]
    G = ZSZGroup(l1, l2, q)
    if side == "left":
        return np.concatenate([G.L(a), G.L(b)], axis=1)
    if side == "right":
        return np.concatenate([G.R(c), G.R(d)], axis=1)
    raise ValueError("side is 'left' or 'right'")


def awgn_sigma(ebn0_db: float, rate: float) -> float:
    """Noise standard deviation of unit-energy BPSK at E_b/N_0 (dB) and code
    rate R: E_b/N_0 = 1 / (2 R sigma^2) (App. "classical channel coding")."""
    return float(np.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))))


def awgn_llrs(N: int, shots: int, sigma: float, seed: int) -> np.ndarray:
    """Seeded channel LLRs 2y/sigma^2 of the all-zero codeword, y = 1 + sigma z
    with z standard normal (numpy's generator), float32 [shots][N]."""
    rng = np.random.default_rng(seed)
    y = 1.0 + sigma * rng.standard_normal((shots, N))
    return (2.0 * y / (sigma * sigma)).astype(np.float32)


def workload(name: str) -> DEM:
    """Named DEMs.

    cc160      ZSZ-LP-160 code capacity, p = 0.01            (64 x 160)
    phen160    ZSZ-LP-160, 9 phenomenological rounds, 1e-3   (576 x 1952)
    phen320/550/775   other candidates, T = 9, 1e-3
    phen840    [[840,168]] code, T = 12, 1e-3               (4032 x 13776)
    hgp56      seeded HGP n1 = 56, T = 12, 1e-3             (18816 x 64288)
    tiny60     [[60,12,6]] code capacity (tests)
    circ320x   circuit-level d-round memory of ZSZ-LP-320 in basis X (x or z;
               160, 240, 320, 390, 550), p = 1e-3      (1920 x 28992 for 320)
    """
    if name == "cc160":
        return code_capacity_dem(zsz_lp("ZSZ-LP-160"), 0.01)
    if name == "tiny60":
        return code_capacity_dem(zsz_lp("ZSZ-LP-60"), 0.02)
    if name.startswith("phen"):
        num = name[4:]
        T = 12 if num == "840" else 9
        return phenomenological_dem(zsz_lp(f"ZSZ-LP-{num}"), T, 1e-3)
    if name.startswith("circ"):
        from . import circuits
        return circuits.memory_dem(f"ZSZ-LP-{name[4:-1]}", name[-1].upper(), 1e-3)
    if name.startswith("hgp"):
        n1 = int(name[3:])
        T = 12 if n1 >= 56 else 9
        return phenomenological_dem(seeded_hgp(n1, seed=1000 + n1), T, 1e-3)
    raise KeyError(name)


def random_priors(N: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Seeded per-mechanism probabilities, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=N))


def random_syndromes(M: int, shots: int, density: float, seed: int) -> np.ndarray:
    """Seeded random detector bit vectors, packed LSB-first into uint32 words."""
    rng = np.random.default_rng(seed)
    bits = (rng.random((shots, M)) < density).astype(np.uint8)
    return pack_bits(bits)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """(rows, nbits) 0/1 -> (rows, ceil(nbits/32)) uint32, bit b of word w = column 32w+b."""
    bits = np.asarray(bits, dtype=np.uint8)
    r, c = bits.shape
    W = (c + 31) // 32
    pad = np.zeros((r, W * 32), dtype=np.uint8)
    pad[:, :c] = bits
    return np.packbits(pad, axis=1, bitorder="little").view(np.uint32).reshape(r, W).copy()


def unpack_bits(words: np.ndarray, nbits: int) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    r = words.shape[0]
    b = np.unpackbits(words.view(np.uint8).reshape(r, -1), axis=1, bitorder="little")
    return b[:, :nbits].astype(np.uint8)
