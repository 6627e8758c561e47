"""CPU oracle for the Relay-BP Monte-Carlo path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's ``cpu_baseline`` leg.  The product package never imports it, and it
imports nothing from the product package (inputs arrive as plain numpy arrays).

* ``rbp_oracle.c`` -- Philox4x32-10 fault sampler (geometric gaps with
  integer thresholds, thinned to per-mechanism priors), GF(2) syndromes, FP32 Relay-BP
  (paper Sec. 6.1: flooding min-sum with memory, sequential relay legs,
  lowest-weight of ``stop_nconv`` solutions, single-precision messages).
* ``spa_oracle.c`` -- BPSK-AWGN channel (Philox4x32-10 + Box-Muller, double)
  and flooding sum-product BP with the phi-domain check update, LLRs and
  variable-to-check messages clipped to +-llr_max, single-precision messages
  (the paper's classical benchmark of its ZSZ-2BGA codes).
* ``stats`` -- block logical error rate, Clopper-Pearson interval and per-round
  rate (Sec. 6.1, Fig. "numerics" caption).
* ``mlp_ref`` -- float64 reference of the learned-proposal network.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbp_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "spa_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-pthread", *_SRCS, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u32p, i32p, f32p, f64p, u8p = (P(ctypes.c_uint32), P(ctypes.c_int32), P(ctypes.c_float),
                                        P(ctypes.c_double), P(ctypes.c_uint8))
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_gap_table.argtypes = [ctypes.c_double, ctypes.c_int32, u32p]
        L.orc_accept_table.argtypes = [ctypes.c_int64, f64p, ctypes.c_double, u32p]
        L.orc_llr.argtypes = [ctypes.c_int64, f64p, f32p]
        L.orc_gamma_table.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_uint64, f32p]
        L.orc_sample.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, i32p, f64p,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u32p, u32p, u32p]
        L.orc_sample.restype = ctypes.c_int
        L.orc_sample_plain.argtypes = [ctypes.c_int32, f64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       u32p]
        L.orc_sample_plain.restype = ctypes.c_int
        L.orc_syndrome.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, ctypes.c_uint64, u32p, u32p]
        L.orc_decode.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, i32p, f64p,
                                 u32p, ctypes.c_uint64, ctypes.c_void_p, f32p, u32p, u32p, u8p, u8p, u8p, i32p,
                                 i32p, f64p, ctypes.c_int32]
        L.orc_decode.restype = ctypes.c_int
        L.orc_trace.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, i32p, f64p,
                                u32p, ctypes.c_void_p, f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                f32p, f32p]
        L.orc_trace.restype = ctypes.c_int
        L.orc_bp_marginals.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, f64p, u32p, ctypes.c_float,
                                       ctypes.c_int32, f32p]
        L.orc_bp_marginals.restype = ctypes.c_int
        L.orc_spa_phi.argtypes = [ctypes.c_float]
        L.orc_spa_phi.restype = ctypes.c_float
        L.orc_awgn.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                               f64p]
        L.orc_spa_decode.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, f32p, ctypes.c_uint64,
                                     ctypes.c_int32, ctypes.c_float, ctypes.c_int32, u8p, u8p, i32p, f32p,
                                     ctypes.c_int32]
        L.orc_spa_decode.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class _Params(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_float), ("gamma_min", ctypes.c_float), ("gamma_max", ctypes.c_float),
                ("pre_iter", ctypes.c_int32), ("max_iterations", ctypes.c_int32), ("num_sets", ctypes.c_int32),
                ("stop_nconv", ctypes.c_int32), ("stopping_criterion", ctypes.c_int32),
                ("gamma_seed", ctypes.c_uint64)]


@dataclasses.dataclass
class RelayParams:
    """Relay-BP settings, named as in Sec. 6.1 (gamma0, pre_iter, num_sets,
    max_iterations, stop_nconv, gamma_dist, stopping_criterion)."""
    gamma0: float = 0.125
    gamma_min: float = -0.24
    gamma_max: float = 0.66
    pre_iter: int = 80
    max_iterations: int = 60
    num_sets: int = 100
    stop_nconv: int = 5
    stopping_criterion: int = 0  # 0 = stop after stop_nconv solutions, 1 = run all legs
    gamma_seed: int = 7

    def _c(self) -> _Params:
        return _Params(self.gamma0, self.gamma_min, self.gamma_max, self.pre_iter, self.max_iterations,
                       self.num_sets, self.stop_nconv, self.stopping_criterion, self.gamma_seed)


def _csc(A: np.ndarray):
    A = np.asarray(A, dtype=np.uint8)
    rows, cols = np.nonzero(A.T)
    ptr = np.zeros(A.shape[1] + 1, dtype=np.int32)
    np.add.at(ptr, rows + 1, 1)
    return np.cumsum(ptr).astype(np.int32), cols.astype(np.int32)


class Graph:
    """H and O of a detector error model in the oracle's own CSC arrays."""

    def __init__(self, H: np.ndarray, O: np.ndarray):
        self.M, self.N = H.shape
        self.k = O.shape[0]
        self.cp, self.ri = _csc(H)
        self.ocp, self.ori = _csc(O)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def gap_table(pmax: float, L: int) -> np.ndarray:
    """T_k = floor((1 - pmax)^k 2^32), k = 1..L (the sampler's gap thresholds)."""
    out = np.zeros(max(L, 1), dtype=np.uint32)
    lib().orc_gap_table(pmax, L, _p(out, ctypes.c_uint32))
    return out[:L]


def accept_table(p: np.ndarray, pmax: float) -> np.ndarray:
    """floor(p_j / pmax 2^32) for p_j < pmax, 0xFFFFFFFF where p_j = pmax."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(p.size, dtype=np.uint32)
    lib().orc_accept_table(p.size, _p(p, ctypes.c_double), pmax, _p(out, ctypes.c_uint32))
    return out


def llr(p: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(p.size, dtype=np.float32)
    lib().orc_llr(p.size, _p(p, ctypes.c_double), _p(out, ctypes.c_float))
    return out


def gamma_table(N: int, R: int, gmin: float, gmax: float, seed: int) -> np.ndarray:
    out = np.zeros((max(R, 1), N), dtype=np.float32)
    lib().orc_gamma_table(N, R, gmin, gmax, seed, _p(out, ctypes.c_float))
    return out[:R]


def sample(g: Graph, priors: np.ndarray, shots: int, seed: int, shot_offset: int = 0, want_errors: bool = False):
    pr = np.ascontiguousarray(priors, dtype=np.float64)
    wm, wk, wn = (g.M + 31) // 32, (g.k + 31) // 32, (g.N + 31) // 32
    syn = np.zeros((shots, wm), dtype=np.uint32)
    obs = np.zeros((shots, max(wk, 1)), dtype=np.uint32)
    err = np.zeros((shots, wn), dtype=np.uint32) if want_errors else None
    rc = lib().orc_sample(g.M, g.N, _p(g.cp, ctypes.c_int32), _p(g.ri, ctypes.c_int32), g.k,
                          _p(g.ocp, ctypes.c_int32), _p(g.ori, ctypes.c_int32), _p(pr, ctypes.c_double), shots,
                          seed, shot_offset, _p(syn, ctypes.c_uint32), _p(obs, ctypes.c_uint32),
                          _p(err, ctypes.c_uint32) if err is not None else None)
    if rc:
        raise RuntimeError(f"orc_sample failed: {rc}")
    return syn, obs, err


def sample_plain(N: int, priors: np.ndarray, shots: int, seed: int, shot_offset: int = 0) -> np.ndarray:
    """Fault words uint32 [shots][ceil(N/32)] from the plain per-mechanism
    Bernoulli definition (one Philox word per mechanism, e_j = [word < thr_j]):
    the reference law the gap sampler is checked against."""
    pr = np.ascontiguousarray(priors, dtype=np.float64)
    assert pr.size == N
    err = np.zeros((shots, (N + 31) // 32), dtype=np.uint32)
    rc = lib().orc_sample_plain(N, _p(pr, ctypes.c_double), shots, seed, shot_offset, _p(err, ctypes.c_uint32))
    if rc:
        raise RuntimeError(f"orc_sample_plain failed: {rc}")
    return err


def syndrome(g: Graph, err_words: np.ndarray) -> np.ndarray:
    e = np.ascontiguousarray(err_words, dtype=np.uint32)
    shots = e.shape[0]
    syn = np.zeros((shots, (g.M + 31) // 32), dtype=np.uint32)
    lib().orc_syndrome(g.M, g.N, _p(g.cp, ctypes.c_int32), _p(g.ri, ctypes.c_int32), shots,
                       _p(e, ctypes.c_uint32), _p(syn, ctypes.c_uint32))
    return syn


def decode(g: Graph, priors: np.ndarray, syndromes: np.ndarray, params: RelayParams, delta=None,
           nthreads: int | None = None, timing: bool = False) -> dict:
    pr = np.ascontiguousarray(priors, dtype=np.float64)
    syn = np.ascontiguousarray(syndromes, dtype=np.uint32)
    shots = syn.shape[0]
    wn, wk = (g.N + 31) // 32, max((g.k + 31) // 32, 1)
    corr = np.zeros((shots, wn), dtype=np.uint32)
    obsp = np.zeros((shots, wk), dtype=np.uint32)
    conv = np.zeros(shots, dtype=np.uint8)
    nconv = np.zeros(shots, dtype=np.uint8)
    path = np.zeros(shots, dtype=np.uint8)
    legs = np.zeros(shots, dtype=np.int32)
    iters = np.zeros(shots, dtype=np.int32)
    secs = np.zeros(shots, dtype=np.float64) if timing else None
    d = None
    if delta is not None:
        d = np.ascontiguousarray(delta, dtype=np.float32)
        assert d.shape == (shots, g.N)
    prm = params._c()
    nt = nthreads or os.cpu_count() or 1
    rc = lib().orc_decode(g.M, g.N, _p(g.cp, ctypes.c_int32), _p(g.ri, ctypes.c_int32), g.k,
                          _p(g.ocp, ctypes.c_int32), _p(g.ori, ctypes.c_int32), _p(pr, ctypes.c_double),
                          _p(syn, ctypes.c_uint32), shots, ctypes.cast(ctypes.byref(prm), ctypes.c_void_p),
                          _p(d, ctypes.c_float) if d is not None else None, _p(corr, ctypes.c_uint32),
                          _p(obsp, ctypes.c_uint32), _p(conv, ctypes.c_uint8), _p(nconv, ctypes.c_uint8),
                          _p(path, ctypes.c_uint8), _p(legs, ctypes.c_int32), _p(iters, ctypes.c_int32),
                          _p(secs, ctypes.c_double) if secs is not None else None, nt)
    if rc:
        raise RuntimeError(f"orc_decode failed: {rc}")
    out = dict(corrections=corr, obs_pred=obsp, converged=conv, nconv=nconv, path=path, legs=legs,
               iters=iters, threads=min(nt, max(shots, 1)))
    if secs is not None:
        out["seconds"] = secs
    return out


def trace(g: Graph, priors: np.ndarray, syndrome_words: np.ndarray, params: RelayParams, leg: int, t: int,
          phase: int = 0, delta=None):
    """(M after iteration t of leg `leg`, mu in CSC edge order) or None if not reached."""
    pr = np.ascontiguousarray(priors, dtype=np.float64)
    syn = np.ascontiguousarray(syndrome_words, dtype=np.uint32).reshape(-1)
    Mo = np.zeros(g.N, dtype=np.float32)
    mu = np.zeros(max(int(g.cp[-1]), 1), dtype=np.float32)
    d = None if delta is None else np.ascontiguousarray(delta, dtype=np.float32).reshape(-1)
    prm = params._c()
    rc = lib().orc_trace(g.M, g.N, _p(g.cp, ctypes.c_int32), _p(g.ri, ctypes.c_int32), g.k,
                         _p(g.ocp, ctypes.c_int32), _p(g.ori, ctypes.c_int32), _p(pr, ctypes.c_double),
                         _p(syn, ctypes.c_uint32), ctypes.cast(ctypes.byref(prm), ctypes.c_void_p),
                         _p(d, ctypes.c_float) if d is not None else None, phase, leg, t,
                         _p(Mo, ctypes.c_float), _p(mu, ctypes.c_float))
    if rc < 0:
        raise RuntimeError(f"orc_trace failed: {rc}")
    return (Mo, mu[: int(g.cp[-1])]) if rc == 1 else None


def bp_marginals(g: Graph, priors: np.ndarray, syndrome_words: np.ndarray, gamma: float, T: int) -> np.ndarray:
    """Marginals after T flooding iterations (constant memory strength, no early stop)."""
    pr = np.ascontiguousarray(priors, dtype=np.float64)
    syn = np.ascontiguousarray(syndrome_words, dtype=np.uint32).reshape(-1)
    out = np.zeros(g.N, dtype=np.float32)
    rc = lib().orc_bp_marginals(g.M, g.N, _p(g.cp, ctypes.c_int32), _p(g.ri, ctypes.c_int32),
                                _p(pr, ctypes.c_double), _p(syn, ctypes.c_uint32), gamma, T, _p(out, ctypes.c_float))
    if rc:
        raise RuntimeError(f"orc_bp_marginals failed: {rc}")
    return out


# ------------------------------------------------------- sum-product BP (AWGN)
def spa_phi(x: float) -> float:
    """phi(x) = -ln tanh(x/2) in single precision, as the oracle decoder evaluates it."""
    return float(lib().orc_spa_phi(float(x)))


def awgn(N: int, shots: int, sigma: float, seed: int, shot_offset: int = 0) -> np.ndarray:
    """Channel LLRs 2y/sigma^2 of the all-zero BPSK codeword, float64 [shots][N]."""
    out = np.zeros((shots, N), dtype=np.float64)
    lib().orc_awgn(N, shots, sigma, seed, shot_offset, _p(out, ctypes.c_double))
    return out


def spa_decode(H: np.ndarray, llr: np.ndarray, max_iterations: int = 100, llr_max: float = 20.0, stop: bool = True,
               marginals: bool = False, nthreads: int | None = None) -> dict:
    """Sum-product BP on channel LLRs float32 [shots][N]: hard decisions uint8
    [shots][N], converged, iterations (and the final marginals)."""
    H = np.asarray(H, dtype=np.uint8)
    M, N = H.shape
    cp, ri = _csc(H)
    L = np.ascontiguousarray(llr, dtype=np.float32)
    shots = L.shape[0]
    assert L.shape == (shots, N)
    bits = np.zeros((shots, N), dtype=np.uint8)
    conv = np.zeros(shots, dtype=np.uint8)
    iters = np.zeros(shots, dtype=np.int32)
    marg = np.zeros((shots, N), dtype=np.float32) if marginals else None
    nt = nthreads or os.cpu_count() or 1
    rc = lib().orc_spa_decode(M, N, _p(cp, ctypes.c_int32), _p(ri, ctypes.c_int32), _p(L, ctypes.c_float), shots,
                              max_iterations, llr_max, 1 if stop else 0, _p(bits, ctypes.c_uint8),
                              _p(conv, ctypes.c_uint8), _p(iters, ctypes.c_int32),
                              _p(marg, ctypes.c_float) if marg is not None else None, nt)
    if rc:
        raise RuntimeError(f"orc_spa_decode failed: {rc}")
    out = dict(bits=bits, converged=conv, iters=iters)
    if marg is not None:
        out["marginals"] = marg
    return out
