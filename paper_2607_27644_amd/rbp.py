"""Thin ctypes binding of librbp (the C ABI in include/rbp.h).

Argument marshalling only: every step of sampling and decoding runs in the HIP
kernels of librbp.  torch provides device memory (tensors) and streams.  torch
is imported first so that librbp binds to the HIP runtime torch already loaded.
If librbp.so is missing this module raises: there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import dataclasses
import os
import weakref
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbp.so")
LIB_MLP_F32_PATH = os.path.join(HERE, "librbp_mlp_f32.so")

RBP_OK = 0
RBP_ERR_INVALID_ARG = -1
RBP_ERR_ABORTED = -6
_ERRNAMES = {-1: "INVALID_ARG", -2: "SHAPE", -3: "UNSUPPORTED", -4: "OOM", -5: "HIP", -6: "ABORTED"}


class RbpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"librbp {_ERRNAMES.get(status, status)}: {msg}")
        self.status = status


class RelayParamsC(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_float), ("gamma_min", ctypes.c_float), ("gamma_max", ctypes.c_float),
                ("pre_iter", ctypes.c_int32), ("max_iterations", ctypes.c_int32), ("num_sets", ctypes.c_int32),
                ("stop_nconv", ctypes.c_int32), ("stopping_criterion", ctypes.c_int32),
                ("gamma_seed", ctypes.c_uint64)]


class SpaParamsC(ctypes.Structure):
    _fields_ = [("max_iterations", ctypes.c_int32), ("llr_max", ctypes.c_float), ("stop", ctypes.c_int32),
                ("waves_per_shot", ctypes.c_int32)]


@dataclasses.dataclass
class SpaParams:
    """Sum-product BP settings of the classical AWGN benchmark (num_iter 100,
    llr_max 20, stop at the first codeword)."""
    max_iterations: int = 100
    llr_max: float = 20.0
    stop: bool = True
    waves_per_shot: int = 0

    def c(self) -> SpaParamsC:
        return SpaParamsC(self.max_iterations, self.llr_max, 1 if self.stop else 0, self.waves_per_shot)


class LaunchConfigC(ctypes.Structure):
    _fields_ = [("waves_per_shot", ctypes.c_int32), ("state", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("shots_per_wg", ctypes.c_int32)]


SHOT_STATS_DTYPE = np.dtype([("converged", np.uint8), ("nconv", np.uint8), ("path", np.uint8), ("r0", np.uint8),
                             ("legs", np.uint16), ("r1", np.uint16), ("iters", np.uint32), ("r2", np.uint32),
                             ("t_start", np.uint64), ("t_end", np.uint64)])
assert SHOT_STATS_DTYPE.itemsize == 32


@dataclasses.dataclass
class RelayParams:
    """Relay-BP settings (names as in the paper's Sec. 6.1)."""
    gamma0: float = 0.125
    gamma_min: float = -0.24
    gamma_max: float = 0.66
    pre_iter: int = 80
    max_iterations: int = 60
    num_sets: int = 100
    stop_nconv: int = 5
    stopping_criterion: int = 0  # 0 NConv, 1 All
    gamma_seed: int = 7

    def c(self) -> RelayParamsC:
        return RelayParamsC(self.gamma0, self.gamma_min, self.gamma_max, self.pre_iter, self.max_iterations,
                            self.num_sets, self.stop_nconv, self.stopping_criterion, self.gamma_seed)


class CoopParamsC(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int32), ("stride", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("spin_limit", ctypes.c_uint32), ("device_fences", ctypes.c_int32)]


@dataclasses.dataclass
class CoopParams:
    """Latency-mode launch (rbp_decode_coop); 0 = library default."""
    workgroups: int = 0
    stride: int = 0
    waves: int = 0
    spin_limit: int = 0
    device_fences: int = 0  # device-scope fences even when the participants share one XCD

    def c(self) -> CoopParamsC:
        return CoopParamsC(self.workgroups, self.stride, self.waves, self.spin_limit, self.device_fences)


class ResidentParamsC(ctypes.Structure):
    _fields_ = [("coop", CoopParamsC), ("idle_seconds", ctypes.c_double), ("wait_seconds", ctypes.c_double)]


_lib = None
# Handles not yet closed.  They are closed by an exit hook that runs before the
# interpreter tears down its modules (exit hooks run last-registered first, and
# this module is imported after torch), so no HIP call is left to a finalizer
# that might run after the HIP runtime has shut down.
_live = weakref.WeakSet()
_finalized = False


@atexit.register
def _close_all():
    global _finalized
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass
    _finalized = True


def lib():
    global _lib
    if _lib is None:
        _lib = _load(LIB_PATH, required=True)
    return _lib


_lib_mlp_f32 = None


def lib_mlp_f32():
    """The FP32 test build of the proposal network (librbp_mlp_f32.so): the
    rbp_mlp_* entry points with FP32 weights, activations and gradients, used to
    check the network kernels element by element against a float64 reference."""
    global _lib_mlp_f32
    if _lib_mlp_f32 is None:
        _lib_mlp_f32 = _load(LIB_MLP_F32_PATH, required=False)
    return _lib_mlp_f32


def _load(path: str, required: bool):
    """Opens one of the built libraries and declares its entry points; with
    required=False the entry points the library does not export are skipped."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, i32, u64, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
    P = ctypes.POINTER
    sigs = {
        "rbp_code_create": [i32, i32, vp, vp, i32, vp, vp, P(vp)],
        "rbp_code_destroy": [vp],
        "rbp_code_info": [vp, P(i32), P(i32), P(i32), P(i32), P(i32), P(i32)],
        "rbp_sample": [vp, vp, u64, u64, u64, vp, vp, vp, vp],
        "rbp_decode": [vp, vp, vp, u64, P(RelayParamsC), vp, vp, vp, vp, vp],
        "rbp_decode_multi": [i32, vp, vp, vp, vp, u64, vp, P(RelayParamsC), vp, vp, vp, vp],
        "rbp_decode_noalloc": [vp, vp, vp, u64, P(RelayParamsC), vp, vp, vp, vp, vp],
        "rbp_decode_proposal": [vp, vp, vp, u64, P(RelayParamsC), vp, vp, vp, vp, vp],
        "rbp_decode_proposal_pos": [vp, vp, vp, u64, P(RelayParamsC), vp, vp, vp, vp, vp],
        "rbp_code_positions": [vp, P(i32), vp],
        "rbp_mlp_set_output_order": [vp, vp, i32],
        "rbp_mlp_forward_bf16": [vp, vp, u64, vp, vp],
        "rbp_set_launch_config": [vp, P(LaunchConfigC)],
        "rbp_get_launch_config": [vp, P(LaunchConfigC), P(i32), P(i32)],
        "rbp_trace": [vp, vp, vp, P(RelayParamsC), vp, i32, i32, i32, vp, vp, P(i32), vp],
        "rbp_mlp_create": [i32, i32, i32, u64, P(vp)],
        "rbp_mlp_destroy": [vp],
        "rbp_mlp_forward": [vp, vp, u64, vp, vp],
        "rbp_mlp_train_step": [vp, vp, vp, vp, u64, ctypes.c_float, vp, vp],
        "rbp_mlp_num_params": [vp, P(i64)],
        "rbp_mlp_gradients": [vp, vp, vp, vp, u64, vp, vp, vp],
        "rbp_code_llr": [vp, vp, vp, vp],
        "rbp_count_failures": [vp, vp, vp, u64, i32, vp, vp],
        "rbp_mlp_get_params": [vp, vp],
        "rbp_mlp_set_params": [vp, vp],
        "rbp_sample_awgn": [vp, u64, ctypes.c_double, u64, u64, vp, vp],
        "rbp_decode_spa": [vp, vp, u64, P(SpaParamsC), vp, vp, vp, vp, vp],
        "rbp_bits_extract": [vp, i32, u64, i64, i32, vp, i32, vp],
        "rbp_window_commit": [vp, u64, vp, i32, vp, i32, vp, vp, vp, vp, vp, i32, vp],
        "rbp_decode_coop": [vp, vp, vp, u64, P(RelayParamsC), P(CoopParamsC), vp, vp, vp, vp],
        "rbp_bits_gather": [vp, i32, u64, vp, i32, vp, i32, vp],
        "rbp_window_residual": [vp, i32, u64, vp, vp],
        "rbp_coop_aborted": [vp, vp, P(i32)],
        "rbp_mlp_save": [vp, ctypes.c_char_p],
        "rbp_mlp_load": [vp, ctypes.c_char_p],
        "rbp_test_set_coop_phantom": [vp, i32],
        "rbp_decode_each": [i32, vp, vp, vp, vp, P(RelayParamsC), vp, vp, vp, vp],
        "rbp_resident_start": [vp, vp, P(RelayParamsC), P(ResidentParamsC), P(vp)],
        "rbp_resident_decode": [vp, vp, vp, vp, vp],
        "rbp_resident_info": [vp, P(u64), P(i32), P(i32), P(ctypes.c_uint32)],
        "rbp_resident_stop": [vp],
    }
    sigs["rbp_measure_lds_bandwidth"] = [i32, ctypes.POINTER(ctypes.c_double)]
    for name, args in sigs.items():
        if not required and not hasattr(L, name):
            continue
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.rbp_last_error.argtypes = []
    L.rbp_last_error.restype = ctypes.c_char_p
    return L


def check(status: int, L=None):
    if status != RBP_OK:
        raise RbpError(status, (L or lib()).rbp_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def words(nbits: int) -> int:
    return (nbits + 31) // 32


def _need(t, name: str, dtype, shape=None, optional: bool = False):
    """Raise unless t is a contiguous CUDA tensor of this dtype (and shape):
    the library takes device pointers, so a host tensor or a wrong layout
    must never reach it."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")


def csc_of(A: np.ndarray):
    A = np.asarray(A, dtype=np.uint8)
    rows, cols = np.nonzero(A.T)
    ptr = np.zeros(A.shape[1] + 1, dtype=np.int32)
    np.add.at(ptr, rows + 1, 1)
    return np.cumsum(ptr).astype(np.int32), cols.astype(np.int32)


class Code:
    """A detector error model handle (rbp_code_create)."""

    def __init__(self, H: np.ndarray, O: np.ndarray):
        self.M, self.N = H.shape
        self.k = O.shape[0]
        cp, ri = csc_of(H)
        ocp, ori = csc_of(O) if self.k > 0 else (np.zeros(self.N + 1, np.int32), np.zeros(1, np.int32))
        self.nnz = int(cp[-1])
        h = ctypes.c_void_p()
        check(lib().rbp_code_create(self.M, self.N, cp.ctypes.data, ri.ctypes.data, self.k, ocp.ctypes.data,
                                    ori.ctypes.data, ctypes.byref(h)))
        self.h = h
        self._residents = weakref.WeakSet()
        _live.add(self)

    @classmethod
    def from_dem(cls, dem) -> "Code":
        return cls(dem.H, dem.O)

    def close(self):
        if getattr(self, "h", None):
            for r in list(getattr(self, "_residents", ())):
                r.close()
            if not _finalized:
                lib().rbp_code_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        vals = [ctypes.c_int32() for _ in range(6)]
        check(lib().rbp_code_info(self.h, *[ctypes.byref(v) for v in vals]))
        return dict(zip(["M", "N", "nnz", "k", "max_row_deg", "max_col_deg"], [v.value for v in vals]))

    # -- sampling ---------------------------------------------------------
    def sample(self, priors, shots: int, seed: int, shot_offset: int = 0, errors: bool = False, stream=None,
               out=None):
        dev = torch.device("cuda")
        if out is None:
            syn = torch.empty((shots, words(self.M)), dtype=torch.int32, device=dev)
            obs = torch.empty((shots, max(words(self.k), 1)), dtype=torch.int32, device=dev)
            err = torch.empty((shots, words(self.N)), dtype=torch.int32, device=dev) if errors else None
        else:
            syn, obs, err = out
            _need(syn, "syndromes", torch.int32, (shots, words(self.M)))
            _need(obs, "obs", torch.int32, (shots, max(words(self.k), 1)))
            _need(err, "errors", torch.int32, (shots, words(self.N)), optional=True)
        pr = self._priors(priors)
        check(lib().rbp_sample(self.h, pr.ctypes.data, shots, seed, shot_offset, _ptr(syn), _ptr(obs), _ptr(err),
                               _stream(stream)))
        return syn, obs, err

    # -- decoding ---------------------------------------------------------
    def _priors(self, priors) -> np.ndarray:
        pr = _f64(priors)
        if pr.shape != (self.N,):
            raise ValueError(f"priors must have shape ({self.N},) (got {pr.shape})")
        return pr

    def _outputs(self, shots: int, dev, stats: bool, out):
        if out is None:
            corr = torch.empty((shots, words(self.N)), dtype=torch.int32, device=dev)
            obsp = torch.empty((shots, max(words(self.k), 1)), dtype=torch.int32, device=dev)
            st = torch.empty((shots, 32), dtype=torch.uint8, device=dev) if stats else None
        else:
            corr, obsp, st = out
            _need(corr, "corrections", torch.int32, (shots, words(self.N)))
            _need(obsp, "obs_pred", torch.int32, (shots, max(words(self.k), 1)))
            _need(st, "stats", torch.uint8, (shots, 32), optional=True)
        return corr, obsp, st

    def decode(self, priors, syndromes: torch.Tensor, params: RelayParams, delta: Optional[torch.Tensor] = None,
               stats: bool = True, stream=None, out=None):
        _need(syndromes, "syndromes", torch.int32)
        shots = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (shots, words(self.M)))
        _need(delta, "delta", torch.float32, (shots, self.N), optional=True)
        dev = syndromes.device
        corr, obsp, st = self._outputs(shots, dev, stats, out)
        pr = self._priors(priors)
        prm = params.c()
        check(lib().rbp_decode(self.h, pr.ctypes.data, _ptr(syndromes), shots, ctypes.byref(prm), _ptr(delta),
                               _ptr(corr), _ptr(obsp), _ptr(st), _stream(stream)))
        return corr, obsp, st

    def positions(self) -> np.ndarray:
        """rbp_code_positions: the mechanism decoded at each decoder position
        (Np entries, -1 for padding)."""
        n = ctypes.c_int32()
        check(lib().rbp_code_positions(self.h, ctypes.byref(n), None))
        out = np.empty(n.value, dtype=np.int32)
        check(lib().rbp_code_positions(self.h, ctypes.byref(n), out.ctypes.data))
        return out

    def decode_proposal(self, priors, syndromes: torch.Tensor, params: RelayParams, delta_bf16: torch.Tensor,
                        stats: bool = True, stream=None, out=None, by_position: bool = False):
        """rbp_decode_proposal: the learned-proposal decode with BF16 adjustments
        (torch.bfloat16 [shots][N], e.g. from MLP.forward_bf16); by_position:
        rbp_decode_proposal_pos, adjustments [shots][Np] in the decoder's
        position order (positions(), MLP.set_output_order)."""
        _need(syndromes, "syndromes", torch.int32)
        shots = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (shots, words(self.M)))
        if by_position and getattr(self, "_np", None) is None:
            self._np = len(self.positions())
        width = self._np if by_position else self.N
        _need(delta_bf16, "delta_bf16", torch.bfloat16, (shots, width))
        corr, obsp, st = self._outputs(shots, syndromes.device, stats, out)
        pr = self._priors(priors)
        prm = params.c()
        fn = lib().rbp_decode_proposal_pos if by_position else lib().rbp_decode_proposal
        check(fn(self.h, pr.ctypes.data, _ptr(syndromes), shots, ctypes.byref(prm), _ptr(delta_bf16), _ptr(corr),
                 _ptr(obsp), _ptr(st), _stream(stream)))
        return corr, obsp, st

    def decode_noalloc(self, priors, syndromes: torch.Tensor, params: RelayParams,
                       delta: Optional[torch.Tensor] = None, stream=None, out=None):
        """rbp_decode_noalloc: the decode without any device allocation in the
        library (its scratch is a fixed array per GPU).  out = (corrections,
        obs_pred, stats or None) is required, so this call allocates nothing
        either; decode() must have run once with the same priors and params."""
        if out is None:
            raise ValueError("decode_noalloc needs out=(corrections, obs_pred, stats)")
        _need(syndromes, "syndromes", torch.int32)
        shots = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (shots, words(self.M)))
        _need(delta, "delta", torch.float32, (shots, self.N), optional=True)
        corr, obsp, st = self._outputs(shots, syndromes.device, True, out)
        pr = self._priors(priors)
        prm = params.c()
        check(lib().rbp_decode_noalloc(self.h, pr.ctypes.data, _ptr(syndromes), shots, ctypes.byref(prm),
                                       _ptr(delta), _ptr(corr), _ptr(obsp), _ptr(st), _stream(stream)))
        return corr, obsp, st

    def decode_coop(self, priors, syndromes: torch.Tensor, params: RelayParams, coop: Optional[CoopParams] = None,
                    stats: bool = True, stream=None, out=None):
        """Latency mode: shots one after another, each by several workgroups.
        Returns when the shots are decoded; raises RbpError (status ABORTED)
        if a barrier wait expired."""
        _need(syndromes, "syndromes", torch.int32)
        shots = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (shots, words(self.M)))
        dev = syndromes.device
        corr, obsp, st = self._outputs(shots, dev, stats, out)
        pr = self._priors(priors)
        prm = params.c()
        cp = (coop or CoopParams()).c()
        check(lib().rbp_decode_coop(self.h, pr.ctypes.data, _ptr(syndromes), shots, ctypes.byref(prm),
                                    ctypes.byref(cp), _ptr(corr), _ptr(obsp), _ptr(st), _stream(stream)))
        return corr, obsp, st

    def resident(self, priors, params: RelayParams, coop: Optional[CoopParams] = None, idle_seconds: float = 0.0,
                 wait_seconds: float = 0.0) -> "Resident":
        """Starts a resident decoder on this code (see Resident)."""
        return Resident(self, priors, params, coop, idle_seconds, wait_seconds)

    def set_coop_phantom(self, phantom: int):
        """Test hook (rbp_test_set_coop_phantom): latency-mode barriers also wait for
        `phantom` workgroups that never arrive, so every launch stops with ABORTED."""
        check(lib().rbp_test_set_coop_phantom(self.h, phantom))

    def coop_aborted(self, stream=None) -> bool:
        v = ctypes.c_int32()
        check(lib().rbp_coop_aborted(self.h, _stream(stream), ctypes.byref(v)))
        return bool(v.value)

    def trace(self, priors, syndrome: torch.Tensor, params: RelayParams, leg: int, t: int, phase: int = 0,
              delta: Optional[torch.Tensor] = None, stream=None):
        _need(syndrome, "syndrome", torch.int32, (words(self.M),))
        _need(delta, "delta", torch.float32, (self.N,), optional=True)
        dev = syndrome.device
        Mo = torch.empty(self.N, dtype=torch.float32, device=dev)
        mu = torch.empty(max(self.nnz, 1), dtype=torch.float32, device=dev)
        reached = ctypes.c_int32()
        pr = self._priors(priors)
        prm = params.c()
        check(lib().rbp_trace(self.h, pr.ctypes.data, _ptr(syndrome), ctypes.byref(prm), _ptr(delta), phase, leg, t,
                              _ptr(Mo), _ptr(mu), ctypes.byref(reached), _stream(stream)))
        if not reached.value:
            return None
        return Mo.cpu().numpy(), mu[: self.nnz].cpu().numpy()

    def llr(self, priors, stream=None) -> torch.Tensor:
        """The decoder's FP32 LLRs for these priors, on the device."""
        out = torch.empty(self.N, dtype=torch.float32, device="cuda")
        pr = _f64(priors)
        check(lib().rbp_code_llr(self.h, pr.ctypes.data, _ptr(out), _stream(stream)))
        return out

    # -- classical channel coding (BPSK-AWGN, sum-product BP) ---------------
    def sample_awgn(self, shots: int, sigma: float, seed: int, shot_offset: int = 0, stream=None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Channel LLRs of the all-zero codeword, float32 [shots][N] (rbp_sample_awgn)."""
        if out is None:
            out = torch.empty((shots, self.N), dtype=torch.float32, device="cuda")
        _need(out, "out", torch.float32, (shots, self.N))
        check(lib().rbp_sample_awgn(self.h, shots, float(sigma), seed, shot_offset, _ptr(out), _stream(stream)))
        return out

    def decode_spa(self, llr: torch.Tensor, params: Optional[SpaParams] = None, marginals: bool = False,
                   stats: bool = True, counts: Optional[torch.Tensor] = None, stream=None, out=None):
        """Sum-product BP (rbp_decode_spa) -> (bits, marginals or None, stats or None).
        counts (int64[3], device) accumulates block errors, undetected errors and
        non-converged shots with respect to the all-zero codeword."""
        params = params or SpaParams()
        _need(llr, "llr", torch.float32)
        shots = llr.shape[0]
        _need(llr, "llr", torch.float32, (shots, self.N))
        dev = llr.device
        if out is None:
            bits = torch.empty((shots, words(self.N)), dtype=torch.int32, device=dev)
            marg = torch.empty((shots, self.N), dtype=torch.float32, device=dev) if marginals else None
            st = torch.empty((shots, 32), dtype=torch.uint8, device=dev) if stats else None
        else:
            bits, marg, st = out
            _need(bits, "bits", torch.int32, (shots, words(self.N)))
            _need(marg, "marginals", torch.float32, (shots, self.N), optional=True)
            _need(st, "stats", torch.uint8, (shots, 32), optional=True)
        _need(counts, "counts", torch.int64, optional=True)
        if counts is not None and counts.numel() < 3:
            raise ValueError("counts needs 3 entries")
        prm = params.c()
        check(lib().rbp_decode_spa(self.h, _ptr(llr), shots, ctypes.byref(prm), _ptr(bits), _ptr(marg), _ptr(st),
                                   _ptr(counts), _stream(stream)))
        return bits, marg, st

    def set_launch_config(self, waves_per_shot: int = 0, state: int = 0, max_slots: int = 0, shots_per_wg: int = 0):
        """rbp_set_launch_config; shots_per_wg 2 or 4 selects the multi-shot
        kernel (compact state, plain decodes of one model)."""
        cfg = LaunchConfigC(waves_per_shot, state, max_slots, shots_per_wg)
        check(lib().rbp_set_launch_config(self.h, ctypes.byref(cfg)))

    def launch_config(self):
        cfg = LaunchConfigC()
        slots, lds = ctypes.c_int32(), ctypes.c_int32()
        check(lib().rbp_get_launch_config(self.h, ctypes.byref(cfg), ctypes.byref(slots), ctypes.byref(lds)))
        return dict(waves_per_shot=cfg.waves_per_shot, state=cfg.state, max_slots=cfg.max_slots,
                    shots_per_wg=cfg.shots_per_wg, slots=slots.value, lds_bytes=lds.value)


def decode_each(codes: Sequence[Code], priors: Sequence, syndromes: Sequence[torch.Tensor], params: RelayParams,
                outs: Optional[Sequence] = None, stream=None):
    """Several models, each in its own launch with its own launch shape (the
    code's launch config), issued together on side streams and joined into
    `stream` (rbp_decode_each).  Returns one (corrections, obs_pred, stats)
    tuple per model, as Code.decode would."""
    n = len(codes)
    if not 1 <= n <= 8 or not (len(priors) == len(syndromes) == n):
        raise ValueError("decode_each needs 1..8 models and one priors/syndromes entry each")
    res = []
    for i, c in enumerate(codes):
        _need(syndromes[i], f"syndromes[{i}]", torch.int32)
        r = syndromes[i].shape[0]
        _need(syndromes[i], f"syndromes[{i}]", torch.int32, (r, words(c.M)))
        res.append(c._outputs(r, syndromes[i].device, True, None if outs is None else outs[i]))
    VP = ctypes.c_void_p * n
    prs = [c._priors(p) for c, p in zip(codes, priors)]
    shots = (ctypes.c_uint64 * n)(*[s.shape[0] for s in syndromes])
    prm = params.c()
    check(lib().rbp_decode_each(n, VP(*[c.h.value for c in codes]), VP(*[p.ctypes.data for p in prs]), shots,
                                VP(*[s.data_ptr() for s in syndromes]), ctypes.byref(prm),
                                VP(*[r[0].data_ptr() for r in res]), VP(*[r[1].data_ptr() for r in res]),
                                VP(*[r[2].data_ptr() if r[2] is not None else None for r in res]), _stream(stream)))
    return res


def decode_multi(codes: Sequence[Code], priors: Sequence, shot_code: torch.Tensor, shot_index: torch.Tensor,
                 syndromes: Sequence[torch.Tensor], params: RelayParams, corrections: Sequence[torch.Tensor],
                 obs_pred: Sequence[torch.Tensor], stats: Optional[torch.Tensor] = None, stream=None,
                 check_indices: bool = True):
    """One persistent launch over several models: shot s is row shot_index[s]
    of model shot_code[s].  With check_indices (default) every code and row
    index is checked against the models and their arrays before the launch
    (one device reduction and a synchronization)."""
    n = len(codes)
    if not 1 <= n <= 8 or not (len(priors) == len(syndromes) == len(corrections) == len(obs_pred) == n):
        raise ValueError("decode_multi needs 1..8 models and one priors/syndromes/corrections/obs_pred entry each")
    _need(shot_code, "shot_code", torch.uint8)
    shots = shot_code.shape[0]
    _need(shot_code, "shot_code", torch.uint8, (shots,))
    _need(shot_index, "shot_index", torch.int32, (shots,))
    _need(stats, "stats", torch.uint8, (shots, 32), optional=True)
    rows = []
    for i, c in enumerate(codes):
        _need(syndromes[i], f"syndromes[{i}]", torch.int32)
        r = syndromes[i].shape[0]
        rows.append(r)
        _need(syndromes[i], f"syndromes[{i}]", torch.int32, (r, words(c.M)))
        _need(corrections[i], f"corrections[{i}]", torch.int32, (r, words(c.N)))
        _need(obs_pred[i], f"obs_pred[{i}]", torch.int32, (r, max(words(c.k), 1)))
    if check_indices and shots > 0:
        code_l = shot_code.to(torch.int64)
        if int(code_l.max().item()) >= n:
            raise ValueError("shot_code has a value >= the number of models")
        idx = shot_index.to(torch.int64)  # int32 rows; negative values are out of range
        lim = torch.tensor(rows, dtype=torch.int64, device=shot_code.device)[code_l]
        if bool(((idx < 0) | (idx >= lim)).any().item()):
            raise ValueError("shot_index has a row outside its model's arrays")
    VP = ctypes.c_void_p * n
    prs = [c._priors(p) for c, p in zip(codes, priors)]
    pr_arr = VP(*[p.ctypes.data for p in prs])
    prm = params.c()
    check(lib().rbp_decode_multi(n, VP(*[c.h.value for c in codes]), pr_arr, _ptr(shot_code), _ptr(shot_index),
                                 shots, VP(*[s.data_ptr() for s in syndromes]), ctypes.byref(prm),
                                 VP(*[c.data_ptr() for c in corrections]), VP(*[o.data_ptr() for o in obs_pred]),
                                 _ptr(stats), _stream(stream)))


def count_failures(obs_pred: torch.Tensor, obs: torch.Tensor, stats: torch.Tensor, count: torch.Tensor,
                   stream=None):
    """count (int64[1] on the device) += block failures of the batch (GPU reduction)."""
    _need(obs, "obs", torch.int32)
    _need(obs_pred, "obs_pred", torch.int32, tuple(obs.shape))
    _need(stats, "stats", torch.uint8, (obs.shape[0], 32))
    _need(count, "count", torch.int64)
    check(lib().rbp_count_failures(_ptr(obs_pred), _ptr(obs), _ptr(stats), obs.shape[0], obs.shape[1], _ptr(count),
                                   _stream(stream)))


def bits_extract(src: torch.Tensor, bit_offset: int, nbits: int, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[s] = bits [bit_offset, bit_offset + nbits) of src[s] (rbp_bits_extract)."""
    _need(src, "src", torch.int32)
    _need(out, "out", torch.int32)
    if out.shape[0] != src.shape[0]:
        raise ValueError("src and out need the same number of rows")
    check(lib().rbp_bits_extract(_ptr(src), src.shape[1], src.shape[0], bit_offset, nbits, _ptr(out), out.shape[1],
                                 _stream(stream)))
    return out


def bits_gather(src: torch.Tensor, rows: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[s] bit t = src[s] bit rows[t] (rbp_bits_gather); rows int32 on the device."""
    _need(src, "src", torch.int32)
    _need(out, "out", torch.int32)
    _need(rows, "rows", torch.int32)
    if out.shape[0] != src.shape[0]:
        raise ValueError("src and out need the same number of rows")
    check(lib().rbp_bits_gather(_ptr(src), src.shape[1], src.shape[0], _ptr(rows), rows.numel(), _ptr(out),
                                out.shape[1], _stream(stream)))
    return out


def window_residual(syndromes: torch.Tensor, acc_stats: torch.Tensor, stream=None):
    """Clear `converged` of the shots whose running syndrome is not zero (rbp_window_residual)."""
    _need(syndromes, "syndromes", torch.int32)
    _need(acc_stats, "acc_stats", torch.uint8, (syndromes.shape[0], 32))
    check(lib().rbp_window_residual(_ptr(syndromes), syndromes.shape[1], syndromes.shape[0], _ptr(acc_stats),
                                    _stream(stream)))


def window_commit(code: "Code", win_corr: torch.Tensor, cmap: torch.Tensor, n_win: int, syndromes: torch.Tensor,
                  obs_pred: torch.Tensor, corrections: torch.Tensor, win_stats: Optional[torch.Tensor] = None,
                  acc_stats: Optional[torch.Tensor] = None, first: bool = False, stream=None):
    """Commit a window's decoded mechanisms to the full model (rbp_window_commit)."""
    shots = win_corr.shape[0]
    for name, t in (("win_corr", win_corr), ("cmap", cmap), ("syndromes", syndromes), ("obs_pred", obs_pred),
                    ("corrections", corrections)):
        _need(t, name, torch.int32)
    for name, t in (("syndromes", syndromes), ("obs_pred", obs_pred), ("corrections", corrections)):
        if t.shape[0] != shots:
            raise ValueError(f"{name} needs {shots} rows")
    _need(win_stats, "win_stats", torch.uint8, (shots, 32), optional=True)
    _need(acc_stats, "acc_stats", torch.uint8, (shots, 32), optional=True)
    check(lib().rbp_window_commit(code.h, shots, _ptr(win_corr), win_corr.shape[1], _ptr(cmap), n_win,
                                  _ptr(syndromes), _ptr(obs_pred), _ptr(corrections), _ptr(win_stats),
                                  _ptr(acc_stats), 1 if first else 0, _stream(stream)))


def measure_lds_bandwidth(width_bytes: int = 16) -> float:
    """Aggregate LDS read bandwidth of the current GPU in bytes/s (rbp_measure_lds_bandwidth)."""
    v = ctypes.c_double()
    check(lib().rbp_measure_lds_bandwidth(width_bytes, ctypes.byref(v)))
    return v.value


def _host_u32(x, n: int, name: str) -> np.ndarray:
    """A host array of n uint32 words (numpy, or a CPU tensor) as a contiguous
    uint32 array; device tensors are refused (the mailbox takes host memory)."""
    if isinstance(x, torch.Tensor):
        if x.device.type != "cpu":
            raise ValueError(f"{name} must be in host memory (got {x.device})")
        x = x.numpy()
    a = np.ascontiguousarray(x)
    if a.dtype == np.int32:
        a = a.view(np.uint32)
    if a.dtype != np.uint32:
        raise TypeError(f"{name} must be uint32 or int32 words (got {a.dtype})")
    if a.shape != (n,):
        raise ValueError(f"{name} must have shape ({n},) (got {a.shape})")
    return a


class Resident:
    """Resident decoder (rbp_resident_*): the latency-mode kernel launched once
    and fed one shot at a time through a mailbox in pinned host memory, so a
    shot's latency holds no launch.  decode() takes one host syndrome and
    returns host arrays; the kernel ends itself after idle_seconds without a
    shot and is relaunched by the next decode()."""

    def __init__(self, code: "Code", priors, params: RelayParams, coop: Optional[CoopParams] = None,
                 idle_seconds: float = 0.0, wait_seconds: float = 0.0):
        self.M, self.N, self.k = code.M, code.N, code.k
        pr = code._priors(priors)
        prm = params.c()
        rp = ResidentParamsC((coop or CoopParams()).c(), float(idle_seconds), float(wait_seconds))
        h = ctypes.c_void_p()
        check(lib().rbp_resident_start(code.h, pr.ctypes.data, ctypes.byref(prm), ctypes.byref(rp), ctypes.byref(h)))
        self.h = h
        self.code = code
        code._residents.add(self)
        _live.add(self)

    def decode(self, syndrome):
        """One shot: syndrome (words(M) uint32/int32 host words) -> correction
        (words(N) uint32), observable prediction (max(words(k), 1) uint32) and
        the statistics record (SHOT_STATS_DTYPE)."""
        syn = _host_u32(syndrome, words(self.M), "syndrome")
        corr = np.empty(words(self.N), dtype=np.uint32)
        obs = np.zeros(max(words(self.k), 1), dtype=np.uint32)
        st = np.zeros(1, dtype=SHOT_STATS_DTYPE)
        check(lib().rbp_resident_decode(self.h, syn.ctypes.data, corr.ctypes.data, obs.ctypes.data, st.ctypes.data))
        return corr, obs, st[0]

    def info(self) -> dict:
        shots, launches, running = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_int32()
        xcds = ctypes.c_uint32()
        check(lib().rbp_resident_info(self.h, ctypes.byref(shots), ctypes.byref(launches), ctypes.byref(running),
                                      ctypes.byref(xcds)))
        return {"shots": shots.value, "launches": launches.value, "running": bool(running.value),
                "xcds": xcds.value}

    def close(self):
        if getattr(self, "h", None):
            h, self.h = self.h, None
            if not _finalized:
                check(lib().rbp_resident_stop(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stats_to_numpy(st: torch.Tensor) -> np.ndarray:
    return st.cpu().numpy().reshape(-1).view(SHOT_STATS_DTYPE)


def to_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


class MLP:
    """Learned proposal network (rbp_mlp_*): syndrome bits -> per-mechanism
    log-prior adjustments delta."""

    def __init__(self, in_dim: int, hidden: int, out_dim: int, seed: int = 0, fp32_test_build: bool = False):
        """fp32_test_build: use the FP32 test build of the kernels
        (lib_mlp_f32()) instead of the BF16 product build."""
        self.in_dim, self.hidden, self.out_dim = in_dim, hidden, out_dim
        self._L = lib_mlp_f32() if fp32_test_build else lib()
        h = ctypes.c_void_p()
        self._check(self._L.rbp_mlp_create(in_dim, hidden, out_dim, seed, ctypes.byref(h)))
        self.h = h
        _live.add(self)
        n = ctypes.c_int64()
        self._check(self._L.rbp_mlp_num_params(self.h, ctypes.byref(n)))
        self.n_params = n.value

    def _check(self, status: int):
        check(status, self._L)

    def close(self):
        if getattr(self, "h", None):
            if not _finalized:
                self._L.rbp_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, syndromes: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _need(syndromes, "syndromes", torch.int32)
        shots = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (shots, words(self.in_dim)))
        if out is None:
            out = torch.empty((shots, self.out_dim), dtype=torch.float32, device=syndromes.device)
        _need(out, "out", torch.float32, (shots, self.out_dim))
        self._check(self._L.rbp_mlp_forward(self.h, _ptr(syndromes), shots, _ptr(out), _stream(stream)))
        return out

    def set_output_order(self, order: Optional[np.ndarray]):
        """rbp_mlp_set_output_order: forward_bf16 then writes len(order) columns,
        column p the output order[p] (-1: zero); None restores the natural order."""
        if order is None:
            self._check(self._L.rbp_mlp_set_output_order(self.h, None, 0))
            self._ord_n = 0
            return
        o = np.ascontiguousarray(order, dtype=np.int32)
        self._check(self._L.rbp_mlp_set_output_order(self.h, o.ctypes.data, len(o)))
        self._ord_n = len(o)

    def forward_bf16(self, syndromes: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """The forward pass with BF16 output (rbp_mlp_forward_bf16): torch.bfloat16
        [shots][out_dim], or [shots][len(order)] after set_output_order."""
        _need(syndromes, "syndromes", torch.int32)
        shots = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (shots, words(self.in_dim)))
        cols = getattr(self, "_ord_n", 0) or self.out_dim
        if out is None:
            out = torch.empty((shots, cols), dtype=torch.bfloat16, device=syndromes.device)
        _need(out, "out", torch.bfloat16, (shots, cols))
        self._check(self._L.rbp_mlp_forward_bf16(self.h, _ptr(syndromes), shots, _ptr(out), _stream(stream)))
        return out

    def train_step(self, syndromes: torch.Tensor, targets: torch.Tensor, llr: torch.Tensor, lr: float,
                   loss_out: Optional[torch.Tensor] = None, stream=None):
        _need(syndromes, "syndromes", torch.int32)
        batch = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (batch, words(self.in_dim)))
        _need(targets, "targets", torch.int32, (batch, words(self.out_dim)))
        _need(llr, "llr", torch.float32, (self.out_dim,))
        _need(loss_out, "loss_out", torch.float32, optional=True)
        self._check(self._L.rbp_mlp_train_step(self.h, _ptr(syndromes), _ptr(targets), _ptr(llr), batch,
                                               ctypes.c_float(lr), _ptr(loss_out), _stream(stream)))

    def gradients(self, syndromes: torch.Tensor, targets: torch.Tensor, llr: torch.Tensor, stream=None):
        _need(syndromes, "syndromes", torch.int32)
        batch = syndromes.shape[0]
        _need(syndromes, "syndromes", torch.int32, (batch, words(self.in_dim)))
        _need(targets, "targets", torch.int32, (batch, words(self.out_dim)))
        _need(llr, "llr", torch.float32, (self.out_dim,))
        g = torch.empty(self.n_params, dtype=torch.float32, device=syndromes.device)
        loss = torch.empty(1, dtype=torch.float32, device=syndromes.device)
        self._check(self._L.rbp_mlp_gradients(self.h, _ptr(syndromes), _ptr(targets), _ptr(llr), batch, _ptr(g),
                                              _ptr(loss), _stream(stream)))
        return g, loss

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self._L.rbp_mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError(f"need {self.n_params} parameters (got {p.size})")
        self._check(self._L.rbp_mlp_set_params(self.h, p.ctypes.data))

    def save(self, path: str):
        """Checkpoint of masters, Adam moments and step (rbp_mlp_save)."""
        self._check(self._L.rbp_mlp_save(self.h, os.fsencode(path)))

    def load(self, path: str):
        """Restore a checkpoint written by save() into this handle (rbp_mlp_load)."""
        self._check(self._L.rbp_mlp_load(self.h, os.fsencode(path)))
