"""Launch-shape autotuner for the persistent Relay-BP decoder.

For one detector error model it times the decoder on a calibration batch for
every wavefronts-per-shot count and state (per-edge messages in LDS or in
device memory, or compact row records in LDS) and, for the compact state, every
shots-per-workgroup count (one shot per workgroup, or 2 or 4 shots in lockstep
sharing the table loads), keeps the fastest, applies it to the handle (rbp_set_launch_config) and caches
the choice by (model hash, device name, relay parameters) in a JSON file
($RBP_TUNE_CACHE, default ~/.cache/rbp/tune.json).  Outputs never depend on the
launch shape (tested), so tuning only changes speed.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional, Tuple

import numpy as np
import torch

from . import rbp

WAVES = (1, 2, 4, 8, 16)
STATES = (1, 2, 3)  # 1 = per-edge state in LDS, 2 = the same in device memory, 3 = compact row records in LDS
SHOTS_PER_WG = (1, 2, 4)  # shots per workgroup (2 and 4: the multi-shot kernel, compact state only)


def cache_path() -> str:
    return os.environ.get("RBP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rbp", "tune.json"))


def model_key(H: np.ndarray, params: rbp.RelayParams) -> str:
    h = hashlib.sha256()
    cp, ri = rbp.csc_of(H)
    h.update(np.asarray(H.shape, np.int64).tobytes())
    h.update(cp.tobytes())
    h.update(ri.tobytes())
    h.update(repr(sorted(vars(params).items())).encode())
    return h.hexdigest()[:20] + "@" + torch.cuda.get_device_name(0).replace(" ", "_")


def _load() -> Dict:
    try:
        return json.load(open(cache_path()))
    except (OSError, ValueError):
        return {}


def _store(d: Dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    json.dump(d, open(tmp, "w"), indent=1)
    os.replace(tmp, p)


def time_config(code: rbp.Code, priors, syn: torch.Tensor, params: rbp.RelayParams, waves: int, state: int,
                repeats: int = 2, shots_per_wg: int = 1) -> float:
    code.set_launch_config(waves, state, 0, shots_per_wg)
    out = code.decode(priors, syn, params)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        code.decode(priors, syn, params, out=out)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(code: rbp.Code, H: np.ndarray, priors, params: rbp.RelayParams, shots: int = 20000, seed: int = 99,
         waves: Iterable[int] = WAVES, states: Iterable[int] = STATES, use_cache: bool = True,
         shots_per_wg: Iterable[int] = SHOTS_PER_WG) -> Dict:
    key = model_key(H, params)
    cache = _load() if use_cache else {}
    if key in cache and "shots_per_wg" in cache[key]:
        c = cache[key]
        code.set_launch_config(c["waves_per_shot"], c["state"], 0, c["shots_per_wg"])
        return dict(c, cached=True)
    syn, _, _ = code.sample(priors, shots, seed)
    trials = []
    for w in waves:
        for st in states:
            for k in shots_per_wg:
                if k > 1 and st != 3:
                    continue
                try:
                    ms = time_config(code, priors, syn, params, w, st, shots_per_wg=k)
                except rbp.RbpError:
                    continue
                trials.append((ms, w, st, k))
    trials.sort()
    ms, w, st, k = trials[0]
    code.set_launch_config(w, st, 0, k)
    res = {"waves_per_shot": w, "state": st, "shots_per_wg": k, "ms": ms, "shots": shots,
           "trials": [{"waves": tw, "state": ts, "shots_per_wg": tk, "ms": tm} for tm, tw, ts, tk in trials]}
    if use_cache:
        cache[key] = res
        _store(cache)
    return dict(res, cached=False)
