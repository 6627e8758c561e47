"""Measurements of the decoding path on its workload configurations.

    python -m paper_2607_27644_amd.experiments <name> [options]   -> one JSON object

names:
  multi      batched uneven decode: one persistent launch over several models
             with shots interleaved (shot i -> model i mod n), against one
             tuned launch per model
  large      a large model (phenomenological [[840,168]] code, 12 rounds, or the
             seeded hypergraph-product code with n1 = 56): throughput, per-shot
             service time, LER
  latency    sequential single-shot latency (one decode call per shot, host
             clock) and the all-legs worst case (stopping_criterion = 1)
  learned    train the proposal network on decoder-generated pairs and compare
             plain Relay-BP, the proposal and the delta = 0 control
  gamma      grid search of the relay memory-strength interval [gamma_min,
             gamma_max] at one noise strength, all intervals on the same
             syndromes (App. "more numerics", Table "relay gamma intervals")
  sweep      LER against the noise strength p with one interval, and the
             sub-threshold fit p^(d_circ/2) exp(c0 + c1 p + c2 p^2) with its
             extrapolation (Sec. 6.1)
  window     sliding-window decoding (window w rounds, commit c rounds) and
             two-layer parallel-window decoding of a long phenomenological
             memory experiment against one global decode: LER, throughput and
             the single-shot latency of one window (Sec. 6.1 latency discussion)
  circuit    circuit-level memory experiments (d rounds of the greedy-AOD
             syndrome extraction, Sec. 6.1 noise model, DEM sizes of Table
             "decoding latency") with the relay intervals of Table "relay gamma
             intervals": batched throughput and service times, sequential
             single-shot latency, the all-legs worst case, block LER, per code
             and memory basis
  resident   sequential single-shot latency of one model, per call (the
             latency mode, rbp_decode_coop) and through the resident decoder
             (rbp_resident_*), in alternating blocks on the same shots: host
             clock, the kernel's own time per shot (device timestamps) and the
             XCDs each resident launch ran on
  awgn       block error rate of the classical ZSZ-2BGA codes over BPSK-AWGN
             against E_b/N_0, sum-product BP (numerics appendix, "classical
             channel coding"), with the decoder's throughput and the Shannon
             limit of rate 1/2
All inputs are seeded and synthetic (see workloads.py).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np
import torch

from . import autotune, circuits, learned, rbp, stats, window, workloads


def _timed(fn, repeats: int = 3):
    best, out = float("inf"), None
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best, out


def _summary(dem, obs, obsp, st, shots, ms):
    s = rbp.stats_to_numpy(st)
    fails = stats.block_failures(rbp.to_u32(obsp), rbp.to_u32(obs), s["converged"])
    svc = (s["t_end"] - s["t_start"]).astype(np.float64) * 0.01
    return {"shots": shots, "ms": ms, "shots_per_s": shots / (ms * 1e-3),
            "ler": stats.ler_summary(int(fails.sum()), shots, dem.rounds, dem.k),
            "mean_iters": float(s["iters"].mean()), "max_iters": int(s["iters"].max()),
            "service_us": stats.percentiles(svc)}


def multi(names, shots_each: int, seed: int = 11, params: rbp.RelayParams | None = None) -> dict:
    params = params or rbp.RelayParams()
    dems = [workloads.workload(n) for n in names]
    codes = [rbp.Code.from_dem(d) for d in dems]
    n = len(dems)
    syns, obss = [], []
    for i, (d, c) in enumerate(zip(dems, codes)):
        syn, obs, _ = c.sample(d.priors, shots_each, seed + i)
        syns.append(syn)
        obss.append(obs)
    total = n * shots_each
    idx = torch.arange(total, device="cuda")
    shot_code = (idx % n).to(torch.uint8)
    shot_index = (idx // n).to(torch.int32)
    corrs = [torch.empty((shots_each, rbp.words(d.N)), dtype=torch.int32, device="cuda") for d in dems]
    obsps = [torch.empty((shots_each, max(rbp.words(d.k), 1)), dtype=torch.int32, device="cuda") for d in dems]
    st = torch.empty((total, 32), dtype=torch.uint8, device="cuda")
    res = {"models": [{"name": nm, "M": d.M, "N": d.N, "nnz": d.nnz, "k": d.k} for nm, d in zip(names, dems)],
           "shots_each": shots_each, "one_launch": {}, "per_model_launches": {}}
    # one launch, every launch shape (0 = the library's choice)
    for waves in (0, 4, 8, 16):
        for state in (0, 1, 3):
            try:
                codes[0].set_launch_config(waves, state, 0)
                ms, _ = _timed(lambda: rbp.decode_multi(codes, [d.priors for d in dems], shot_code, shot_index,
                                                        syns, params, corrs, obsps, st))
                res["one_launch"][f"waves{waves}_state{state}"] = {"ms": ms, "shots_per_s": total / (ms * 1e-3)}
            except rbp.RbpError as ex:
                res["one_launch"][f"waves{waves}_state{state}"] = {"error": str(ex)}
    best = min((v for v in res["one_launch"].values() if "ms" in v), key=lambda v: v["ms"])
    res["one_launch_best"] = best
    codes[0].set_launch_config(0, 0, 0)
    # per model, each tuned
    tot_ms = 0.0
    for nm, d, c, syn in zip(names, dems, codes, syns):
        tr = autotune.tune(c, d.H, d.priors, params, use_cache=False)
        ms, _ = _timed(lambda: c.decode(d.priors, syn, params))
        tot_ms += ms
        res["per_model_launches"][nm] = {"ms": ms, "shots_per_s": shots_each / (ms * 1e-3),
                                         "waves": tr["waves_per_shot"], "state": tr["state"],
                                         "shots_per_wg": tr["shots_per_wg"]}
    res["per_model_total"] = {"ms": tot_ms, "shots_per_s": total / (tot_ms * 1e-3)}
    # the same tuned launches issued together on side streams (rbp_decode_each)
    ms, _ = _timed(lambda: rbp.decode_each(codes, [d.priors for d in dems], syns, params))
    res["per_model_concurrent"] = {"ms": ms, "shots_per_s": total / (ms * 1e-3)}
    return res


def large(name: str, shots: int, seed: int = 21, params: rbp.RelayParams | None = None, tune: bool = True) -> dict:
    params = params or rbp.RelayParams()
    t0 = time.perf_counter()
    dem = workloads.workload(name)
    t1 = time.perf_counter()
    code = rbp.Code.from_dem(dem)
    tr = autotune.tune(code, dem.H, dem.priors, params, shots=min(shots, 4000), use_cache=False) if tune else None
    syn, obs, _ = code.sample(dem.priors, shots, seed)
    ms, out = _timed(lambda: code.decode(dem.priors, syn, params), repeats=2)
    r = _summary(dem, obs, out[1], out[2], shots, ms)
    r.update({"model": {"name": name, "M": dem.M, "N": dem.N, "nnz": dem.nnz, "k": dem.k, "rounds": dem.rounds},
              "build_s": t1 - t0, "tuned": tr, "launch": code.launch_config(),
              "algorithmic_bytes_per_shot_iteration": 8 * dem.nnz + 8 * dem.N})
    it = rbp.stats_to_numpy(out[2])["iters"].astype(np.float64).sum()
    r["algorithmic_GBps"] = it * (8 * dem.nnz + 8 * dem.N) / (ms * 1e-3) / 1e9
    return r


def latency(name: str, shots: int = 300, all_shots: int = 100, seed: int = 31) -> dict:
    params = rbp.RelayParams()
    dem = workloads.workload(name)
    code = rbp.Code.from_dem(dem)
    syn, _, _ = code.sample(dem.priors, shots, seed)
    out = code.decode(dem.priors, syn[:1], params)
    torch.cuda.synchronize()
    lat = []
    for i in range(shots):
        t0 = time.perf_counter()
        code.decode(dem.priors, syn[i:i + 1], params, out=out)
        torch.cuda.synchronize()
        lat.append(1e6 * (time.perf_counter() - t0))
    allp = rbp.RelayParams(stopping_criterion=1)
    lat_all = []
    for i in range(all_shots):
        t0 = time.perf_counter()
        code.decode(dem.priors, syn[i:i + 1], allp, out=out)
        torch.cuda.synchronize()
        lat_all.append(1e6 * (time.perf_counter() - t0))
    return {"model": {"name": name, "M": dem.M, "N": dem.N, "nnz": dem.nnz},
            "sequential_us": stats.percentiles(np.array(lat)),
            "all_legs_us": stats.percentiles(np.array(lat_all)), "launch": code.launch_config()}


def resident_exp(name: str, p: float = 1e-3, shots: int = 100, block: int = 20, workgroups: int = 0,
                 seed: int = 51) -> dict:
    """Per-call latency mode against the resident decoder on the same shots, in
    alternating blocks (a fresh resident launch per block), so that both see
    the same conditions.  Circuit-level models ("circ320x") take the relay
    interval of Table "relay gamma intervals" and 1,000 legs; the others the
    default parameters."""
    import sys
    dem, priors = _model_at(name, p)
    if name.startswith("circ"):
        gmin, gmax = CIRCUIT_GAMMA[f"ZSZ-LP-{name[4:-1]}"]
        params = rbp.RelayParams(num_sets=1000, gamma_min=gmin, gamma_max=gmax)
    else:
        params = rbp.RelayParams()
    code = rbp.Code.from_dem(dem)
    coop = rbp.CoopParams(workgroups=workgroups)
    syn, _, _ = code.sample(priors, shots, seed)
    hsyn = syn.cpu().numpy().view(np.uint32)
    out = code.decode_coop(priors, syn[:1], params, coop)
    torch.cuda.synchronize()
    host = {"per_call": np.zeros(shots), "resident": np.zeros(shots)}
    dev = {"per_call": np.zeros(shots), "resident": np.zeros(shots)}
    xcds = []
    for b0 in range(0, shots, block):
        idx = range(b0, min(shots, b0 + block))
        for i in idx:
            t0 = time.perf_counter()
            code.decode_coop(priors, syn[i:i + 1], params, coop, out=out)
            torch.cuda.synchronize()
            host["per_call"][i] = 1e6 * (time.perf_counter() - t0)
            st = rbp.stats_to_numpy(out[2])
            dev["per_call"][i] = (int(st["t_end"][0]) - int(st["t_start"][0])) / 100.0
        with code.resident(priors, params, coop, idle_seconds=10.0) as rd:
            rd.decode(hsyn[idx[0]])
            for i in idx:
                t0 = time.perf_counter()
                _, _, st = rd.decode(hsyn[i])
                host["resident"][i] = 1e6 * (time.perf_counter() - t0)
                dev["resident"][i] = (int(st["t_end"]) - int(st["t_start"])) / 100.0
            xcds.append(rd.info()["xcds"])
        print(f"[resident] {name}: block {b0 // block + 1} done", file=sys.stderr, flush=True)
    code.close()
    ratio = dev["resident"] / np.maximum(dev["per_call"], 1e-9)
    return {"model": name, "p": p, "dem": [dem.M, dem.N], "shots": shots, "block": block,
            "coop_workgroups": workgroups, "device_clock_mhz": 100,
            "host_us": {k: stats.percentiles(v) for k, v in host.items()},
            "device_us": {k: stats.percentiles(v) for k, v in dev.items()},
            "host_minus_device_us_p50": {k: float(np.median(host[k] - dev[k])) for k in host},
            "resident_over_per_call_device_median": float(np.median(ratio)), "resident_xcd_masks": xcds}


# Table "relay gamma intervals" (App. "more numerics"): [gamma_min, gamma_max]
# of each code's circuit-level memory decoding
CIRCUIT_GAMMA = {"ZSZ-LP-160": (-0.15, 0.61), "ZSZ-LP-240": (-0.1, 0.6), "ZSZ-LP-320": (-0.16, 0.66),
                 "ZSZ-LP-390": (-0.16, 0.7), "ZSZ-LP-550": (-0.12, 0.62)}


def _seq_latency(code, priors, syn, params, n: int) -> np.ndarray:
    out = code.decode(priors, syn[:1], params)
    torch.cuda.synchronize()
    lat = []
    for i in range(n):
        t0 = time.perf_counter()
        code.decode(priors, syn[i:i + 1], params, out=out)
        torch.cuda.synchronize()
        lat.append(1e6 * (time.perf_counter() - t0))
    return np.array(lat)


def circuit_exp(codes, p: float = 1e-3, shots: int = 100000, seq_shots: int = 300, all_shots: int = 3,
                num_sets: int = 1000, bases: str = "XZ", seed: int = 61, tune: bool = True) -> dict:
    import sys
    rows = []
    for name in codes:
        gmin, gmax = CIRCUIT_GAMMA[name]
        params = rbp.RelayParams(num_sets=num_sets, gamma_min=gmin, gamma_max=gmax)
        for basis in bases:
            t0 = time.perf_counter()
            dem = circuits.memory_dem(name, basis, p)
            build_s = time.perf_counter() - t0
            code = rbp.Code.from_dem(dem)
            tr = autotune.tune(code, dem.H, dem.priors, params, shots=4000, use_cache=False) if tune else None
            syn, obs, _ = code.sample(dem.priors, shots, seed)
            ms, out = _timed(lambda: code.decode(dem.priors, syn, params), repeats=2)
            r = _summary(dem, obs, out[1], out[2], shots, ms)
            st = rbp.stats_to_numpy(out[2])
            it = st["iters"].astype(np.float64).sum()
            print(f"[circuit] {name} {basis}: batched {r['shots_per_s']:.0f} shots/s", file=sys.stderr, flush=True)
            # one shot per launch: the widest workgroup (16 waves) on the shot
            tuned = code.launch_config()
            code.set_launch_config(16, 2, 0)
            seq = _seq_latency(code, dem.priors, syn, params, seq_shots)
            # the all-legs worst case (num_sets + 1 legs) on the first shots with a
            # nonzero syndrome, in latency mode below
            nzs = [i for i in range(min(shots, 1000)) if bool(syn[i].any())][:all_shots]
            code.set_launch_config(tuned["waves_per_shot"], tuned["state"], 0)
            # latency mode: each shot spread over the CUs of one XCD
            out1 = code.decode_coop(dem.priors, syn[:1], params)
            torch.cuda.synchronize()
            lat_c = []
            for i in range(seq_shots):
                t1 = time.perf_counter()
                code.decode_coop(dem.priors, syn[i:i + 1], params, out=out1)
                torch.cuda.synchronize()
                lat_c.append(1e6 * (time.perf_counter() - t1))
            lat_c = np.array(lat_c)
            lat_all_c = []
            for i in nzs:
                t1 = time.perf_counter()
                code.decode_coop(dem.priors, syn[i:i + 1], dataclasses.replace(params, stopping_criterion=1), out=out1)
                torch.cuda.synchronize()
                lat_all_c.append(1e3 * (time.perf_counter() - t1))
            if code.coop_aborted():
                raise RuntimeError("latency-mode launch stopped on an expired barrier wait")
            print(f"[circuit] {name} {basis}: sequential mean {seq.mean():.0f} us (one CU), "
                  f"{lat_c.mean():.0f} us (latency mode); all-legs {np.mean(lat_all_c):.1f} ms (latency mode)",
                  file=sys.stderr, flush=True)
            r.update({"code": name, "basis": basis, "p": p, "rounds": dem.rounds,
                      "dem": {"N_det": dem.M, "N_loc": dem.N, "nnz": dem.nnz, "k": dem.k,
                              "max_row_deg": int(dem.H.sum(axis=1).max()),
                              "paper_size": circuits.PAPER_DEM_SIZES.get(name)},
                      "build_s": build_s, "relay": dataclasses.asdict(params), "tuned": tr,
                      "launch": tuned, "sequential_launch": {"waves_per_shot": 16, "state": 2},
                      "nonconverged": int((st["converged"] == 0).sum()),
                      "algorithmic_GBps": it * (8 * dem.nnz + 8 * dem.N) / (ms * 1e-3) / 1e9,
                      "sequential_one_cu_us": stats.percentiles(seq),
                      "latency_mode_us": stats.percentiles(lat_c),
                      "latency_mode_launch": {"workgroups": torch.cuda.get_device_properties(0).multi_processor_count // 8, "stride": 8, "waves": 8},
                      "latency_mode_all_legs_ms": stats.percentiles(np.array(lat_all_c))})
            rows.append(r)
            code.close()
    return {"experiment": "circuit-level memory", "rows": rows}


def learned_exp(name: str, pairs: int, eval_shots: int, p_eval, p_lo: float, p_hi: float) -> dict:
    dem = workloads.workload(name)
    cfg = learned.TrainConfig(pairs=pairs, p_lo=p_lo, p_hi=p_hi)
    evals = {f"{p:g}": np.full(dem.N, p) for p in p_eval}
    return learned.train_and_evaluate(dem, cfg, evals, eval_shots, 777)


# code distances d of Table 1 (Sec. 1); the phenomenological models have no
# hook errors, so their effective distance is d itself
CODE_DISTANCE = {"cc160": 10, "phen160": 10, "phen240": 12, "phen320": 14, "phen390": 16, "phen550": 18,
                 "phen775": 22}


# shots per decode call of the LER experiments: slow points (circuit-level DEMs
# near threshold, where non-converging shots run every relay leg) report
# progress after each chunk
CHUNK = 20000


def _failures(code, dem, priors, syn, obs, params) -> tuple:
    import sys
    n = syn.shape[0]
    f = it = nc = 0
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        corr, obsp, st = code.decode(priors, syn[a:b], params)
        s = rbp.stats_to_numpy(st)
        f += int(stats.block_failures(rbp.to_u32(obsp), rbp.to_u32(obs[a:b]), s["converged"]).sum())
        it += float(s["iters"].astype(np.float64).sum())
        nc += int((s["converged"] == 0).sum())
        if n > CHUNK:
            print(f"[chunk] {b}/{n} shots: {f} failures", file=sys.stderr, flush=True)
    return f, it / max(n, 1), nc


def _model_at(name: str, p: float):
    """(DEM, priors) of a named model at noise strength p: a circuit-level
    memory ("circ160x": ZSZ-LP-160, X basis) carries its own merged priors,
    the other models take p for every mechanism."""
    if name.startswith("circ"):
        dem = circuits.memory_dem(f"ZSZ-LP-{name[4:-1]}", name[-1].upper(), p)
        return dem, dem.priors
    dem = workloads.workload(name)
    return dem, np.full(dem.N, p)


def gamma_grid(name: str, p: float, gmins, gmaxs, shots: int, seed: int = 41,
               params: rbp.RelayParams | None = None) -> dict:
    """Grid search of [gamma_min, gamma_max] for the lowest LER at noise p.

    Every interval decodes the same sampled syndromes, so the comparison is
    paired.  The chosen interval has the fewest failures; among equal counts
    the one with fewer BP iterations per shot, then the earlier grid point
    (gamma_min outer, gamma_max inner loop).  Intervals with gamma_min >
    gamma_max are skipped.
    """
    import sys
    base = params or rbp.RelayParams()
    dem, priors = _model_at(name, p)
    code = rbp.Code.from_dem(dem)
    syn, obs, _ = code.sample(priors, shots, seed)
    rows = []
    for gmin in gmins:
        for gmax in gmaxs:
            if gmin > gmax:
                continue
            prm = dataclasses.replace(base, gamma_min=float(gmin), gamma_max=float(gmax))
            f, it, nc = _failures(code, dem, priors, syn, obs, prm)
            lo, hi = stats.clopper_pearson(f, shots)
            rows.append({"gamma_min": float(gmin), "gamma_max": float(gmax), "failures": f, "ler": f / shots,
                         "ci95": [lo, hi], "mean_iters": it, "nonconverged": nc})
            print(f"[gamma] {name} [{gmin}, {gmax}]: {f} failures, {it:.1f} iterations", file=sys.stderr,
                  flush=True)
    best = min(range(len(rows)), key=lambda i: (rows[i]["failures"], rows[i]["mean_iters"], i))
    return {"model": name, "p": p, "shots": shots, "seed": seed, "grid": rows, "best": rows[best]}


def ler_sweep(name: str, ps, shots: int, seed: int = 51, params: rbp.RelayParams | None = None,
              d_circ: float | None = None, p_fit_max: float = 4e-3, p_eval: float = 1e-3) -> dict:
    """LER per qubit-round against p, and the sub-threshold fit (Sec. 6.1).

    The fit uses the points with p <= p_fit_max and at least one failure,
    weighted by their failure counts, with d_circ defaulting to the code
    distance; the fitted curve is evaluated at p_eval.
    """
    import sys
    params = params or rbp.RelayParams()
    dem, _ = _model_at(name, ps[0])
    code = rbp.Code.from_dem(dem)
    if d_circ is None:
        # circuit-level models: d_circ = d - 2 as the paper takes (App. "more numerics")
        d_circ = (circuits.DISTANCE[f"ZSZ-LP-{name[4:-1]}"] - 2 if name.startswith("circ")
                  else CODE_DISTANCE.get(name, 0))
    d_circ = float(d_circ)
    rows = []
    for i, p in enumerate(ps):
        _, priors = _model_at(name, p)  # the same mechanisms at every p, only their priors change
        syn, obs, _ = code.sample(priors, shots, seed + i)
        f, it, nc = _failures(code, dem, priors, syn, obs, params)
        s = stats.ler_summary(f, shots, dem.rounds, dem.k)
        lo, hi = s["ci95"]
        rows.append({"p": float(p), **s, "per_qubit_round_ci95": [stats.per_round(lo, dem.rounds * dem.k),
                                                                   stats.per_round(hi, dem.rounds * dem.k)],
                     "mean_iters": it, "nonconverged": nc})
        print(f"[sweep] {name} p = {p:g}: {f} failures, {it:.1f} iterations", file=sys.stderr, flush=True)
    out = {"model": name, "rounds": dem.rounds, "k": dem.k, "shots_per_point": shots, "seed": seed,
           "d_circ": d_circ, "gamma": [params.gamma_min, params.gamma_max], "points": rows}
    fit = [r for r in rows if r["p"] <= p_fit_max and r["failures"] > 0]
    if len(fit) >= 3 and d_circ > 0:
        c = stats.fit_ler([r["p"] for r in fit], [r["per_qubit_round"] for r in fit], d_circ,
                          [r["failures"] for r in fit])
        out["fit"] = {"c": list(c), "points": len(fit), "p_fit_max": p_fit_max,
                      "per_qubit_round_at": {f"{p_eval:g}": float(stats.ler_model(p_eval, c, d_circ))}}
    return out


def windowed(code_name: str = "ZSZ-LP-160", rounds: int = 30, p: float = 8e-3, shots: int = 200000,
             configs=((10, 1), (10, 5), (5, 1)), seed: int = 71, params: rbp.RelayParams | None = None,
             latency_shots: int = 300, parallel=((5, 3, 3), (4, 3, 2), (6, 4, 4))) -> dict:
    """Sliding-window and parallel-window against global decoding of one
    T-round memory experiment (parallel: (core, buffer, gap) in rounds)."""
    params = params or rbp.RelayParams()
    dem = workloads.phenomenological_dem(workloads.zsz_lp(code_name), rounds, p)
    m = dem.M // rounds
    code = rbp.Code.from_dem(dem)
    syn, obs, _ = code.sample(dem.priors, shots, seed)

    def summary(obsp, st, ms):
        s = rbp.stats_to_numpy(st)
        f = stats.block_failures(rbp.to_u32(obsp), rbp.to_u32(obs), s["converged"])
        return {"ms": ms, "shots_per_s": shots / (ms * 1e-3), "rounds_per_s": shots * rounds / (ms * 1e-3),
                "ler": stats.ler_summary(int(f.sum()), shots, rounds, dem.k),
                "nonconverged": int((s["converged"] == 0).sum()), "mean_iters": float(s["iters"].mean())}

    out = {"model": f"{code_name} phenomenological, T = {rounds}, p = {p:g}", "M": dem.M, "N": dem.N,
           "shots": shots, "seed": seed}
    ms, (corr, obsp, st) = _timed(lambda: code.decode(dem.priors, syn, params))
    out["global"] = summary(obsp, st, ms)
    for w, c in configs:
        dec = window.SlidingWindowDecoder(dem.H, dem.O, m, w, c)
        ms, (corr, obsp, st) = _timed(lambda: dec.decode(dem.priors, syn, params))
        r = summary(obsp, st, ms)
        r["windows"] = len(dec.windows)
        # single-shot latency of one full-size window, host clock around each
        # call: the first window, whose syndrome is the sampled one (an
        # interior window's syndrome exists only after the earlier commits)
        win = dec.windows[0]
        nb = win.rounds * m
        buf = torch.empty((1, rbp.words(nb)), dtype=torch.int32, device=syn.device)
        o1 = (torch.empty((1, rbp.words(win.cols.size)), dtype=torch.int32, device=syn.device),
              torch.empty((1, 1), dtype=torch.int32, device=syn.device),
              torch.empty((1, 32), dtype=torch.uint8, device=syn.device))
        pr = dem.priors[win.cols]
        lat = []
        for i in range(latency_shots):
            rbp.bits_extract(syn[i:i + 1], win.start * m, nb, buf)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            win.code.decode(pr, buf, params, out=o1)
            torch.cuda.synchronize()
            lat.append(1e6 * (time.perf_counter() - t0))
        r["window_latency_us"] = stats.percentiles(np.array(lat))
        r["window_shape"] = {"rounds": win.rounds, "detectors": nb, "mechanisms": int(win.cols.size)}
        out[f"w{w}_c{c}"] = r
        dec.close()
    for core, buf, gap in parallel:
        dec = window.ParallelWindowDecoder(dem.H, dem.O, m, core, buf, gap)
        ms, (corr, obsp, st) = _timed(lambda: dec.decode(dem.priors, syn, params))
        r = summary(obsp, st, ms)
        r["windows"] = {"A": len(dec.layers[0]), "B": len(dec.layers[1]), "distinct_matrices": len(dec.codes)}
        out[f"parallel_core{core}_buffer{buf}_gap{gap}"] = r
        dec.close()
    return out


def awgn_fer(names, ebn0s, max_frames: int = 10 ** 7, min_errors: int = 100, chunk: int = 10 ** 6,
             seed: int = 61, params: rbp.SpaParams | None = None, side: str = "left") -> dict:
    """Frame (block) error rate of the all-zero codeword over BPSK-AWGN.

    Frames are drawn in chunks (shot offsets continue across chunks, so the
    frames are those of one seeded stream) until min_errors block errors or
    max_frames frames.  A block error is a decoded word other than the
    all-zero one; an undetected error is such a word that satisfies every
    check.  Throughput counts decode launches only, and separately the whole
    sample + decode loop.
    """
    params = params or rbp.SpaParams()
    out = {"shannon_limit_db": stats.shannon_limit_db(0.5), "params": dataclasses.asdict(params), "codes": {}}
    for name in names:
        H = workloads.zsz_2bga(name, side)
        n = H.shape[1]
        k = n - workloads.gf2_rank(H)
        rate = k / n
        code = rbp.Code(H, np.zeros((0, n), dtype=np.uint8))
        dev = torch.device("cuda")
        cap = min(chunk, max_frames)
        llr = torch.empty((cap, n), dtype=torch.float32, device=dev)
        bits = torch.empty((cap, rbp.words(n)), dtype=torch.int32, device=dev)
        st = torch.empty((cap, 32), dtype=torch.uint8, device=dev)
        rows = []
        for ebn0 in ebn0s:
            sigma = workloads.awgn_sigma(ebn0, rate)
            counts = torch.zeros(3, dtype=torch.int64, device=dev)
            iters = torch.zeros(1, dtype=torch.int64, device=dev)
            frames, dec_ms = 0, 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while frames < max_frames and int(counts[0].item()) < min_errors:
                m = min(cap, max_frames - frames)
                code.sample_awgn(m, sigma, seed, shot_offset=frames, out=llr[:m])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                code.decode_spa(llr[:m], params, counts=counts, out=(bits[:m], None, st[:m]))
                e1.record()
                iters += st[:m].view(torch.int32)[:, 2].sum()
                torch.cuda.synchronize()
                dec_ms += e0.elapsed_time(e1)
                frames += m
            wall = time.perf_counter() - t0
            c = counts.cpu().numpy()
            lo, hi = stats.clopper_pearson(int(c[0]), frames)
            rows.append({"ebn0_db": ebn0, "sigma": sigma, "frames": frames, "block_errors": int(c[0]),
                         "undetected": int(c[1]), "nonconverged": int(c[2]), "fer": c[0] / frames,
                         "ci95": [lo, hi], "mean_iters": float(iters.item()) / frames,
                         "decode_frames_per_s": frames / (dec_ms * 1e-3), "frames_per_s": frames / wall})
        out["codes"][name] = {"n": n, "k": k, "side": side, "points": rows}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what")
    ap.add_argument("--models", default="phen160,phen320,phen550,phen775")
    ap.add_argument("--model", default="phen840")
    ap.add_argument("--shots", type=int, default=100000)
    ap.add_argument("--pairs", type=int, default=1000000)
    ap.add_argument("--p-eval", default="1e-3")
    ap.add_argument("--p-range", default="5e-4,2e-3")
    ap.add_argument("--p", type=float, default=1e-2)
    ap.add_argument("--gmin", default="-0.3,-0.24,-0.15,-0.1,0.0")
    ap.add_argument("--gmax", default="0.5,0.6,0.66,0.75")
    ap.add_argument("--ps", default="4e-3,6e-3,8e-3,1e-2,1.2e-2,1.5e-2")
    ap.add_argument("--p-fit-max", type=float, default=1e-2)
    ap.add_argument("--codes", default="ZSZ-2BGA-64,ZSZ-2BGA-96,ZSZ-2BGA-128,ZSZ-2BGA-156,ZSZ-2BGA-220,ZSZ-2BGA-310")
    ap.add_argument("--ebn0", default="0.5,1.0,1.25,1.5,2.0,2.5,3.0,3.5,4.0")
    ap.add_argument("--max-frames", type=int, default=10 ** 7)
    ap.add_argument("--min-errors", type=int, default=100)
    ap.add_argument("--rounds", type=int, default=30)
    ap.add_argument("--p-window", type=float, default=8e-3)
    ap.add_argument("--num-sets-grid", type=int, default=100, help="relay legs of the gamma and sweep runs")
    ap.add_argument("--sweep-gamma", default="-0.24,0.66", help="relay interval of the sweep")
    ap.add_argument("--circuit-codes", default="ZSZ-LP-320,ZSZ-LP-390,ZSZ-LP-550")
    ap.add_argument("--p-circuit", type=float, default=1e-3)
    ap.add_argument("--seq-shots", type=int, default=300)
    ap.add_argument("--all-shots", type=int, default=3)
    ap.add_argument("--num-sets", type=int, default=1000)
    ap.add_argument("--bases", default="XZ")
    ap.add_argument("--chunk", type=int, default=20000, help="shots per decode call of the LER experiments")
    ap.add_argument("--seed", type=int, default=51,
                    help="syndrome seed of the sweep (point i draws from seed + i); change it to add shots to a point")
    a = ap.parse_args()
    global CHUNK
    CHUNK = max(1, a.chunk)
    torch.cuda.set_device(0)
    if a.what == "multi":
        r = multi(a.models.split(","), a.shots)
    elif a.what == "large":
        r = large(a.model, a.shots)
    elif a.what == "latency":
        r = latency(a.model, a.shots)
    elif a.what == "learned":
        lo, hi = (float(x) for x in a.p_range.split(","))
        r = learned_exp(a.model, a.pairs, a.shots, [float(x) for x in a.p_eval.split(",")], lo, hi)
    elif a.what == "gamma":
        r = gamma_grid(a.model, a.p, [float(x) for x in a.gmin.split(",")], [float(x) for x in a.gmax.split(",")],
                       a.shots, params=rbp.RelayParams(num_sets=a.num_sets_grid))
    elif a.what == "window":
        r = windowed(rounds=a.rounds, p=a.p_window, shots=a.shots)
    elif a.what == "awgn":
        r = awgn_fer(a.codes.split(","), [float(x) for x in a.ebn0.split(",")], a.max_frames, a.min_errors)
    elif a.what == "circuit":
        r = circuit_exp(a.circuit_codes.split(","), a.p_circuit, a.shots, a.seq_shots, a.all_shots, a.num_sets,
                        a.bases)
    elif a.what == "resident":
        r = resident_exp(a.model, a.p_circuit, a.seq_shots, 20)
    elif a.what == "sweep":
        gmin, gmax = (float(x) for x in a.sweep_gamma.split(","))
        r = ler_sweep(a.model, [float(x) for x in a.ps.split(",")], a.shots, seed=a.seed, p_fit_max=a.p_fit_max,
                      params=rbp.RelayParams(gamma_min=gmin, gamma_max=gmax, num_sets=a.num_sets_grid))
    else:
        raise SystemExit(__doc__)
    # every handle closed and the device idle before the interpreter exits
    rbp._close_all()
    torch.cuda.synchronize()
    print(json.dumps(r, default=float), flush=True)


if __name__ == "__main__":
    main()
