#!/usr/bin/env python3
"""Benchmark of the Monte-Carlo Relay-BP path on one MI355X.

One step = sample a batch of shots of the phenomenological ZSZ-LP-160 model
(9 rounds, 576 detectors x 1952 mechanisms, priors 1e-3) on the GPU, decode it
with Relay-BP (gamma0 0.125, pre_iter 80, max_iterations 60, 100 relay legs,
stop_nconv 5, gamma in [-0.24, 0.66]) and count block failures on the GPU; the
failure count comes back to the host at the end of the timed steps.  The
learned path adds the proposal network's forward pass before decoding.
Beside the headline: the classical AWGN benchmark, sequential single-shot
latency, and the paper's latency-table workload (circuit-level ZSZ-LP-320
memory decoded one shot at a time in latency mode).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded shots/s + p50/p99 latency at fixed LER: Relay-BP vs learned proposal"
LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz = 78643 GB/s
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shots", type=int, default=100000)
    ap.add_argument("--workload", default="phen160")
    ap.add_argument("--seed", type=int, default=20260101)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-pairs", type=int, default=1_000_000)
    ap.add_argument("--no-awgn", action="store_true")
    ap.add_argument("--no-circuit", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates rocprof byte counters)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("rbp_decode.hip", "rbp_common.h"):
        h.update(open(os.path.join(ROOT, "paper_2607_27644_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, launch_shots: int):
    """HBM bytes per decode launch from the committed counter summary, if it was
    taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"relay_bp_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("shots") != launch_shots:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(dem, shots_total: int, seed: int, params, target_s: float):
    import numpy as np

    import oracle
    threads = min(16, os.cpu_count() or 1)
    g = oracle.Graph(dem.H, dem.O)
    op = oracle.RelayParams(**{k: getattr(params, k) for k in oracle.RelayParams.__dataclass_fields__})

    def run(n):
        t0 = time.perf_counter()
        syn, obs, _ = oracle.sample(g, dem.priors, n, seed)
        r = oracle.decode(g, dem.priors, syn, op, nthreads=threads, timing=True)
        return time.perf_counter() - t0, r

    dt, _ = run(2000)
    # about target_s of work, at most 10 steps' worth of shots
    n = int(min(10 * shots_total, max(2000, 2000 * target_s / max(dt, 1e-3))))
    dt, r = run(n)
    return {"value": n / dt, "unit": "shots/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} shots of the same model and seed (the first {min(n, shots_total)} are the first "
                      f"timed step's shots): oracle sampling + Relay-BP decode on {threads} threads, {dt:.1f} s",
            "mean_iters_per_shot": float(np.mean(r["iters"])),
            # each shot runs on one thread: its decode time is single-core latency
            "single_core_latency_us": {"p50": float(np.percentile(r["seconds"], 50) * 1e6),
                                       "p99": float(np.percentile(r["seconds"], 99) * 1e6)},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def circuit_latency(seed: int, shots: int = 100, batch: int = 4000) -> dict:
    """The paper's latency table workload: circuit-level d-round memory of
    ZSZ-LP-320 (DEM 1920 x 28992), p = 1e-3, num_sets 1000, gamma in
    [-0.16, 0.66]; single shots in latency mode (one XCD's CUs per shot, host
    clock around each call) and one batched launch, X and Z memory."""
    import numpy as np
    import torch
    from paper_2607_27644_amd import circuits, experiments, rbp, stats
    gmin, gmax = experiments.CIRCUIT_GAMMA["ZSZ-LP-320"]
    params = rbp.RelayParams(num_sets=1000, gamma_min=gmin, gamma_max=gmax)
    res = {"code": "ZSZ-LP-320", "p": 1e-3, "relay": {"num_sets": 1000, "gamma": [gmin, gmax]}}
    lat_all = []
    for basis in "XZ":
        dem = circuits.memory_dem("ZSZ-LP-320", basis, 1e-3)
        code = rbp.Code.from_dem(dem)
        syn, obs, _ = code.sample(dem.priors, batch, seed)
        out = code.decode_coop(dem.priors, syn[:1], params)
        torch.cuda.synchronize()
        lat = []
        for i in range(shots):
            t0 = time.perf_counter()
            code.decode_coop(dem.priors, syn[i:i + 1], params, out=out)
            torch.cuda.synchronize()
            lat.append(1e6 * (time.perf_counter() - t0))
        if code.coop_aborted():
            raise RuntimeError("latency-mode launch stopped on an expired barrier wait")
        code.set_launch_config(8, 2, 0)
        corr, obsp, st = code.decode(dem.priors, syn, params)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        code.decode(dem.priors, syn, params, out=(corr, obsp, st))
        e1.record()
        torch.cuda.synchronize()
        s = rbp.stats_to_numpy(st)
        res[f"{basis}_memory"] = {"dem": [dem.M, dem.N], "latency_mode_us": stats.percentiles(np.array(lat)),
                                  "batched_shots_per_s": batch / (e0.elapsed_time(e1) * 1e-3),
                                  "mean_iters": float(s["iters"].mean())}
        lat_all += lat
        code.close()
    res["latency_mode_us_xz"] = stats.percentiles(np.array(lat_all))
    res["paper_l40s_ms"] = {"mean": 1.2, "p99": 2.0, "p99.9": 3.2, "note": "NVIDIA L40S, Table 'decoding latency'"}
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; shots shard across GPUs by "
                                   "shot_offset with no communication, so run one process per GPU "
                                   "(multi-GPU launch is not part of this build)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_27644_amd import rbp, stats, workloads

    torch.cuda.set_device(0)
    dem = workloads.workload(args.workload)
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    S = args.shots
    dev = torch.device("cuda")
    syn = torch.empty((S, rbp.words(dem.M)), dtype=torch.int32, device=dev)
    obs = torch.empty((S, max(rbp.words(dem.k), 1)), dtype=torch.int32, device=dev)
    corr = torch.empty((S, rbp.words(dem.N)), dtype=torch.int32, device=dev)
    obsp = torch.empty_like(obs)
    st = torch.empty((S, 32), dtype=torch.uint8, device=dev)
    fail_count = torch.zeros(1, dtype=torch.int64, device=dev)

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ev = []
    net = None
    delta_buf = None

    def step(i: int, record: bool, path: str = "plain"):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record:
            e[0].record()
        code.sample(dem.priors, S, args.seed + i, out=(syn, obs, None))
        if record:
            e[1].record()
        delta = None
        if path == "learned":
            delta = net.forward(syn, out=delta_buf)
        elif path == "proposal_zero":
            delta = delta_buf
        if record:
            e[2].record()
        code.decode(dem.priors, syn, params, delta=delta, out=(corr, obsp, st))
        if record:
            e[3].record()
            ev.append(e)
        rbp.count_failures(obsp, obs, st, fail_count)
        return None

    def timed(path: str):
        ev.clear()
        for i in range(args.warmup):
            step(1000 + i, False, path)
        torch.cuda.synchronize()
        fail_count.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(i, True, path)
        fail_total = int(fail_count.item())  # synchronizes: the steps' work is inside the window
        wall = time.perf_counter() - t0
        last = rbp.stats_to_numpy(st).copy()
        ms = lambda a, b: float(np.mean([e[a].elapsed_time(e[b]) for e in ev]))
        return {"wall": wall, "fails": fail_total, "last": last, "sample_ms": ms(0, 1), "mlp_ms": ms(1, 2),
                "decode_ms": ms(2, 3)}

    P = timed("plain")
    wall, fail_total, last = P["wall"], P["fails"], P["last"]
    ms_step = 1e3 * wall / args.steps
    value = S * args.steps / wall

    dec_ms, smp_ms = P["decode_ms"], P["sample_ms"]
    iters = last["iters"].astype(np.int64)
    B_it = 8 * dem.nnz + 8 * dem.N  # algorithmic bytes of one flooding iteration of one shot
    alg_bytes = float(iters.sum()) * B_it
    achieved = alg_bytes / (dec_ms * 1e-3) / 1e9
    traffic = load_traffic(args.workload, S)

    ticks = (last["t_end"] - last["t_start"]).astype(np.float64)
    service_us = ticks * 0.01  # 100 MHz device wall clock
    nz = last["path"] != 3
    out = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": f"phenomenological DEM of ZSZ-LP-160 [[160,32,10]] over 9 rounds "
                        f"({dem.M} detectors x {dem.N} mechanisms, nnz {dem.nnz}), priors 1e-3, "
                        f"{S} shots per step, Relay-BP gamma0=0.125 pre_iter=80 max_iterations=60 "
                        f"num_sets=100 stop_nconv=5 gamma_dist=[-0.24,0.66], FP32 messages",
            "shots_per_step": S, "path": "plain Relay-BP (value); learned proposal and delta=0 control below",
        },
        "decode_only_shots_per_s": S / (dec_ms * 1e-3),
        "decode_kernel_ms": dec_ms, "sample_kernel_ms": smp_ms,
        "latency_us": {"batched_service_time": stats.percentiles(service_us),
                       "batched_service_time_nonzero_syndrome": stats.percentiles(service_us[nz])},
        "ler": stats.ler_summary(fail_total, S * args.steps, dem.rounds, dem.k),
        "mean_iters_per_shot": float(iters.mean()), "mean_legs_per_shot": float(last["legs"].mean()),
        "roofline": {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / LDS_PEAK_GBS, "traffic": traffic,
                     "kernel": "relay_bp_kernel", "algorithmic_bytes_per_shot_iteration": B_it,
                     "shot_iterations_per_launch": int(iters.sum())},
        "launch": code.launch_config(),
    }

    if not args.no_learned:
        from paper_2607_27644_amd import learned
        cfg = learned.TrainConfig(pairs=args.train_pairs)
        t0 = time.perf_counter()
        chunks = learned.generate_pairs(code, dem.priors, cfg, params)
        t1 = time.perf_counter()
        net = rbp.MLP(dem.M, cfg.hidden, dem.N, seed=cfg.seed)
        hist = learned.train(net, chunks, cfg)
        learned.scale_output(net, cfg.delta_scale)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del chunks
        delta_buf = torch.empty((S, dem.N), dtype=torch.float32, device=dev)
        paths = {}
        for path in ("learned", "proposal_zero"):
            if path == "proposal_zero":
                delta_buf.zero_()
            R = timed(path)
            it = R["last"]["iters"].astype(np.float64)
            sv = (R["last"]["t_end"] - R["last"]["t_start"]).astype(np.float64) * 0.01
            paths[path] = {
                "value": S * args.steps / R["wall"], "unit": "shots/s", "ms_per_step": 1e3 * R["wall"] / args.steps,
                "mlp_ms": R["mlp_ms"], "decode_kernel_ms": R["decode_ms"],
                "ler": stats.ler_summary(R["fails"], S * args.steps, dem.rounds, dem.k),
                "mean_iters_per_shot": float(it.mean()),
                "path_counts": {str(k): int((R["last"]["path"] == k).sum()) for k in range(4)},
                "latency_us": {"batched_service_time": stats.percentiles(sv)}}
        paths["learned"]["training"] = {"pairs": cfg.pairs, "p_range": [cfg.p_lo, cfg.p_hi], "epochs": cfg.epochs,
                                        "batch": cfg.batch, "hidden": cfg.hidden, "params": net.n_params,
                                        "delta_scale": cfg.delta_scale,
                                        "generate_s": t1 - t0, "train_s": t2 - t1, "final_loss": hist[-1][1]}
        paths["learned"]["vs_plain"] = paths["learned"]["value"] / value
        paths["proposal_zero"]["note"] = "control: the same proposal leg with delta = 0 (no network)"
        out["learned"] = paths["learned"]
        out["proposal_zero"] = paths["proposal_zero"]

    if not args.no_awgn:
        # the classical benchmark beside the headline: the [310,155] ZSZ-2BGA code
        # over BPSK-AWGN at 2.5 dB, sum-product BP (num_iter 100, llr_max 20)
        from paper_2607_27644_amd import experiments
        experiments.awgn_fer(["ZSZ-2BGA-310"], [2.5], max_frames=100_000, min_errors=10 ** 12, chunk=100_000)
        r = experiments.awgn_fer(["ZSZ-2BGA-310"], [2.5], max_frames=4_000_000, min_errors=10 ** 12,
                                 chunk=1_000_000)
        pt = r["codes"]["ZSZ-2BGA-310"]["points"][0]
        out["awgn"] = {"code": "ZSZ-2BGA-310 [310,155]", "ebn0_db": pt["ebn0_db"], "frames": pt["frames"],
                       "fer": pt["fer"], "ci95": pt["ci95"], "undetected": pt["undetected"],
                       "mean_iters": pt["mean_iters"], "decode_frames_per_s": pt["decode_frames_per_s"],
                       "frames_per_s_with_sampling": pt["frames_per_s"],
                       "shannon_limit_db": r["shannon_limit_db"]}

    if not args.no_sequential:
        # the paper's latency mode: one shot per decode call, host clock around each
        one_syn = syn[:1]
        lat = []
        c1, o1, s1 = corr[:1], obsp[:1], st[:1]
        for i in range(400):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            code.decode(dem.priors, syn[i:i + 1], params, out=(c1, o1, s1))
            torch.cuda.synchronize()
            lat.append(1e6 * (time.perf_counter() - ta))
        del one_syn
        out["latency_us"]["sequential_single_shot"] = stats.percentiles(np.array(lat))

    if not args.no_circuit:
        out["circuit_latency"] = circuit_latency(args.seed)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dem, S, args.seed, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
