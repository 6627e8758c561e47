#!/usr/bin/env python3
"""Benchmark of the Monte-Carlo Relay-BP path on one MI355X.

Workload: the largest single-GPU configuration, the 12-round phenomenological
detector error model of the [[840,168]] ZSZ-LP code (Table "more ZSZ-LP
codes"; 4032 detectors x 13776 mechanisms, nnz 43680), all priors 1e-3,
Relay-BP with gamma0 0.125, pre_iter 80, max_iterations 60, 100 relay legs,
stop_nconv 5, gamma in [-0.24, 0.66], FP32 messages.  One step = sample a
batch of shots on the GPU, decode it, count block failures on the GPU; the
failure count comes back to the host after the timed steps.

Paths, each timed the same way on the same shots:
  plain           Relay-BP (the headline `value`)
  first_solution  Relay-BP stopping at its first solution (stop_nconv 1): the
                  stop rule of the proposal path without a proposal
  learned         proposal network (trained in-run on decoder-generated pairs)
                  -> proposal leg, plain Relay-BP as the fallback
  proposal_zero   the same proposal leg with delta = 0 (no network)
Paired points at p = 5e-3 and 2.5e-2 decode the same syndromes with every
path (the [[840,168]] model shows no failure in 10^5 shots below about 2 %).  Beside the headline: sequential
single-shot latency (one decode call per shot, and the resident decoder fed
through pinned host memory), the batched uneven decode of four codes, the paper's
latency-table workload (circuit-level ZSZ-LP-320 memory), the classical AWGN
benchmark and the earlier ZSZ-LP-160 workload.  Prints one JSON line.
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
LDS_NOMINAL_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz (a CDNA3-style figure)
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def progress(msg: str):
    """One line per finished stage on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shots", type=int, default=100000)
    ap.add_argument("--workload", default="phen840")
    ap.add_argument("--seed", type=int, default=20260101)
    ap.add_argument("--ler-ps", default="5e-3,2.5e-2", help="noise strengths of the paired LER points")
    ap.add_argument("--ler-shots", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-first-solution", action="store_true")
    ap.add_argument("--train-pairs", type=int, default=1_000_000)
    ap.add_argument("--hidden", type=int, default=128, help="width of the proposal network's hidden layers")
    ap.add_argument("--delta-scale", type=float, default=0.5, help="shrinkage of the network's output")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary workloads")
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(dem, seed: int, params, target_s: float):
    """The oracle (sampler + Relay-BP) on the host's cores, on the first shots
    of the timed steps' seed."""
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

    dt, _ = run(1000)
    n = int(max(1000, 1000 * target_s / max(dt, 1e-3)))
    dt, r = run(n)
    return {"value": n / dt, "unit": "shots/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {n} shots of the first timed step (same model, seed and relay settings): "
                      f"oracle sampling + Relay-BP decode on {threads} threads, {dt:.1f} s",
            "mean_iters_per_shot": float(np.mean(r["iters"])),
            "single_core_latency_us": {"p50": float(np.percentile(r["seconds"], 50) * 1e6),
                                       "p99": float(np.percentile(r["seconds"], 99) * 1e6)},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def lds_peak():
    """Measured aggregate LDS read bandwidth (GB/s): the best of 4-, 8- and
    16-byte reads."""
    from paper_2607_27644_amd import rbp
    m = {w: rbp.measure_lds_bandwidth(w) / 1e9 for w in (4, 8, 16)}
    best = max(m, key=m.get)
    return m[best], {f"b{8 * w}": v for w, v in m.items()}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; shots shard across GPUs by "
                                   "shot_offset with no communication, so one process per GPU would each "
                                   "run it on its own shot range; no multi-GPU launcher is provided",
                          "n_gpus": args.gpus}))
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
    B_it = 8 * dem.nnz + 8 * dem.N  # algorithmic bytes of one flooding iteration of one shot

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    lds_gbs, lds_all = lds_peak()
    ev = []
    state = {"net": None, "delta": None}

    def step(i: int, record: bool, path: str, prm):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record:
            e[0].record()
        code.sample(dem.priors, S, args.seed + i, out=(syn, obs, None))
        if record:
            e[1].record()
        if path == "learned":
            state["net"].forward_bf16(syn, out=state["delta"])
        if record:
            e[2].record()
        if path in ("learned", "proposal_zero"):
            code.decode_proposal(dem.priors, syn, prm, state["delta"], out=(corr, obsp, st), by_position=True)
        else:
            code.decode(dem.priors, syn, prm, out=(corr, obsp, st))
        if record:
            e[3].record()
            ev.append(e)
        rbp.count_failures(obsp, obs, st, fail_count)

    def timed(path: str, prm):
        ev.clear()
        for i in range(args.warmup):
            step(1000 + i, False, path, prm)
        torch.cuda.synchronize()
        fail_count.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(i, True, path, prm)
        fails = int(fail_count.item())  # synchronizes: the steps' work is inside the window
        wall = time.perf_counter() - t0
        last = rbp.stats_to_numpy(st).copy()
        ms = lambda a, b: float(np.mean([x[a].elapsed_time(x[b]) for x in ev]))
        it = last["iters"].astype(np.float64)
        dec_ms = ms(2, 3)
        svc = (last["t_end"] - last["t_start"]).astype(np.float64) * 0.01  # 100 MHz device clock
        achieved = float(it.sum()) * B_it / (dec_ms * 1e-3) / 1e9
        return {
            "value": S * args.steps / wall, "unit": "shots/s", "ms_per_step": 1e3 * wall / args.steps,
            "wall_s": wall, "decode_kernel_ms": dec_ms, "sample_kernel_ms": ms(0, 1), "mlp_ms": ms(1, 2),
            "decode_only_shots_per_s": S / (dec_ms * 1e-3),
            "ler": stats.ler_summary(fails, S * args.steps, dem.rounds, dem.k),
            "mean_iters_per_shot": float(it.mean()), "mean_legs_per_shot": float(last["legs"].mean()),
            "path_counts": {str(k): int((last["path"] == k).sum()) for k in range(4)},
            "latency_us": {"batched_service_time": stats.percentiles(svc)},
            "roofline_decode": {"bound": "lds", "achieved": achieved, "peak": lds_gbs, "unit": "GB/s",
                                "frac": achieved / lds_gbs, "shot_iterations_per_launch": int(it.sum())},
        }

    P = timed("plain", params)
    launch = code.launch_config()
    kern = "relay_bp_compact_kernel" if launch["state"] == 3 else "relay_bp_kernel"
    traffic = load_traffic(args.workload, S)
    out = {
        "metric": METRIC, "value": P["value"], "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": P["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": f"12-round phenomenological DEM of the [[840,168]] ZSZ-LP code ({dem.M} detectors x "
                        f"{dem.N} mechanisms, nnz {dem.nnz}), priors 1e-3, {S} shots per step, Relay-BP "
                        f"gamma0=0.125 pre_iter=80 max_iterations=60 num_sets=100 stop_nconv=5 "
                        f"gamma_dist=[-0.24,0.66], FP32 messages" if args.workload == "phen840" else
                        f"{dem.name} ({dem.M} x {dem.N}, nnz {dem.nnz}), {S} shots per step",
            "shots_per_step": S, "total_timed_shots": S * args.steps,
            "path": "plain Relay-BP (value); first-solution Relay-BP, learned proposal and delta=0 control below",
        },
        "decode_only_shots_per_s": P["decode_only_shots_per_s"],
        "decode_kernel_ms": P["decode_kernel_ms"], "sample_kernel_ms": P["sample_kernel_ms"],
        "latency_us": P["latency_us"], "ler": P["ler"],
        "mean_iters_per_shot": P["mean_iters_per_shot"], "mean_legs_per_shot": P["mean_legs_per_shot"],
        "roofline": {"bound": "lds", "achieved": P["roofline_decode"]["achieved"], "peak": lds_gbs, "unit": "GB/s",
                     "frac": P["roofline_decode"]["frac"], "traffic": traffic, "kernel": kern,
                     "algorithmic_bytes_per_shot_iteration": B_it,
                     "shot_iterations_per_launch": P["roofline_decode"]["shot_iterations_per_launch"],
                     "peak_measured_GBps": lds_all, "peak_nominal_GBps": LDS_NOMINAL_GBS,
                     "note": "decode launch timed with HIP events on the decode stream (includes the ~20 us "
                             "heaviest-first ordering kernels before it)"},
        "launch": launch,
    }
    paths = {}
    fs = rbp.RelayParams(stop_nconv=1)
    if not args.no_first_solution:
        paths["first_solution"] = timed("plain", fs)
        paths["first_solution"]["note"] = "Relay-BP with stop_nconv = 1: the proposal path's stop rule, no proposal"

    progress("headline steps done")
    if not args.no_learned:
        from paper_2607_27644_amd import learned
        cfg = learned.TrainConfig(pairs=args.train_pairs, hidden=args.hidden, delta_scale=args.delta_scale)
        t0 = time.perf_counter()
        chunks = learned.generate_pairs(code, dem.priors, cfg, params)
        t1 = time.perf_counter()
        net = rbp.MLP(dem.M, cfg.hidden, dem.N, seed=cfg.seed)
        hist = learned.train(net, chunks, cfg)
        learned.scale_output(net, cfg.delta_scale)
        # the network writes its adjustments in the decoder's position order, which
        # the proposal leg copies to LDS with contiguous loads
        vord = code.positions()
        net.set_output_order(vord)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del chunks
        state["net"] = net
        state["delta"] = torch.empty((S, len(vord)), dtype=torch.bfloat16, device=dev)
        paths["learned"] = timed("learned", params)
        state["delta"].zero_()
        paths["proposal_zero"] = timed("proposal_zero", params)
        L = paths["learned"]
        flops = 2.0 * net.n_params * S
        L["roofline_mlp"] = {"bound": "mfma", "achieved": flops / (L["mlp_ms"] * 1e-3) / 1e12,
                             "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": flops / (L["mlp_ms"] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                             "algorithmic_flops_per_shot": 2.0 * net.n_params}
        L["training"] = {"pairs": cfg.pairs, "p_range": [cfg.p_lo, cfg.p_hi], "epochs": cfg.epochs,
                         "batch": cfg.batch, "hidden": cfg.hidden, "params": net.n_params,
                         "delta_scale": cfg.delta_scale, "generate_s": t1 - t0, "train_s": t2 - t1,
                         "final_loss": hist[-1][1]}
        L["vs_proposal_zero"] = L["value"] / paths["proposal_zero"]["value"]
        if "first_solution" in paths:
            L["vs_first_solution"] = L["value"] / paths["first_solution"]["value"]
        L["vs_plain"] = L["value"] / P["value"]
        paths["proposal_zero"]["note"] = "control: the same proposal leg with delta = 0 (no network)"
        L["note"] = ("network -> BF16 adjustments in the decoder's position order (rbp_mlp_forward_bf16 after "
                     "rbp_mlp_set_output_order) -> proposal leg with the adjustments in LDS, plain Relay-BP as the "
                     "fallback (rbp_decode_proposal_pos)")
    out.update(paths)

    # logical error rates at higher p, every path on the same syndromes
    out["ler_high_p"] = []
    for lp in [float(x) for x in args.ler_ps.split(",") if x]:
        pri = np.full(dem.N, lp)
        n = args.ler_shots
        hsyn, hobs, _ = code.sample(pri, n, args.seed + 777)
        res = {"p": lp, "shots": n}
        masks = {}
        runs = [("plain", params, None), ("first_solution", fs, None)]
        if state["net"] is not None:
            runs += [("learned", params, "net"), ("proposal_zero", params, "zero")]
        for name, prm, dk in runs:
            d = None
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            if dk == "net":
                d = state["net"].forward_bf16(hsyn)
            elif dk == "zero":
                d = torch.zeros((n, len(code.positions())), dtype=torch.bfloat16, device=dev)
            if d is not None:
                c, o, s = code.decode_proposal(pri, hsyn, prm, d, by_position=True)
            else:
                c, o, s = code.decode(pri, hsyn, prm)
            e1.record()
            torch.cuda.synchronize()
            sn = rbp.stats_to_numpy(s)
            f = stats.block_failures(rbp.to_u32(o), rbp.to_u32(hobs), sn["converged"])
            masks[name] = f
            res[name] = {"ler": stats.ler_summary(int(f.sum()), n, dem.rounds, dem.k),
                         "shots_per_s_network_and_decode": n / (e0.elapsed_time(e1) * 1e-3),
                         "mean_iters_per_shot": float(sn["iters"].mean()),
                         "non_converged": int((sn["converged"] == 0).sum())}
            del d, c, o, s
        for name in masks:
            if name != "plain":
                a, b = masks["plain"], masks[name]
                res[name]["paired_vs_plain"] = {"plain_only": int((a & ~b).sum()), "this_only": int((b & ~a).sum()),
                                                "both": int((a & b).sum())}
        out["ler_high_p"].append(res)

    progress("learned and paired-LER stages done")
    if not args.no_sequential:
        # the paper's sequential mode: one shot per decode call, host clock around
        # each; and the same shots through the resident decoder (one launch, the
        # syndrome handed over and the correction returned through pinned host
        # memory); the two alternate in blocks of 40 shots, so that they are
        # compared under the same conditions
        lat, rlat = np.zeros(200), np.zeros(200)
        c1, o1, s1 = corr[:1], obsp[:1], st[:1]
        hsyn = syn[:200].cpu().numpy().view(np.uint32)
        for b0 in range(0, 200, 40):
            for i in range(b0, b0 + 40):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                code.decode(dem.priors, syn[i:i + 1], params, out=(c1, o1, s1))
                torch.cuda.synchronize()
                lat[i] = 1e6 * (time.perf_counter() - ta)
            with code.resident(dem.priors, params, idle_seconds=10.0) as rd:
                rd.decode(hsyn[b0])
                for i in range(b0, b0 + 40):
                    ta = time.perf_counter()
                    rd.decode(hsyn[i])
                    rlat[i] = 1e6 * (time.perf_counter() - ta)
        out["latency_us"]["sequential_single_shot"] = stats.percentiles(lat)
        out["latency_us"]["resident_single_shot"] = stats.percentiles(rlat)

    progress("sequential latency done")
    if not args.no_extras:
        out["extras"] = extras(args.seed)

    progress("extras done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dem, args.seed, params, args.cpu_seconds)
    code.close()
    if state["net"] is not None:
        state["net"].close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def extras(seed: int) -> dict:
    """Secondary workloads: the earlier ZSZ-LP-160 headline, the batched uneven
    decode of four codes, the paper's latency-table workload and the classical
    AWGN benchmark."""
    import numpy as np
    import torch

    from paper_2607_27644_amd import autotune, circuits, experiments, rbp, stats, workloads
    res = {}
    # phenomenological ZSZ-LP-160 (576 x 1952), 10^5 shots per launch
    dem = workloads.workload("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, obs, _ = code.sample(dem.priors, 100000, seed)
    ms, out = experiments._timed(lambda: code.decode(dem.priors, syn, params))
    it = rbp.stats_to_numpy(out[2])["iters"].astype(np.float64).sum()
    res["phen160"] = {"decode_ms": ms, "decode_shots_per_s": 1e5 / (ms * 1e-3),
                      "algorithmic_GBps": it * (8 * dem.nnz + 8 * dem.N) / (ms * 1e-3) / 1e9,
                      "launch": code.launch_config()}
    code.close()
    # batched uneven decode: 4 codes (ZSZ-LP-160/320/550/775, 9 rounds), shots interleaved
    progress("extras: phen160 done")
    res["uneven_batch"] = experiments.multi(["phen160", "phen320", "phen550", "phen775"], 50000, seed=seed)
    progress("extras: uneven batch done")
    # the paper's latency-table workload: circuit-level ZSZ-LP-320 memory (1920 x 28992), p = 1e-3
    gmin, gmax = experiments.CIRCUIT_GAMMA["ZSZ-LP-320"]
    prm = rbp.RelayParams(num_sets=1000, gamma_min=gmin, gamma_max=gmax)
    cl = {"code": "ZSZ-LP-320", "p": 1e-3, "relay": {"num_sets": 1000, "gamma": [gmin, gmax]}}
    lat_all, res_all = [], []
    for basis in "XZ":
        d = circuits.memory_dem("ZSZ-LP-320", basis, 1e-3)
        c = rbp.Code.from_dem(d)
        s, _, _ = c.sample(d.priors, 4000, seed)
        o = c.decode_coop(d.priors, s[:1], prm)
        torch.cuda.synchronize()
        # per-call latency mode and the resident decoder on the same shots, in
        # alternating blocks of 20
        lat, rlat = [0.0] * 100, [0.0] * 100
        dev, rdev, xcds = [0.0] * 100, [0.0] * 100, []  # the kernel's own time per shot (device clock)
        hs = s[:100].cpu().numpy().view(np.uint32)
        for b0 in range(0, 100, 20):
            for i in range(b0, b0 + 20):
                t0 = time.perf_counter()
                c.decode_coop(d.priors, s[i:i + 1], prm, out=o)
                torch.cuda.synchronize()
                lat[i] = 1e6 * (time.perf_counter() - t0)
                so = rbp.stats_to_numpy(o[2])
                dev[i] = float(so["t_end"][0] - so["t_start"][0]) * 0.01
            with c.resident(d.priors, prm, idle_seconds=10.0) as rd:
                rd.decode(hs[b0])
                for i in range(b0, b0 + 20):
                    t0 = time.perf_counter()
                    _, _, sr = rd.decode(hs[i])
                    rlat[i] = 1e6 * (time.perf_counter() - t0)
                    rdev[i] = float(sr["t_end"] - sr["t_start"]) * 0.01
                xcds.append(rd.info()["xcds"])
        # batched: the launch shape tuned for this DEM (waves per shot, device-memory state)
        tr = autotune.tune(c, d.H, d.priors, prm, shots=2000, waves=(4, 8, 16), states=(2,), use_cache=False)
        ms, out = experiments._timed(lambda: c.decode(d.priors, s, prm), repeats=2)
        cl[f"{basis}_memory"] = {"dem": [d.M, d.N], "latency_mode_us": stats.percentiles(np.array(lat)),
                                 "resident_us": stats.percentiles(np.array(rlat)),
                                 "kernel_us_p50": {"latency_mode": float(np.median(dev)),
                                                   "resident": float(np.median(rdev))},
                                 "resident_xcd_masks": xcds,
                                 "batched_launch": {"waves_per_shot": tr["waves_per_shot"], "state": tr["state"]},
                                 "batched_shots_per_s": 4000 / (ms * 1e-3),
                                 "mean_iters": float(rbp.stats_to_numpy(out[2])["iters"].mean())}
        lat_all += lat
        res_all += rlat
        c.close()
    cl["latency_mode_us_xz"] = stats.percentiles(np.array(lat_all))
    cl["resident_us_xz"] = stats.percentiles(np.array(res_all))
    cl["paper_l40s_ms"] = {"mean": 1.2, "p99": 2.0, "p99.9": 3.2, "note": "NVIDIA L40S, Table 'decoding latency'"}
    res["circuit_latency"] = cl
    progress("extras: circuit latency done")
    # classical ZSZ-2BGA [310,155] code over BPSK-AWGN at 2.5 dB, sum-product BP
    r = experiments.awgn_fer(["ZSZ-2BGA-310"], [2.5], max_frames=2_000_000, min_errors=10 ** 12, chunk=1_000_000)
    pt = r["codes"]["ZSZ-2BGA-310"]["points"][0]
    res["awgn"] = {"code": "ZSZ-2BGA-310 [310,155]", "ebn0_db": pt["ebn0_db"], "frames": pt["frames"],
                   "fer": pt["fer"], "decode_frames_per_s": pt["decode_frames_per_s"]}
    return res


if __name__ == "__main__":
    main()
