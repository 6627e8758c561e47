"""Learned proposal for Relay-BP: data generation, training and evaluation.

The proposal network maps a syndrome to per-mechanism log-prior adjustments
delta; the decoder runs one proposal leg with priors Lambda + delta and falls
back to plain Relay-BP when that leg does not converge (rbp_decode with
prior_delta).  Training pairs (syndrome, Relay-BP correction) come from the
path itself: shots are sampled at a prior p drawn per chunk from [p_lo, p_hi]
and decoded with plain Relay-BP; the loss is binary cross-entropy of the
correction bits against sigmoid(-(Lambda + delta)).  After training the
proposal is shrunk (delta_scale) before it is used.  Everything runs on the GPU
through librbp; this module only orchestrates the calls.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Tuple

import numpy as np
import torch

from . import rbp, stats


@dataclasses.dataclass
class TrainConfig:
    pairs: int = 1_000_000
    chunk: int = 50_000
    p_lo: float = 5e-4
    p_hi: float = 2e-3
    hidden: int = 512
    batch: int = 4096
    epochs: int = 3
    lr: float = 1e-3
    seed: int = 1234
    # Proposal shrinkage: delta is scaled by this factor by scaling the output
    # layer once after training (exact in BF16 for a power of two).  The raw
    # network is confident enough to drive the proposal leg to wrong but
    # syndrome-consistent solutions at p >= 5e-3; 1/8 keeps the logical error
    # rate of plain Relay-BP at 5e-3 and 1e-2 on the phenomenological
    # ZSZ-LP-160 model.
    delta_scale: float = 0.125


def generate_pairs(code: rbp.Code, base_priors: np.ndarray, cfg: TrainConfig, params: rbp.RelayParams):
    """Chunks of (syndromes, corrections, llr) with one prior scale per chunk.

    base_priors are scaled so that their mean equals the chunk's p (uniform
    priors stay uniform)."""
    rng = np.random.default_rng(cfg.seed)
    out: List[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = []
    made = 0
    k = 0
    while made < cfg.pairs:
        n = min(cfg.chunk, cfg.pairs - made)
        p = rng.uniform(cfg.p_lo, cfg.p_hi)
        pri = np.clip(base_priors * (p / float(np.mean(base_priors))), 1e-9, 0.5)
        syn, _, _ = code.sample(pri, n, seed=cfg.seed * 1000 + k)
        corr, _, _ = code.decode(pri, syn, params, stats=False)
        out.append((syn, corr, code.llr(pri)))
        made += n
        k += 1
    torch.cuda.synchronize()
    return out


def scale_output(net: rbp.MLP, factor: float):
    """delta -> factor * delta: scales the last layer's weights and bias."""
    if factor == 1.0:
        return
    p = net.get_params()
    o3 = net.hidden * net.in_dim + net.hidden + net.hidden * net.hidden + net.hidden
    p[o3:] *= np.float32(factor)
    net.set_params(p)


def train(net: rbp.MLP, chunks, cfg: TrainConfig, log_every: int = 0):
    """Adam over shuffled batches drawn inside each chunk (one LLR vector per batch)."""
    rng = np.random.default_rng(cfg.seed + 1)
    loss = torch.zeros(1, device="cuda")
    history = []
    step = 0
    for ep in range(cfg.epochs):
        order = rng.permutation(len(chunks))
        for ci in order:
            syn, corr, llr = chunks[ci]
            n = syn.shape[0]
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            for b0 in range(0, n - cfg.batch + 1, cfg.batch):
                idx = perm[b0:b0 + cfg.batch]
                net.train_step(syn.index_select(0, idx).contiguous(), corr.index_select(0, idx).contiguous(), llr,
                               cfg.lr, loss_out=loss)
                step += 1
                if log_every and step % log_every == 0:
                    history.append((step, float(loss.item())))
        history.append((step, float(loss.item())))
    return history


def evaluate(code: rbp.Code, net: rbp.MLP, priors: np.ndarray, shots: int, seed: int, params: rbp.RelayParams,
             rounds: int, k: int, repeats: int = 3) -> dict:
    """Plain Relay-BP against proposal + fallback on the same syndromes."""
    syn, obs, _ = code.sample(priors, shots, seed)
    torch.cuda.synchronize()
    res = {}
    zero = torch.zeros((shots, code.N), dtype=torch.float32, device="cuda")
    for name in ("plain", "learned", "proposal_zero"):
        times, mlp_times = [], []
        for _ in range(repeats):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            delta = net.forward(syn) if name == "learned" else (zero if name == "proposal_zero" else None)
            e1.record()
            corr, obsp, st = code.decode(priors, syn, params, delta=delta)
            e2.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e2))
            mlp_times.append(e0.elapsed_time(e1))
        s = rbp.stats_to_numpy(st)
        o = rbp.to_u32(obs)
        op = rbp.to_u32(obsp)
        fails = stats.block_failures(op, o, s["converged"])
        ms = float(np.median(times))
        res[name] = {
            "shots_per_s": shots / (ms * 1e-3), "ms": ms, "mlp_ms": float(np.median(mlp_times)),
            "ler": stats.ler_summary(int(fails.sum()), shots, rounds, k),
            "mean_iters": float(s["iters"].mean()), "mean_legs": float(s["legs"].mean()),
            "path_counts": {int(p): int((s["path"] == p).sum()) for p in range(4)},
            "service_us": stats.percentiles((s["t_end"] - s["t_start"]).astype(np.float64) * 0.01),
            "fails_mask": fails,
        }
    a, b = res["plain"]["fails_mask"], res["learned"]["fails_mask"]
    res["paired"] = {"plain_only": int((a & ~b).sum()), "learned_only": int((b & ~a).sum()),
                     "both": int((a & b).sum())}
    for name in ("plain", "learned", "proposal_zero"):
        del res[name]["fails_mask"]
    return res


def train_and_evaluate(dem, cfg: TrainConfig, eval_priors: np.ndarray, eval_shots: int, eval_seed: int,
                       params: rbp.RelayParams | None = None) -> dict:
    params = params or rbp.RelayParams()
    code = rbp.Code.from_dem(dem)
    t0 = time.perf_counter()
    chunks = generate_pairs(code, dem.priors, cfg, params)
    t1 = time.perf_counter()
    net = rbp.MLP(dem.M, cfg.hidden, dem.N, seed=cfg.seed)
    hist = train(net, chunks, cfg)
    scale_output(net, cfg.delta_scale)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if isinstance(eval_priors, dict):
        ev = {key: evaluate(code, net, pr, eval_shots, eval_seed, params, dem.rounds, dem.k)
              for key, pr in eval_priors.items()}
    else:
        ev = evaluate(code, net, eval_priors, eval_shots, eval_seed, params, dem.rounds, dem.k)
    ev["train"] = {"pairs": cfg.pairs, "gen_s": t1 - t0, "train_s": t2 - t1, "final_loss": hist[-1][1],
                   "steps": hist[-1][0], "params": net.n_params}
    return ev
