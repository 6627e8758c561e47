"""What the trained proposal network gains over Relay-BP without it.

The network is trained on the GPU with the project's kernels on pairs the
decoder generates (phenomenological ZSZ-LP-160, priors in [5e-4, 2e-3]) and
used as a proposal for the first leg, plain Relay-BP being the fallback.  On
the same syndromes at p = 5e-3 it is compared with plain Relay-BP and with the
proposal leg run without a network (delta = 0).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import stats as ostats  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import learned, rbp
    return rbp, learned


def _run(rbp, code, priors, syn, obs, params, delta):
    corr, obsp, st = code.decode(priors, syn, params, delta=delta)
    s = rbp.stats_to_numpy(st)
    fails = ostats.block_failures(rbp.to_u32(obsp), rbp.to_u32(obs), s["converged"])
    return fails, s


def test_trained_proposal_gain_over_plain_and_untrained(mods):
    rbp, learned = mods
    dem = W.workload("phen160")
    params = rbp.RelayParams()
    code = rbp.Code.from_dem(dem)
    cfg = learned.TrainConfig()
    chunks = learned.generate_pairs(code, dem.priors, cfg, params)
    net = rbp.MLP(dem.M, cfg.hidden, dem.N, seed=cfg.seed)
    hist = learned.train(net, chunks, cfg)
    assert hist[-1][1] < 0.5 * learned_initial_loss(rbp, learned, dem, code, params, cfg)
    learned.scale_output(net, cfg.delta_scale)

    shots = 40000
    priors = np.full(dem.N, 5e-3)
    syn, obs, _ = code.sample(priors, shots, 2718)
    f_plain, s_plain = _run(rbp, code, priors, syn, obs, params, None)
    f_net, s_net = _run(rbp, code, priors, syn, obs, params, net.forward(syn))
    zero = torch.zeros((shots, dem.N), dtype=torch.float32, device="cuda")
    f_zero, s_zero = _run(rbp, code, priors, syn, obs, params, zero)

    it_plain, it_net, it_zero = (float(s["iters"].mean()) for s in (s_plain, s_net, s_zero))
    # the gain: far fewer BP iterations per shot than plain Relay-BP ...
    assert it_net < 0.3 * it_plain
    # ... and fewer than the proposal leg without a network
    assert it_net < it_zero
    # the proposal is accepted on most shots with a non-zero syndrome
    nonzero = s_net["path"] != 3
    assert np.mean(s_net["path"][nonzero] == 1) > 0.99
    # at no loss of logical error rate beyond a few paired disagreements
    learned_only = int((f_net & ~f_plain).sum())
    assert learned_only <= 3, (int(f_plain.sum()), int(f_net.sum()), learned_only)
    assert int(f_net.sum()) <= int(f_plain.sum()) + 3


def learned_initial_loss(rbp, learned, dem, code, params, cfg):
    """Loss of an untrained network on one training batch (same data recipe)."""
    small = learned.TrainConfig(pairs=cfg.batch, chunk=cfg.batch, seed=cfg.seed + 7)
    syn, corr, llr = learned.generate_pairs(code, dem.priors, small, params)[0]
    fresh = rbp.MLP(dem.M, cfg.hidden, dem.N, seed=cfg.seed)
    _, loss = fresh.gradients(syn, corr, llr)
    return float(loss.item())
