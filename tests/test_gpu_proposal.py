"""The BF16 proposal path: the network's BF16 output is the round-to-nearest-
even of its FP32 output, and rbp_decode_proposal with BF16 adjustments equals
rbp_decode with the same adjustments widened to float, bit for bit, for every
decoder state (per-edge in LDS, compact, device memory); the oracle decodes the
widened adjustments to the same corrections."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import rbp as mod
    return mod


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def oparams(p):
    return oracle.RelayParams(**{k: getattr(p, k) for k in oracle.RelayParams.__dataclass_fields__})


def test_bf16_forward_is_the_rounded_fp32_forward(rbp):
    dem = W.workload("phen160")
    net = rbp.MLP(dem.M, 128, dem.N, seed=3)
    p = net.get_params()
    p[-dem.N:] = np.random.default_rng(0).normal(0, 0.5, dem.N).astype(np.float32)  # non-zero output bias
    net.set_params(p)
    code = rbp.Code.from_dem(dem)
    syn, _, _ = code.sample(np.full(dem.N, 5e-3), 140000, seed=1)  # more than one 131072-row forward chunk
    f32 = net.forward(syn)
    b16 = net.forward_bf16(syn)
    assert torch.equal(b16, f32.to(torch.bfloat16))


@pytest.mark.parametrize("name,state", [("phen160", 1), ("phen160", 3), ("phen840", 3), ("phen840", 2),
                                        ("cc160", 3)])
def test_proposal_bf16_equals_widened_fp32(rbp, name, state):
    dem = W.workload(name)
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, state, 0)
    params = rbp.RelayParams(num_sets=20)
    shots = 4000 if dem.N > 5000 else 10000
    syn, _, _ = code.sample(dem.priors, shots, seed=9)
    rng = np.random.default_rng(2)
    # small adjustments on even shots (their proposal legs converge), large ones on
    # odd shots (their proposal legs fail and fall back to plain Relay-BP)
    sd = np.where(np.arange(shots) % 2 == 0, 1.0, 12.0)[:, None]
    d16 = torch.from_numpy((rng.normal(0, 1.0, (shots, dem.N)) * sd).astype(np.float32)).cuda().to(torch.bfloat16)
    a = code.decode_proposal(dem.priors, syn, params, d16)
    b = code.decode(dem.priors, syn, params, delta=d16.float().contiguous())
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(a[2][:, :16], b[2][:, :16])
    st = rbp.stats_to_numpy(a[2])
    assert (st["path"] == 1).any() and (st["path"] == 2).any()  # both outcomes of the proposal leg occur


def test_proposal_bf16_against_oracle(rbp):
    dem = W.workload("cc160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=20)
    shots = 1500
    syn, _, _ = code.sample(dem.priors, shots, seed=6)
    rng = np.random.default_rng(1)
    d16 = torch.from_numpy(rng.normal(0, 4, (shots, dem.N)).astype(np.float32)).cuda().to(torch.bfloat16)
    corr, obsp, st = code.decode_proposal(dem.priors, syn, params, d16)
    torch.cuda.synchronize()
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, u32(syn), oparams(params),
                        delta=d16.float().cpu().numpy(), nthreads=16)
    same = (u32(corr) == ref["corrections"]).all(axis=1)
    assert same.mean() >= 0.999
    s = rbp.stats_to_numpy(st)
    for key in ("converged", "nconv", "path", "legs", "iters"):
        assert np.array_equal(s[key][same], ref[key][same]), key


def by_position(d16, vord):
    """[shots][N] adjustments by mechanism -> [shots][Np] by decoder position
    (padding 0), the plain gather"""
    out = torch.zeros((d16.shape[0], len(vord)), dtype=torch.bfloat16, device=d16.device)
    live = np.flatnonzero(vord >= 0)
    idx = torch.from_numpy(vord[live].astype(np.int64)).cuda()
    out[:, torch.from_numpy(live).cuda()] = d16[:, idx]
    return out


@pytest.mark.parametrize("name,state", [("phen160", 1), ("phen160", 3), ("phen840", 3), ("phen840", 2),
                                        ("cc160", 3)])
def test_proposal_by_position_equals_by_mechanism(rbp, name, state):
    """rbp_decode_proposal_pos on the adjustments gathered into position order
    gives the same outputs as rbp_decode_proposal, bit for bit, in every state."""
    dem = W.workload(name)
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, state, 0)
    params = rbp.RelayParams(num_sets=20)
    shots = 4000 if dem.N > 5000 else 10000
    syn, _, _ = code.sample(dem.priors, shots, seed=19)
    rng = np.random.default_rng(4)
    sd = np.where(np.arange(shots) % 2 == 0, 1.0, 12.0)[:, None]
    d16 = torch.from_numpy((rng.normal(0, 1.0, (shots, dem.N)) * sd).astype(np.float32)).cuda().to(torch.bfloat16)
    vord = code.positions()
    assert sorted(vord[vord >= 0].tolist()) == list(range(dem.N)) and (vord[dem.N:] == -1).all()
    dpos = by_position(d16, vord)
    dpos[:, dem.N:] = 7.0  # padding entries are ignored
    a = code.decode_proposal(dem.priors, syn, params, d16)
    b = code.decode_proposal(dem.priors, syn, params, dpos, by_position=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(a[2][:, :16], b[2][:, :16])
    path = rbp.stats_to_numpy(b[2])["path"]
    assert (path == 1).any() and (path == 2).any()


def test_network_output_in_position_order(rbp):
    """MLP.set_output_order: the BF16 forward writes the output columns in the
    given order (zeros at -1), equal to the gathered natural output, also after
    the weights change (a training step, set_params); None restores the order."""
    dem = W.workload("phen160")
    code = rbp.Code.from_dem(dem)
    vord = code.positions()
    net = rbp.MLP(dem.M, 128, dem.N, seed=5)
    p = net.get_params()
    p[-dem.N:] = np.random.default_rng(1).normal(0, 0.5, dem.N).astype(np.float32)
    net.set_params(p)
    syn, _, err = code.sample(np.full(dem.N, 5e-3), 3000, seed=2, errors=True)
    nat = net.forward_bf16(syn)
    net.set_output_order(vord)
    pos = net.forward_bf16(syn)
    torch.cuda.synchronize()
    assert pos.shape == (3000, len(vord))
    assert torch.equal(pos, by_position(nat, vord))
    llr = code.llr(np.full(dem.N, 5e-3))
    net.train_step(syn[:1024], err[:1024], llr, lr=1e-3)
    net.set_output_order(None)
    nat2 = net.forward_bf16(syn)
    net.set_output_order(vord)
    pos2 = net.forward_bf16(syn)
    torch.cuda.synchronize()
    assert not torch.equal(nat2, nat)
    assert torch.equal(pos2, by_position(nat2, vord))
    # a training step with the order set keeps the ordered copy current
    net.train_step(syn[:1024], err[:1024], llr, lr=1e-3)
    pos3 = net.forward_bf16(syn)
    net.set_output_order(None)
    nat3 = net.forward_bf16(syn)
    torch.cuda.synchronize()
    assert torch.equal(pos3, by_position(nat3, vord))
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        net.set_output_order(np.array([0, dem.N], dtype=np.int32))
