"""Several models, each in its own launch with its own launch shape, issued
together on side streams (rbp_decode_each).

Every model's outputs and statistics (bar the two device timestamps, bytes 16
to 31 of a record) must equal a plain rbp_decode of that model with the same
launch shape, which is parity-tested against the oracle; the oracle is also
checked directly on a sample.  The launches run concurrently, so this also
checks that nothing is shared between handles.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

_DEMS = {}
# (waves per shot, state): compact LDS, per-edge LDS, compact with 16 waves, device memory
SHAPES = {"phen160": (8, 3), "phen320": (8, 1), "phen550": (16, 3), "phen775": (16, 2)}


@pytest.fixture(scope="module")
def rbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import rbp as mod
    return mod


def dem_of(name):
    if name not in _DEMS:
        _DEMS[name] = W.workload(name)
    return _DEMS[name]


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def setup(rbp, names, shots, seed):
    dems = [dem_of(n) for n in names]
    codes = [rbp.Code.from_dem(d) for d in dems]
    syns = []
    for i, (n, d, c) in enumerate(zip(names, dems, codes)):
        c.set_launch_config(*SHAPES[n], 0)
        syns.append(c.sample(d.priors, shots[i], seed=seed + i)[0])
    return dems, codes, syns


def same(a, b):
    assert torch.equal(a[0], b[0])
    assert torch.equal(a[1], b[1])
    assert torch.equal(a[2][:, :16], b[2][:, :16])


def test_each_equals_single_model_decodes(rbp):
    names = list(SHAPES)
    dems, codes, syns = setup(rbp, names, [6000, 5000, 3000, 2500], 41)
    params = rbp.RelayParams()
    refs = [c.decode(d.priors, s, params) for d, c, s in zip(dems, codes, syns)]
    torch.cuda.synchronize()
    for _ in range(2):
        got = rbp.decode_each(codes, [d.priors for d in dems], syns, params)
        torch.cuda.synchronize()
        for g, r in zip(got, refs):
            same(g, r)


def test_each_on_a_side_stream_and_with_empty_models(rbp):
    names = ["phen160", "phen550"]
    dems, codes, syns = setup(rbp, names, [3000, 0], 42)
    params = rbp.RelayParams(num_sets=30, gamma_min=-0.3, gamma_max=0.8)
    ref = codes[0].decode(dems[0].priors, syns[0], params)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = rbp.decode_each(codes, [d.priors for d in dems], syns, params, stream=s)
    s.synchronize()
    same(got[0], ref)
    assert got[1][0].shape[0] == 0


def test_each_against_oracle(rbp):
    names = ["phen160", "phen320"]
    dems, codes, syns = setup(rbp, names, [400, 300], 43)
    params = rbp.RelayParams()
    got = rbp.decode_each(codes, [d.priors for d in dems], syns, params)
    torch.cuda.synchronize()
    op = oracle.RelayParams(**{f: getattr(params, f) for f in oracle.RelayParams.__dataclass_fields__})
    for d, s, g in zip(dems, syns, got):
        ref = oracle.decode(oracle.Graph(d.H, d.O), d.priors, u32(s), op, nthreads=16)
        same_rows = (u32(g[0]) == ref["corrections"]).all(axis=1)
        assert same_rows.mean() >= 0.995
        st = rbp.stats_to_numpy(g[2])
        for key in ("converged", "nconv", "legs", "iters"):
            assert np.array_equal(st[key][same_rows], ref[key][same_rows]), key


def test_each_rejects_bad_arguments(rbp):
    names = ["phen160", "phen320"]
    dems, codes, syns = setup(rbp, names, [10, 10], 44)
    params = rbp.RelayParams()
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        rbp.decode_each([codes[0], codes[0]], [dems[0].priors] * 2, [syns[0], syns[0]], params)
    with pytest.raises(rbp.RbpError, match="UNSUPPORTED"):
        rbp.decode_each(codes, [dems[0].priors, np.full(dems[1].N, 0.7)], syns, params)
    with pytest.raises(ValueError):
        rbp.decode_each(codes, [dems[0].priors], syns, params)
