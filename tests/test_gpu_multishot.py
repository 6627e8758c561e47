"""Several shots per workgroup (the multi-shot compact kernel): K = 2 or 4
shots decoded in lockstep by one workgroup, sharing every group's table loads.
Each shot's arithmetic is that of the one-shot compact kernel, so every output
and statistic (all but the two device timestamps) must be identical to it,
for every model, batch size, prior set and stop criterion; the oracle checks a
sample directly."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402
from gf2 import gf2_product  # noqa: E402

pytestmark = pytest.mark.gpu

COMPACT = 3
_DEMS = {}


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


def _same(a, b):
    assert torch.equal(a[0], b[0])
    assert torch.equal(a[1], b[1])
    assert torch.equal(a[2][:, :16], b[2][:, :16])  # bytes 16..31: device timestamps


def _both(rbp, code, priors, syn, params, k, waves=0):
    code.set_launch_config(waves, COMPACT, 0, 1)
    one = code.decode(priors, syn, params)
    code.set_launch_config(waves, COMPACT, 0, k)
    assert code.launch_config()["shots_per_wg"] == k
    many = code.decode(priors, syn, params)
    torch.cuda.synchronize()
    code.set_launch_config(0, 0, 0, 0)
    return one, many


@pytest.mark.parametrize("k", [2, 4])
@pytest.mark.parametrize("name,shots", [("phen160", 20000), ("cc160", 10000), ("tiny60", 3001), ("phen320", 5000)])
def test_multishot_equals_one_shot(rbp, name, shots, k):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    syn, _, _ = code.sample(dem.priors, shots, seed=77)
    one, many = _both(rbp, code, dem.priors, syn, rbp.RelayParams(), k)
    _same(one, many)


@pytest.mark.parametrize("k", [2, 4])
def test_multishot_launch_shapes(rbp, k):
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    syn, _, _ = code.sample(dem.priors, 9000, seed=5)
    params = rbp.RelayParams()
    code.set_launch_config(0, COMPACT, 0, 1)
    ref = code.decode(dem.priors, syn, params)
    for waves, slots in [(4, 0), (8, 0), (16, 0), (8, 7), (2, 1)]:
        code.set_launch_config(waves, COMPACT, slots, k)
        out = code.decode(dem.priors, syn, params)
        torch.cuda.synchronize()
        _same(ref, out)
    code.set_launch_config(0, 0, 0, 0)


@pytest.mark.parametrize("k", [2, 4])
def test_multishot_random_priors_dense_syndromes_all_criterion(rbp, k):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    rng = np.random.default_rng(3)
    priors = rng.uniform(0.002, 0.06, dem.N)
    syn, _, _ = code.sample(priors, 4000, seed=8)
    for params in (rbp.RelayParams(num_sets=30, gamma_min=-0.3, gamma_max=0.8), rbp.RelayParams(
            num_sets=6, stopping_criterion=1)):
        one, many = _both(rbp, code, priors, syn, params, k)
        _same(one, many)


@pytest.mark.parametrize("k", [2, 4])
def test_multishot_small_and_zero_batches(rbp, k):
    """Fewer shots than sub-slots, a batch of zero syndromes, and zero
    syndromes mixed into a batch."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    for n in (1, 3, 5, 257):
        syn, _, _ = code.sample(dem.priors, n, seed=n)
        one, many = _both(rbp, code, dem.priors, syn, params, k)
        _same(one, many)
    zero = torch.zeros((41, rbp.words(dem.M)), dtype=torch.int32, device="cuda")
    one, many = _both(rbp, code, dem.priors, zero, params, k)
    _same(one, many)
    st = rbp.stats_to_numpy(many[2])
    assert (st["path"] == 3).all() and not u32(many[0]).any()
    syn, _, _ = code.sample(dem.priors, 2000, seed=9)
    syn[::3] = 0
    one, many = _both(rbp, code, dem.priors, syn, params, k)
    _same(one, many)


def test_multishot_against_oracle(rbp):
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, 3000, seed=31)
    code.set_launch_config(0, COMPACT, 0, 4)
    corr, obsp, st = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    code.set_launch_config(0, 0, 0, 0)
    op = oracle.RelayParams(**{f: getattr(params, f) for f in oracle.RelayParams.__dataclass_fields__})
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, u32(syn), op, nthreads=16)
    same = (u32(corr) == ref["corrections"]).all(axis=1)
    assert same.mean() >= 0.999
    s = rbp.stats_to_numpy(st)
    for key in ("converged", "nconv", "path", "legs", "iters"):
        assert np.array_equal(s[key][same], ref[key][same]), key
    conv = s["converged"] == 1
    e = W.unpack_bits(u32(corr), dem.N)
    assert np.array_equal(gf2_product(e, dem.H)[conv], W.unpack_bits(u32(syn), dem.M)[conv])


def test_multishot_limits(rbp):
    """Shots that do not fit in LDS together are refused; the setting is
    ignored where it does not apply (a proposal decode); bad values are
    rejected."""
    dem = dem_of("phen840")
    code = rbp.Code.from_dem(dem)
    syn, _, _ = code.sample(dem.priors, 10, seed=1)
    code.set_launch_config(0, COMPACT, 0, 2)
    with pytest.raises(rbp.RbpError, match="UNSUPPORTED"):
        code.decode(dem.priors, syn, rbp.RelayParams())
    small = dem_of("phen160")
    c2 = rbp.Code.from_dem(small)
    syn2, _, _ = c2.sample(small.priors, 500, seed=2)
    d16 = torch.zeros((500, small.N), dtype=torch.bfloat16, device="cuda")
    c2.set_launch_config(0, COMPACT, 0, 1)
    ref = c2.decode_proposal(small.priors, syn2, rbp.RelayParams(), d16)
    c2.set_launch_config(0, COMPACT, 0, 4)
    out = c2.decode_proposal(small.priors, syn2, rbp.RelayParams(), d16)
    torch.cuda.synchronize()
    _same(ref, out)
    for bad in (3, 8, -1):
        with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
            c2.set_launch_config(0, COMPACT, 0, bad)


def test_multishot_allocation_free_entry_point(rbp):
    """rbp_decode_noalloc takes the multi-shot kernel too (its shot counter and
    ordering scratch are the fixed device array): equal to rbp_decode."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, 12000, seed=44)
    code.set_launch_config(0, COMPACT, 0, 4)
    ref = code.decode(dem.priors, syn, params)
    out = code.decode_noalloc(dem.priors, syn, params,
                              out=(torch.empty_like(ref[0]), torch.empty_like(ref[1]), torch.empty_like(ref[2])))
    torch.cuda.synchronize()
    code.set_launch_config(0, 0, 0, 0)
    _same(ref, out)
