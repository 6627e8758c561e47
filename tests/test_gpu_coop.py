"""Latency mode (rbp_decode_coop): one shot at a time, its sweeps spread over
several workgroups with grid barriers between them.

Its arithmetic is the persistent decoder's, group by group, so every output
and statistic (bar the two device timestamps, bytes 16 to 31 of a record) must
equal rbp_decode's, which is parity-tested against the oracle; the oracle is
also checked directly on a sample.  A barrier whose arrivals never complete
(host-forced phantom participants, tiny poll bound) must stop the launch and
be reported, and the next launch must run normally.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

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


def same_outputs(a, b):
    np.testing.assert_array_equal(u32(a[0]), u32(b[0]))
    np.testing.assert_array_equal(u32(a[1]), u32(b[1]))
    np.testing.assert_array_equal(a[2].cpu().numpy()[:, :16], b[2].cpu().numpy()[:, :16])


@pytest.mark.parametrize("name,shots", [("tiny60", 100), ("phen160", 200), ("circ160x", 120), ("circ160z", 120)])
def test_coop_equals_batched(rbp, name, shots):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, shots, seed=71)
    ref = code.decode(dem.priors, syn, params)
    got = code.decode_coop(dem.priors, syn, params)
    torch.cuda.synchronize()
    assert not code.coop_aborted()
    same_outputs(got, ref)


@pytest.mark.parametrize("wg,stride,waves,dev", [(32, 8, 8, 0), (32, 8, 8, 1), (64, 1, 8, 0), (7, 3, 8, 0),
                                                 (16, 16, 4, 0), (1, 1, 4, 0), (256, 1, 2, 0)])
def test_coop_launch_shapes(rbp, wg, stride, waves, dev):
    dem = dem_of("circ160x")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=20)
    syn, _, _ = code.sample(dem.priors, 40, seed=72)
    ref = code.decode(dem.priors, syn, params)
    got = code.decode_coop(dem.priors, syn, params,
                           rbp.CoopParams(workgroups=wg, stride=stride, waves=waves, device_fences=dev))
    torch.cuda.synchronize()
    assert not code.coop_aborted()
    same_outputs(got, ref)


def test_coop_all_criterion_and_zero_syndrome(rbp):
    dem = dem_of("circ160x")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=5, stopping_criterion=1)
    syn, _, _ = code.sample(dem.priors, 12, seed=73)
    syn[3] = 0
    ref = code.decode(dem.priors, syn, params)
    got = code.decode_coop(dem.priors, syn, params)
    torch.cuda.synchronize()
    same_outputs(got, ref)
    s = rbp.stats_to_numpy(got[2])
    assert s["path"][3] == 3 and s["legs"][3] == 0
    assert (s["legs"][s["path"] != 3] == 6).all()


def test_coop_matches_oracle(rbp):
    dem = dem_of("circ160z")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, 48, seed=74)
    corr, obsp, st = code.decode_coop(dem.priors, syn, params)
    torch.cuda.synchronize()
    op = oracle.RelayParams(**{k: getattr(params, k) for k in oracle.RelayParams.__dataclass_fields__})
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, u32(syn), op, nthreads=16)
    np.testing.assert_array_equal(u32(corr), ref["corrections"])
    s = rbp.stats_to_numpy(st)
    np.testing.assert_array_equal(s["iters"], ref["iters"])
    np.testing.assert_array_equal(s["converged"], ref["converged"])


def test_coop_expired_barrier_is_reported(rbp):
    """A barrier forced to expire from the host (the test hook adds a phantom
    participant that never arrives; tiny poll bound) stops the launch, which
    returns ABORTED; the next launch runs normally."""
    dem = dem_of("tiny60")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, 4, seed=75)
    code.set_coop_phantom(1)
    with pytest.raises(rbp.RbpError, match="ABORTED") as ex:
        code.decode_coop(dem.priors, syn, params, rbp.CoopParams(workgroups=4, stride=1, spin_limit=2000))
    assert ex.value.status == rbp.RBP_ERR_ABORTED
    assert code.coop_aborted()
    code.set_coop_phantom(0)
    ref = code.decode(dem.priors, syn, params)
    got = code.decode_coop(dem.priors, syn, params)
    torch.cuda.synchronize()
    assert not code.coop_aborted()
    same_outputs(got, ref)
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        code.decode_coop(dem.priors, syn, params, rbp.CoopParams(waves=9))
