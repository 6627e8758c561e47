"""Resident decoder (rbp_resident_*): the latency-mode kernel launched once and
fed one shot at a time through a mailbox in pinned host memory.

It runs the latency mode's arithmetic, so every output and statistic (bar the
two device timestamps, bytes 16 to 31 of a record) must equal rbp_decode_coop's
on the same syndromes, which equals rbp_decode's and the oracle's; the oracle
is also checked directly.  References are computed before a resident kernel
starts and compared after it stops: while it runs, a device-wide
synchronization would wait for it.  The kernel's own ends (no shot for
idle_seconds, an expired barrier forced from the host) must be reported and
recovered from by the next decode.
"""
import time

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


def reference(rbp, code, dem, shots, seed, params, coop=None, priors=None):
    priors = dem.priors if priors is None else priors
    syn, _, _ = code.sample(priors, shots, seed=seed)
    corr, obsp, st = code.decode_coop(priors, syn, params, coop)
    torch.cuda.synchronize()
    return u32(syn), (u32(corr), u32(obsp), st.cpu().numpy())


def run_resident(res, syn):
    out = [res.decode(syn[i]) for i in range(syn.shape[0])]
    corr = np.stack([o[0] for o in out])
    obs = np.stack([o[1] for o in out])
    st = np.stack([o[2] for o in out]).view(np.uint8).reshape(len(out), 32)
    return corr, obs, st


def same(got, ref):
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1][:, : got[1].shape[1]])
    np.testing.assert_array_equal(got[2][:, :16], ref[2][:, :16])


@pytest.mark.parametrize("name,shots,wg", [("tiny60", 60, 1), ("phen160", 150, 1), ("phen160", 150, 0),
                                           ("circ160x", 60, 0), ("circ160z", 60, 4)])
def test_resident_equals_latency_mode(rbp, name, shots, wg):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    coop = rbp.CoopParams(workgroups=wg)
    syn, ref = reference(rbp, code, dem, shots, 91, params, coop)
    with code.resident(dem.priors, params, coop, idle_seconds=5.0) as res:
        got = run_resident(res, syn)
        info = res.info()
    assert info["shots"] == shots and info["launches"] == 1
    assert bin(info["xcds"]).count("1") == 1  # the default stride keeps the participants on one XCD
    same(got, ref)


def test_resident_matches_oracle(rbp):
    dem = dem_of("circ160z")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, 40, seed=92)
    syn = u32(syn)
    with code.resident(dem.priors, params, idle_seconds=5.0) as res:
        corr, _, st = run_resident(res, syn)
    op = oracle.RelayParams(**{k: getattr(params, k) for k in oracle.RelayParams.__dataclass_fields__})
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn, op, nthreads=16)
    np.testing.assert_array_equal(corr, ref["corrections"])
    s = st.reshape(-1).view(rbp.SHOT_STATS_DTYPE)
    np.testing.assert_array_equal(s["iters"], ref["iters"])
    np.testing.assert_array_equal(s["converged"], ref["converged"])
    np.testing.assert_array_equal(s["legs"], ref["legs"])


def test_resident_zero_syndromes_and_all_criterion(rbp):
    dem = dem_of("circ160x")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=5, stopping_criterion=1)
    syn, _, _ = code.sample(dem.priors, 10, seed=93)
    syn[2] = 0
    syn[7] = 0
    ref_t = code.decode_coop(dem.priors, syn, params)
    torch.cuda.synchronize()
    ref = (u32(ref_t[0]), u32(ref_t[1]), ref_t[2].cpu().numpy())
    with code.resident(dem.priors, params, idle_seconds=5.0) as res:
        got = run_resident(res, u32(syn))
    same(got, ref)
    s = got[2].reshape(-1).view(rbp.SHOT_STATS_DTYPE)
    assert s["path"][2] == 3 and s["path"][7] == 3 and not got[0][[2, 7]].any()


def test_resident_idle_end_and_relaunch(rbp):
    """The kernel ends itself after idle_seconds without a shot; the next decode
    launches it again and resumes the shot count; results are unchanged."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    coop = rbp.CoopParams(workgroups=1)
    syn, ref = reference(rbp, code, dem, 9, 94, params, coop)
    with code.resident(dem.priors, params, coop, idle_seconds=0.2) as res:
        first = run_resident(res, syn[:4])
        time.sleep(0.8)
        assert not res.info()["running"]
        second = run_resident(res, syn[4:])
        info = res.info()
    assert info["launches"] == 2 and info["shots"] == 9
    same(tuple(np.concatenate([a, b]) for a, b in zip(first, second)), ref)


def test_resident_expired_barrier_is_reported(rbp):
    """A barrier forced to expire from the host (a phantom participant that
    never arrives, tiny poll bound) ends the kernel: decode returns ABORTED;
    without the phantom a new resident decoder runs normally."""
    dem = dem_of("tiny60")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    coop = rbp.CoopParams(workgroups=4, stride=1, spin_limit=2000)
    syn, ref = reference(rbp, code, dem, 5, 95, params, coop)
    code.set_coop_phantom(1)
    res = code.resident(dem.priors, params, coop, idle_seconds=5.0)
    with pytest.raises(rbp.RbpError, match="ABORTED") as ex:
        res.decode(syn[0])
    assert ex.value.status == rbp.RBP_ERR_ABORTED
    assert not res.info()["running"]
    res.close()
    code.set_coop_phantom(0)
    with code.resident(dem.priors, params, coop, idle_seconds=5.0) as res:
        got = run_resident(res, syn)
    same(got, ref)


def test_resident_guards(rbp):
    """Arguments are checked; while a resident decoder runs, the code's priors
    and relay parameters cannot change and the code cannot be destroyed."""
    dem = dem_of("tiny60")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, ref = reference(rbp, code, dem, 3, 96, params)
    other = np.asarray(dem.priors, dtype=np.float64) * 0.5
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        code.resident(dem.priors, params, rbp.CoopParams(waves=9))
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        code.resident(dem.priors, params, idle_seconds=-1.0)
    res = code.resident(dem.priors, params, idle_seconds=5.0)
    try:
        with pytest.raises(ValueError):
            res.decode(np.zeros(syn.shape[1] + 1, np.uint32))
        with pytest.raises(ValueError):
            res.decode(torch.zeros(syn.shape[1], dtype=torch.int32, device="cuda"))
        with pytest.raises(TypeError):
            res.decode(syn[0].astype(np.float32))
        d_syn = torch.from_numpy(syn.view(np.int32)).cuda()
        with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
            code.decode_coop(other, d_syn, params)
        with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
            code.decode_coop(dem.priors, d_syn, rbp.RelayParams(gamma_min=-0.3))
        assert rbp.lib().rbp_code_destroy(code.h) == rbp.RBP_ERR_INVALID_ARG
        got = run_resident(res, syn)
    finally:
        res.close()
    same(got, ref)
    # stopped: the code takes other priors again
    corr, _, _ = code.decode_coop(other, torch.from_numpy(syn.view(np.int32)).cuda(), params)
    torch.cuda.synchronize()
    assert corr.shape == (3, (dem.N + 31) // 32)
