"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Sampling, syndromes and observables must be bit-exact; traced messages and
marginals must agree to 1e-5 relative (they are expected to be bitwise equal:
both sides evaluate the same single-precision operations in the same order);
corrections must be identical on at least 99.9 % of shots.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import stats as ostats  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402
from gf2 import gf2_product  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import rbp as mod
    return mod


_DEMS = {}


def dem_of(name):
    if name not in _DEMS:
        _DEMS[name] = W.workload(name)
    return _DEMS[name]


def oparams(p):
    return oracle.RelayParams(**{k: getattr(p, k) for k in oracle.RelayParams.__dataclass_fields__})


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def rel_close(a, b, rtol=1e-5, atol=1e-6):
    return np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)) + atol)


# ----------------------------------------------------------------- sampling
@pytest.mark.parametrize("name,shots", [("cc160", 10000), ("phen160", 20000), ("tiny60", 3001)])
def test_sample_bit_exact(rbp, name, shots):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    syn, obs, err = code.sample(dem.priors, shots, seed=987, errors=True)
    g = oracle.Graph(dem.H, dem.O)
    osyn, oobs, oerr = oracle.sample(g, dem.priors, shots, seed=987, want_errors=True)
    assert np.array_equal(u32(syn), osyn)
    assert np.array_equal(u32(obs)[:, : oobs.shape[1]], oobs)
    assert np.array_equal(u32(err), oerr)


def test_sample_offsets_and_ragged(rbp):
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    g = oracle.Graph(dem.H, dem.O)
    for off, n in [(0, 1), (5, 3), (123457, 1000), (2 ** 33 + 7, 65)]:
        syn, obs, _ = code.sample(dem.priors, n, seed=42, shot_offset=off)
        osyn, oobs, _ = oracle.sample(g, dem.priors, n, seed=42, shot_offset=off)
        assert np.array_equal(u32(syn), osyn), (off, n)
        assert np.array_equal(u32(obs), oobs), (off, n)


def test_sample_random_priors_bit_exact(rbp):
    dem = dem_of("cc160")
    pri = W.random_priors(dem.N, 1e-3, 0.5, seed=3)
    code = rbp.Code.from_dem(dem)
    syn, obs, err = code.sample(pri, 2000, seed=1, errors=True)
    osyn, oobs, oerr = oracle.sample(oracle.Graph(dem.H, dem.O), pri, 2000, seed=1, want_errors=True)
    assert np.array_equal(u32(err), oerr) and np.array_equal(u32(syn), osyn)


def test_sample_full_size_sampled_shots(rbp):
    """10^5 shots of the phenomenological ZSZ-LP-160 model in one launch; the
    oracle recomputes 400 shots spread over the range one by one."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    shots = 100000
    syn, obs, _ = code.sample(dem.priors, shots, seed=20260101)
    s_all, o_all = u32(syn), u32(obs)
    g = oracle.Graph(dem.H, dem.O)
    for i in np.linspace(0, shots - 1, 400).astype(int):
        osyn, oobs, _ = oracle.sample(g, dem.priors, 1, seed=20260101, shot_offset=int(i))
        assert np.array_equal(s_all[i], osyn[0]) and np.array_equal(o_all[i], oobs[0])


# ----------------------------------------------------------------- traces
@pytest.mark.parametrize("name", ["cc160", "phen160"])
def test_traced_messages_match(rbp, name):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    g = oracle.Graph(dem.H, dem.O)
    params = rbp.RelayParams(num_sets=6)
    osyn, _, _ = oracle.sample(g, dem.priors, 300, seed=77)
    nz = [s for s in range(300) if osyn[s].any()][:10]
    syn_dev = torch.from_numpy(osyn.view(np.int32)).cuda()
    checked = 0
    for s in nz:
        for leg, t in [(0, 1), (0, 2), (0, 5), (1, 1), (1, 2), (2, 3), (4, 1)]:
            ref = oracle.trace(g, dem.priors, osyn[s], oparams(params), leg=leg, t=t)
            got = code.trace(dem.priors, syn_dev[s].contiguous(), params, leg=leg, t=t)
            assert (ref is None) == (got is None), (s, leg, t)
            if ref is None:
                continue
            assert rel_close(got[0], ref[0]), (s, leg, t)
            assert rel_close(got[1], ref[1]), (s, leg, t)
            checked += 1
    assert checked >= 10


def test_traced_proposal_leg(rbp):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    g = oracle.Graph(dem.H, dem.O)
    params = rbp.RelayParams(num_sets=4)
    osyn, _, _ = oracle.sample(g, dem.priors, 50, seed=78)
    rng = np.random.default_rng(0)
    s = next(i for i in range(50) if osyn[i].any())
    d = rng.normal(0, 3, dem.N).astype(np.float32)
    syn_dev = torch.from_numpy(osyn[s:s + 1].view(np.int32)).cuda()
    d_dev = torch.from_numpy(d).cuda()
    for phase, leg, t in [(1, 0, 1), (1, 0, 2), (0, 0, 1), (0, 1, 2)]:
        ref = oracle.trace(g, dem.priors, osyn[s], oparams(params), leg=leg, t=t, phase=phase, delta=d)
        got = code.trace(dem.priors, syn_dev[0].contiguous(), params, leg=leg, t=t, phase=phase, delta=d_dev)
        assert (ref is None) == (got is None)
        if ref is not None:
            assert rel_close(got[0], ref[0]) and rel_close(got[1], ref[1])


# ----------------------------------------------------------------- decode parity
def _compare(rbp, dem, syn_np, out, ref, min_agree=0.999):
    corr, obsp, st = out
    stats = rbp.stats_to_numpy(st)
    c = u32(corr)
    same = (c == ref["corrections"]).all(axis=1)
    assert same.mean() >= min_agree, same.mean()
    o = u32(obsp)[:, : ref["obs_pred"].shape[1]]
    assert np.array_equal(o[same], ref["obs_pred"][same])
    for key in ("converged", "nconv", "path"):
        assert np.array_equal(stats[key][same], ref[key][same]), key
    assert np.array_equal(stats["legs"][same], ref["legs"][same])
    assert np.array_equal(stats["iters"][same], ref["iters"][same])
    # every converged GPU correction reproduces its syndrome
    e = W.unpack_bits(c, dem.N)
    conv = stats["converged"] == 1
    resyn = gf2_product(e, dem.H)
    assert np.array_equal(resyn[conv], W.unpack_bits(syn_np, dem.M)[conv])
    return same.mean()


@pytest.mark.parametrize("name,shots", [("cc160", 10000), ("phen160", 20000), ("tiny60", 2000)])
def test_decode_matches_oracle(rbp, name, shots):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, obs, _ = code.sample(dem.priors, shots, seed=31337)
    out = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    g = oracle.Graph(dem.H, dem.O)
    syn_np = u32(syn)
    ref = oracle.decode(g, dem.priors, syn_np, oparams(params), nthreads=16)
    _compare(rbp, dem, syn_np, out, ref)
    # logical error rates agree within their 95 % intervals
    stats = rbp.stats_to_numpy(out[2])
    obs_np = u32(obs)[:, : ref["obs_pred"].shape[1]]
    fg = ostats.block_failures(u32(out[1])[:, : obs_np.shape[1]], obs_np, stats["converged"]).sum()
    fo = ostats.block_failures(ref["obs_pred"], obs_np, ref["converged"]).sum()
    a, b = ostats.clopper_pearson(int(fg), shots), ostats.clopper_pearson(int(fo), shots)
    assert a[0] <= b[1] and b[0] <= a[1]


def test_gpu_failure_count_matches_host(rbp):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=3, pre_iter=3, max_iterations=3)
    pri = np.full(dem.N, 0.03)
    syn, obs, _ = code.sample(pri, 5000, seed=2)
    corr, obsp, st = code.decode(pri, syn, params)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    rbp.count_failures(obsp, obs, st, cnt)
    rbp.count_failures(obsp, obs, st, cnt)
    host = ostats.block_failures(u32(obsp), u32(obs), rbp.stats_to_numpy(st)["converged"]).sum()
    assert host > 0
    assert int(cnt.item()) == 2 * host


def test_decode_random_priors_and_dense_syndromes(rbp):
    """Non-uniform priors and random (mostly unsatisfiable-looking) syndromes
    exercise long legs, relay legs and non-convergence."""
    dem = dem_of("cc160")
    pri = W.random_priors(dem.N, 5e-3, 0.2, seed=8)
    code = rbp.Code.from_dem(dem)
    syn_np = W.random_syndromes(dem.M, 600, 0.08, seed=9)
    params = rbp.RelayParams(num_sets=15)
    syn = torch.from_numpy(syn_np.view(np.int32)).cuda()
    out = code.decode(pri, syn, params)
    torch.cuda.synchronize()
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), pri, syn_np, oparams(params), nthreads=16)
    _compare(rbp, dem, syn_np, out, ref)


def test_all_criterion_parity(rbp):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=10, stopping_criterion=1)
    syn, _, _ = code.sample(dem.priors, 500, seed=5)
    out = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    syn_np = u32(syn)
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn_np, oparams(params), nthreads=16)
    _compare(rbp, dem, syn_np, out, ref)
    stats = rbp.stats_to_numpy(out[2])
    assert (stats["legs"][stats["path"] != 3] == 11).all()


@pytest.mark.parametrize("kind", ["zero", "noise", "truth"])
def test_proposal_paths_match_oracle(rbp, kind):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=20)
    shots = 1500
    syn, obs, err = code.sample(dem.priors, shots, seed=6, errors=True)
    syn_np = u32(syn)
    e = W.unpack_bits(u32(err), dem.N)
    lam = np.log((1 - dem.priors) / dem.priors).astype(np.float32)
    if kind == "zero":
        d = np.zeros((shots, dem.N), np.float32)
    elif kind == "noise":
        d = np.random.default_rng(1).normal(0, 20, (shots, dem.N)).astype(np.float32)
    else:
        d = np.where(e == 1, -2 * lam - 10, 10).astype(np.float32)
    out = code.decode(dem.priors, syn, params, delta=torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn_np, oparams(params), delta=d, nthreads=16)
    _compare(rbp, dem, syn_np, out, ref)


# ----------------------------------------------------------------- launch-shape invariance (race detector)
def test_outputs_do_not_depend_on_launch_shape(rbp):
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=30)
    syn, _, _ = code.sample(dem.priors, 3000, seed=17)
    base = None
    for waves, state, slots in [(1, 1, 0), (2, 1, 0), (4, 1, 0), (8, 1, 0), (4, 2, 0), (16, 2, 0), (4, 1, 7),
                                (1, 2, 33)]:
        code.set_launch_config(waves, state, slots)
        corr, obsp, st = code.decode(dem.priors, syn, params)
        torch.cuda.synchronize()
        s = rbp.stats_to_numpy(st)
        cur = (u32(corr), u32(obsp), s["converged"], s["legs"], s["iters"])
        if base is None:
            base = cur
        else:
            for a, b in zip(base, cur):
                assert np.array_equal(a, b), (waves, state, slots)
    code.set_launch_config(0, 0, 0)


@pytest.mark.parametrize("shots,slots", [(20000, 0), (8193, 7)])
def test_heaviest_first_order_changes_no_output(rbp, shots, slots):
    """Batches of 8192 shots or more are decoded heaviest syndrome first; every
    output, statistics included (all but the two device timestamps, bytes 16 to
    31), must equal the decode of the same shots in chunks below that size
    (kept in their own order)."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, shots, seed=808)
    code.set_launch_config(0, 0, slots)
    corr, obsp, st = code.decode(dem.priors, syn, params)
    parts = [code.decode(dem.priors, syn[a:a + 4000].contiguous(), params) for a in range(0, shots, 4000)]
    torch.cuda.synchronize()
    code.set_launch_config(0, 0, 0)
    np.testing.assert_array_equal(u32(corr), np.concatenate([u32(p[0]) for p in parts]))
    np.testing.assert_array_equal(u32(obsp), np.concatenate([u32(p[1]) for p in parts]))
    np.testing.assert_array_equal(st.cpu().numpy()[:, :16], np.concatenate([p[2].cpu().numpy()[:, :16] for p in parts]))


# ----------------------------------------------------------------- edge cases
def test_edge_cases(rbp):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    # zero shots is a no-op
    syn = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    code.decode(dem.priors, syn, params)
    # all-zero syndromes: zero corrections, converged, path 3
    syn = torch.zeros((37, 2), dtype=torch.int32, device="cuda")
    corr, obsp, st = code.decode(dem.priors, syn, params)
    s = rbp.stats_to_numpy(st)
    assert not u32(corr).any() and not u32(obsp).any()
    assert (s["converged"] == 1).all() and (s["path"] == 3).all()
    # one shot, and a shot count that is not a multiple of anything
    for n in (1, 3, 257):
        syn, _, _ = code.sample(dem.priors, n, seed=n)
        corr, _, st = code.decode(dem.priors, syn, params)
        ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, u32(syn), oparams(params), nthreads=4)
        assert np.array_equal(u32(corr), ref["corrections"])
    # errors come back as exceptions with the library's message
    bad = dem.priors.copy()
    bad[3] = 0.7
    with pytest.raises(rbp.RbpError, match="UNSUPPORTED"):
        code.decode(bad, syn, params)
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        code.decode(dem.priors, syn, rbp.RelayParams(pre_iter=0))
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        code.decode(dem.priors, syn, rbp.RelayParams(stop_nconv=300))
    # the bounds under which saturated marginals keep every message finite
    for bad_params in (rbp.RelayParams(pre_iter=65537), rbp.RelayParams(max_iterations=70000),
                       rbp.RelayParams(gamma_max=16.5), rbp.RelayParams(gamma0=float("nan"))):
        with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
            code.decode(dem.priors, syn, bad_params)
    code.decode(dem.priors, syn, rbp.RelayParams(pre_iter=65536, num_sets=0))


def test_row_degree_32_kernel(rbp):
    """A model with a row of degree 20 takes the wide-row kernel."""
    rng = np.random.default_rng(4)
    H = (rng.random((12, 60)) < 0.15).astype(np.uint8)
    H[0, :20] = 1
    H[H.sum(1) == 1, 0] ^= 1
    H = H[H.sum(1) != 1]
    O = (rng.random((3, 60)) < 0.2).astype(np.uint8)
    pri = np.full(60, 0.03)
    code = rbp.Code(H, O)
    assert code.info()["max_row_deg"] > 12
    params = rbp.RelayParams(num_sets=10)
    syn, _, _ = code.sample(pri, 800, seed=3)
    out = code.decode(pri, syn, params)
    torch.cuda.synchronize()
    ref = oracle.decode(oracle.Graph(H, O), pri, u32(syn), oparams(params), nthreads=8)
    _compare(rbp, type("D", (), {"N": 60, "M": H.shape[0], "H": H})(), u32(syn), out, ref)


# ----------------------------------------------------------------- batched uneven decode
def test_multi_code_decode_matches_single(rbp):
    names = ["cc160", "tiny60", "phen160"]
    dems = [dem_of(n) for n in names] + [W.phenomenological_dem(W.seeded_hgp(16, 1016), 3, 2e-3)]
    codes = [rbp.Code.from_dem(d) for d in dems]
    params = rbp.RelayParams(num_sets=25)
    per = 700
    syns, singles = [], []
    for i, (d, c) in enumerate(zip(dems, codes)):
        syn, _, _ = c.sample(d.priors, per, seed=100 + i)
        syns.append(syn)
        singles.append(c.decode(d.priors, syn, params))
    torch.cuda.synchronize()
    n = len(dems)
    shot_code = torch.arange(n * per, device="cuda", dtype=torch.int64) % n
    shot_index = torch.arange(n * per, device="cuda", dtype=torch.int64) // n
    corrs = [torch.zeros_like(s[0]) for s in singles]
    obsps = [torch.zeros_like(s[1]) for s in singles]
    st = torch.zeros((n * per, 32), dtype=torch.uint8, device="cuda")
    rbp.decode_multi(codes, [d.priors for d in dems], shot_code.to(torch.uint8), shot_index.to(torch.int32), syns,
                     params, corrs, obsps, st)
    torch.cuda.synchronize()
    stats = rbp.stats_to_numpy(st)
    for i in range(n):
        assert np.array_equal(u32(corrs[i]), u32(singles[i][0])), names[i] if i < 3 else "hgp"
        assert np.array_equal(u32(obsps[i]), u32(singles[i][1]))
        s1 = rbp.stats_to_numpy(singles[i][2])
        assert np.array_equal(stats["iters"][i::n], s1["iters"])
    # and one model against the oracle
    ref = oracle.decode(oracle.Graph(dems[3].H, dems[3].O), dems[3].priors, u32(syns[3]), oparams(params),
                        nthreads=16)
    assert (u32(corrs[3]) == ref["corrections"]).all(axis=1).mean() >= 0.999


# ----------------------------------------------------------------- full-size launch, sampled check
def test_full_size_decode_sampled(rbp):
    """The benchmark workload (10^5 shots, phenomenological ZSZ-LP-160, default
    relay settings) in one launch; the oracle decodes 3000 shots spread over it."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams()
    shots = 100000
    syn, obs, _ = code.sample(dem.priors, shots, seed=20260101)
    corr, obsp, st = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    idx = np.linspace(0, shots - 1, 3000).astype(int)
    syn_np = u32(syn)[idx]
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn_np, oparams(params), nthreads=16)
    same = (u32(corr)[idx] == ref["corrections"]).all(axis=1)
    assert same.mean() >= 0.999
    s = rbp.stats_to_numpy(st)
    assert (s["converged"] == 1).mean() > 0.999


# ----------------------------------------------------------------- largest models, sampled check
@pytest.mark.parametrize("name,shots,checked,num_sets", [("phen840", 20000, 3000, 100), ("hgp56", 4000, 1000, 20)])
def test_largest_models_sampled(rbp, name, shots, checked, num_sets):
    """Full-size launches on the largest models with the per-slot state in
    device memory; the oracle decodes a spread sample of the same shots, and
    the corrections must be identical on >= 99.9 % of them.  (hgp56 uses 20
    relay legs: its non-converging shots would otherwise cost the CPU oracle
    about 17 s each.)"""
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, 2, 0)
    params = rbp.RelayParams(num_sets=num_sets)
    syn, obs, _ = code.sample(dem.priors, shots, seed=4242)
    corr, obsp, st = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    assert code.launch_config()["state"] == 2
    idx = np.linspace(0, shots - 1, checked).astype(int)
    syn_np = u32(syn)[idx]
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn_np, oparams(params), nthreads=16)
    same = (u32(corr)[idx] == ref["corrections"]).all(axis=1)
    assert same.mean() >= 0.999, same.mean()
    s = rbp.stats_to_numpy(st)
    assert np.array_equal(s["iters"][idx][same], ref["iters"][same])
    # converged corrections reproduce their syndromes (checked on the sample)
    e = W.unpack_bits(u32(corr)[idx], dem.N)
    conv = s["converged"][idx] == 1
    resyn = gf2_product(e, dem.H)
    assert np.array_equal(resyn[conv], W.unpack_bits(syn_np, dem.M)[conv])
