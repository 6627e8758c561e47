"""GPU parity of the compact decoder state (one 16-byte record per check row
instead of one float per edge; the state of the 12-round [[840,168]] model
then fits in LDS) against the CPU oracle and against the per-edge state.

The compact form stores the two least |nu| of each row, the edge attaining the
least and the outgoing signs, and forms nu = M - mu from the marginals; every
message and marginal is the same FP32 value as in the per-edge form, so traces
are compared to 1e-5 relative (bitwise equal in practice) and decodes must give
identical corrections on at least 99.9 % of shots.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402
from gf2 import gf2_product  # noqa: E402

pytestmark = pytest.mark.gpu

COMPACT = 3


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


def _compare(rbp, dem, syn_np, out, ref, min_agree=0.999):
    corr, obsp, st = out
    stats = rbp.stats_to_numpy(st)
    c = u32(corr)
    same = (c == ref["corrections"]).all(axis=1)
    assert same.mean() >= min_agree, same.mean()
    o = u32(obsp)[:, : ref["obs_pred"].shape[1]]
    assert np.array_equal(o[same], ref["obs_pred"][same])
    for key in ("converged", "nconv", "path", "legs", "iters"):
        assert np.array_equal(stats[key][same], ref[key][same]), key
    e = W.unpack_bits(c, dem.N)
    conv = stats["converged"] == 1
    resyn = gf2_product(e, dem.H)
    assert np.array_equal(resyn[conv], W.unpack_bits(syn_np, dem.M)[conv])
    return same.mean()


def test_compact_is_chosen_where_the_edge_state_does_not_fit(rbp):
    assert rbp.Code.from_dem(dem_of("phen840")).launch_config()["state"] == COMPACT
    assert rbp.Code.from_dem(dem_of("phen160")).launch_config()["state"] == 1
    # rows over 16 edges cannot take it
    assert rbp.Code.from_dem(dem_of("hgp56")).launch_config()["state"] == 2


@pytest.mark.parametrize("name", ["cc160", "phen160", "phen840"])
def test_compact_traces_match_oracle(rbp, name):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, COMPACT, 0)
    g = oracle.Graph(dem.H, dem.O)
    params = rbp.RelayParams(num_sets=6)
    osyn, _, _ = oracle.sample(g, dem.priors, 300, seed=77)
    nz = [s for s in range(300) if osyn[s].any()][:8]
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
    assert checked >= 8


def test_compact_traced_proposal_leg(rbp):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, COMPACT, 0)
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


@pytest.mark.parametrize("name,shots", [("cc160", 10000), ("phen160", 20000), ("tiny60", 2000)])
def test_compact_decode_matches_oracle(rbp, name, shots):
    dem = dem_of(name)
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, COMPACT, 0)
    params = rbp.RelayParams()
    syn, _, _ = code.sample(dem.priors, shots, seed=31337)
    out = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    syn_np = u32(syn)
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn_np, oparams(params), nthreads=16)
    _compare(rbp, dem, syn_np, out, ref)


def test_compact_random_priors_dense_syndromes_and_all_criterion(rbp):
    dem = dem_of("cc160")
    pri = W.random_priors(dem.N, 5e-3, 0.2, seed=8)
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, COMPACT, 0)
    syn_np = W.random_syndromes(dem.M, 600, 0.08, seed=9)
    syn = torch.from_numpy(syn_np.view(np.int32)).cuda()
    g = oracle.Graph(dem.H, dem.O)
    for params in (rbp.RelayParams(num_sets=15), rbp.RelayParams(num_sets=10, stopping_criterion=1)):
        out = code.decode(pri, syn, params)
        torch.cuda.synchronize()
        ref = oracle.decode(g, pri, syn_np, oparams(params), nthreads=16)
        _compare(rbp, dem, syn_np, out, ref)


@pytest.mark.parametrize("kind", ["zero", "noise", "truth"])
def test_compact_proposal_paths_match_oracle(rbp, kind):
    dem = dem_of("cc160")
    code = rbp.Code.from_dem(dem)
    code.set_launch_config(0, COMPACT, 0)
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


def test_compact_equals_per_edge_state_for_every_launch_shape(rbp):
    """Race check: the compact decode of the same shots equals the per-edge
    decode bit for bit (outputs and statistics) for several launch shapes."""
    dem = dem_of("phen160")
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=30)
    syn, _, _ = code.sample(dem.priors, 3000, seed=17)
    code.set_launch_config(0, 1, 0)
    corr, obsp, st = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    s0 = rbp.stats_to_numpy(st)
    base = (u32(corr), u32(obsp), s0["converged"], s0["nconv"], s0["path"], s0["legs"], s0["iters"])
    for waves, slots in [(1, 0), (2, 0), (4, 0), (8, 0), (16, 0), (4, 7), (2, 33)]:
        code.set_launch_config(waves, COMPACT, slots)
        corr, obsp, st = code.decode(dem.priors, syn, params)
        torch.cuda.synchronize()
        s = rbp.stats_to_numpy(st)
        cur = (u32(corr), u32(obsp), s["converged"], s["nconv"], s["path"], s["legs"], s["iters"])
        for a, b in zip(base, cur):
            assert np.array_equal(a, b), (waves, slots)


def test_compact_zero_and_tied_magnitudes(rbp):
    """Priors of exactly 0.5 (Lambda = +0) on about 2 % of the mechanisms and
    one shared prior on the rest: the check sweep meets |nu| = 0, messages of
    either zero sign and exact ties between the two least magnitudes, where
    the row minima must still select the same bits as an unsigned minimum.
    The compact decode of the 12-round [[840,168]] model equals the per-edge
    decode (device-memory state) bit for bit, and the oracle on a spread
    sample of 200 shots."""
    dem = dem_of("phen840")
    rng = np.random.default_rng(23)
    pri = np.full(dem.N, 2e-3)
    pri[rng.random(dem.N) < 0.02] = 0.5
    code = rbp.Code.from_dem(dem)
    params = rbp.RelayParams(num_sets=10)
    syn, _, _ = code.sample(pri, 2000, seed=29)
    outs = []
    for state in (COMPACT, 2):
        code.set_launch_config(0, state, 0)
        corr, obsp, st = code.decode(pri, syn, params)
        torch.cuda.synchronize()
        assert code.launch_config()["state"] == state
        s = rbp.stats_to_numpy(st)
        outs.append((u32(corr), u32(obsp), s["converged"], s["nconv"], s["path"], s["legs"], s["iters"]))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    idx = np.linspace(0, 1999, 200).astype(int)
    syn_np = u32(syn)[idx]
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), pri, syn_np, oparams(params), nthreads=16)
    assert np.array_equal(outs[0][0][idx], ref["corrections"])
    for key, got in zip(("converged", "nconv", "path", "legs", "iters"), outs[0][2:]):
        assert np.array_equal(got[idx], ref[key]), key


def test_compact_wide_and_mixed_rows(rbp):
    """Rows of 13 to 16 edges (stored as 16, padding read from the +inf cell),
    mixed row and variable groups, and a mechanism in no check."""
    rng = np.random.default_rng(5)
    H = (rng.random((40, 150)) < 0.06).astype(np.uint8)
    for r in range(H.shape[0]):  # at most 12 random edges per row
        H[r, np.flatnonzero(H[r])[12:]] = 0
    H[0] = 0
    H[0, :16] = 1
    H[1] = 0
    H[1, 20:34] = 1
    H[:, 149] = 0
    H[H.sum(1) == 1, 0] ^= 1
    H = H[H.sum(1) != 1]
    O = (rng.random((4, 150)) < 0.1).astype(np.uint8)
    pri = W.random_priors(150, 0.01, 0.08, seed=2)
    code = rbp.Code(H, O)
    assert code.info()["max_row_deg"] == 16
    code.set_launch_config(0, COMPACT, 0)
    params = rbp.RelayParams(num_sets=12)
    syn, _, _ = code.sample(pri, 1500, seed=3)
    out = code.decode(pri, syn, params)
    torch.cuda.synchronize()
    ref = oracle.decode(oracle.Graph(H, O), pri, u32(syn), oparams(params), nthreads=8)
    _compare(rbp, type("D", (), {"N": 150, "M": H.shape[0], "H": H})(), u32(syn), out, ref)


def test_phen840_full_size_against_oracle(rbp):
    """The 12-round [[840,168]] model (4032 x 13776), 10^5 shots in one launch on
    the compact state; the oracle decodes 3,000 shots spread over the batch:
    identical corrections on >= 99.9 % and identical statistics there."""
    dem = dem_of("phen840")
    code = rbp.Code.from_dem(dem)
    assert code.launch_config()["state"] == COMPACT
    params = rbp.RelayParams()
    shots = 100000
    syn, obs, _ = code.sample(dem.priors, shots, seed=4242)
    corr, obsp, st = code.decode(dem.priors, syn, params)
    torch.cuda.synchronize()
    idx = np.linspace(0, shots - 1, 3000).astype(int)
    syn_np = u32(syn)[idx]
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn_np, oparams(params), nthreads=16)
    sub = (corr[idx], obsp[idx], st[idx])
    assert _compare(rbp, dem, syn_np, sub, ref) >= 0.999


def test_compact_multi_model_launch(rbp):
    """One compact launch over the four phenomenological candidates
    (ZSZ-LP-160/320/550/775, 9 rounds) equals the single-model decodes, and
    1000 shots of every model (one in four) decode as the oracle does on at
    least 99.9% of them."""
    names = ["phen160", "phen320", "phen550", "phen775"]
    dems = [dem_of(n) for n in names]
    codes = [rbp.Code.from_dem(d) for d in dems]
    for c in codes:
        c.set_launch_config(0, COMPACT, 0)
    params = rbp.RelayParams()
    per = 4000
    syns, singles = [], []
    for i, (d, c) in enumerate(zip(dems, codes)):
        syn, _, _ = c.sample(d.priors, per, seed=300 + i)
        syns.append(syn)
        singles.append(c.decode(d.priors, syn, params))
    torch.cuda.synchronize()
    n = len(dems)
    shot_code = (torch.arange(n * per, device="cuda") % n).to(torch.uint8)
    shot_index = (torch.arange(n * per, device="cuda") // n).to(torch.int32)
    corrs = [torch.zeros_like(s[0]) for s in singles]
    obsps = [torch.zeros_like(s[1]) for s in singles]
    st = torch.zeros((n * per, 32), dtype=torch.uint8, device="cuda")
    rbp.decode_multi(codes, [d.priors for d in dems], shot_code, shot_index, syns, params, corrs, obsps, st)
    torch.cuda.synchronize()
    stats = rbp.stats_to_numpy(st)
    for i in range(n):
        assert np.array_equal(u32(corrs[i]), u32(singles[i][0])), names[i]
        assert np.array_equal(u32(obsps[i]), u32(singles[i][1])), names[i]
        assert np.array_equal(stats["iters"][i::n], rbp.stats_to_numpy(singles[i][2])["iters"])
        idx = np.arange(0, per, 4)
        ref = oracle.decode(oracle.Graph(dems[i].H, dems[i].O), dems[i].priors, u32(syns[i])[idx], oparams(params),
                            nthreads=16)
        assert (u32(corrs[i])[idx] == ref["corrections"]).all(axis=1).mean() >= 0.999, names[i]
