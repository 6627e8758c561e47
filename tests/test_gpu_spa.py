"""GPU parity of the classical channel-coding path (BPSK-AWGN sampling and
sum-product BP of the ZSZ-2BGA codes) against the CPU oracle.

Tolerances follow from the arithmetic.  Both sides evaluate the same single-
precision operations in the same order except phi = -ln tanh(x/2): the oracle
calls the C library's log1pf(2 / expm1f(x)), the kernel a formulation from the
hardware exp2 / log2 / reciprocal with two short series, within 2e-6 relative
for the |nu| <= 20 it sees.  Hence: channel LLRs (single vs double precision)
agree to 1e-5 (1 + |llr|); marginals after one iteration to 1e-5 relative;
after five iterations to 2e-3 relative (the differences are propagated, not
created); one iteration on a single check matches the float64 tanh rule
2 atanh(prod tanh(L/2)) to 1e-5.  In
full decodes, shots that never reach a codeword iterate chaotically for all
max_iterations and their final hard decision depends on the last ulp: moving
the oracle's own inputs by one ulp changes about 0.4 % of such words at 3 dB
on the [64,32] code, always on non-converged shots.  So the decoded words must
agree on at least 99.9 % of the shots both sides decode to a codeword, and the
convergence flags and block-error indicators on at least 99.9 % of all shots.
The launch shape changes nothing (bitwise).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402
from gf2 import gf2_product  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import rbp as mod
    return mod


def code_of(rbp, H):
    return rbp.Code(H, np.zeros((0, H.shape[1]), dtype=np.uint8))


def bits_of(rbp, t, N):
    w = t.cpu().numpy().view(np.uint32)
    b = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")
    return b[:, :N]


def mixed_code():
    """Random code with ragged row and column degrees: rows of degree 0, 2..20
    (so padded row groups, rows above 12 edges and a partial last group),
    columns of degree 1..4."""
    rng = np.random.default_rng(77)
    M, N = 70, 150
    H = np.zeros((M, N), dtype=np.uint8)
    for j in range(N):
        H[rng.choice(M - 1, size=int(rng.integers(1, 5)), replace=False), j] = 1
    # rows need degree 0 or >= 2: top up the rows with a single edge
    for i in range(M - 1):
        if H[i].sum() == 1:
            H[i, rng.choice(np.flatnonzero(H[i] == 0))] = 1
    # a few heavy rows
    for i in (3, 11):
        H[i, rng.choice(N, size=18, replace=False)] = 1
    return H  # row M-1 stays empty


@pytest.mark.parametrize("name,shots,sigma", [("ZSZ-2BGA-64", 3000, 0.8), ("ZSZ-2BGA-310", 2001, 1.1)])
def test_awgn_sampler_matches_oracle(rbp, name, shots, sigma):
    H = W.zsz_2bga(name)
    code = code_of(rbp, H)
    llr = code.sample_awgn(shots, sigma, seed=123).cpu().numpy()
    ref = oracle.awgn(H.shape[1], shots, sigma, 123)
    assert np.all(np.abs(llr - ref) <= 1e-5 * (1.0 + np.abs(ref)))
    part = code.sample_awgn(10, sigma, seed=123, shot_offset=shots - 10).cpu().numpy()
    np.testing.assert_array_equal(part, llr[-10:])


def rel_ok(a, b, rtol, atol):
    return np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)) + atol


@pytest.mark.parametrize("T,rtol", [(1, 1e-5), (5, 2e-3)])
@pytest.mark.parametrize("which", ["ZSZ-2BGA-64", "ZSZ-2BGA-310", "mixed"])
def test_marginals_match_oracle(rbp, which, T, rtol):
    H = mixed_code() if which == "mixed" else W.zsz_2bga(which)
    N = H.shape[1]
    code = code_of(rbp, H)
    L = W.awgn_llrs(N, 513, W.awgn_sigma(1.5, 0.5), seed=31)
    P = rbp.SpaParams(max_iterations=T, stop=False)
    bits, marg, st = code.decode_spa(torch.from_numpy(L).cuda(), P, marginals=True)
    ref = oracle.spa_decode(H, L, max_iterations=T, stop=False, marginals=True, nthreads=8)
    m = marg.cpu().numpy()
    ok = rel_ok(m, ref["marginals"], rtol, rtol)
    assert ok.mean() == 1.0, (which, T, float(ok.mean()), float(np.abs(m - ref["marginals"]).max()))
    s = rbp.stats_to_numpy(st)
    assert (s["iters"] == T).all()


@pytest.mark.parametrize("name,ebn0", [("ZSZ-2BGA-64", 1.5), ("ZSZ-2BGA-64", 3.0), ("ZSZ-2BGA-310", 1.5),
                                       ("ZSZ-2BGA-310", 2.5)])
def test_full_decode_matches_oracle(rbp, name, ebn0):
    H = W.zsz_2bga(name)
    N = H.shape[1]
    code = code_of(rbp, H)
    shots = 4001
    L = W.awgn_llrs(N, shots, W.awgn_sigma(ebn0, 0.5), seed=int(ebn0 * 10) + N)
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    bits, _, st = code.decode_spa(torch.from_numpy(L).cuda(), rbp.SpaParams(), counts=counts)
    ref = oracle.spa_decode(H, L, max_iterations=100, nthreads=8)
    b = bits_of(rbp, bits, N)
    s = rbp.stats_to_numpy(st)
    both = (s["converged"] == 1) & (ref["converged"] == 1)
    same = (b[both] == ref["bits"][both]).all(axis=1)
    assert same.mean() >= 0.999, same.mean()
    assert (s["iters"][both] == ref["iters"][both]).mean() >= 0.999
    assert (s["converged"] == ref["converged"]).mean() >= 0.999
    assert (b.any(axis=1) == ref["bits"].any(axis=1)).mean() >= 0.999
    # converged outputs are codewords
    conv = s["converged"] == 1
    assert not gf2_product(b[conv], H).any()
    # the in-kernel counts are the host's reading of the outputs
    nz = b.any(axis=1)
    c = counts.cpu().numpy()
    assert c[0] == nz.sum() and c[1] == (nz & conv).sum() and c[2] == (~conv).sum()
    assert (s["path"] == nz).all()


@pytest.mark.parametrize("D", [2, 3, 6, 11])
def test_single_check_against_tanh_rule(rbp, D):
    """phi as the kernel evaluates it, through one check update: magnitudes
    from 1e-6 to the clip value, both signs."""
    rng = np.random.default_rng(40 + D)
    H = np.ones((1, D), dtype=np.uint8)
    mag = np.exp(rng.uniform(np.log(1e-6), np.log(20.0), size=(2000, D)))
    L = (mag * rng.choice([-1.0, 1.0], size=mag.shape)).astype(np.float32)
    code = code_of(rbp, H)
    _, marg, _ = code.decode_spa(torch.from_numpy(L).cuda(), rbp.SpaParams(max_iterations=1, stop=False),
                                 marginals=True)
    Ld = L.astype(np.float64)
    th = np.tanh(Ld / 2.0)
    ref = np.stack([Ld[:, j] + 2.0 * np.arctanh(np.clip(np.prod(np.delete(th, j, axis=1), axis=1), -1 + 1e-16,
                                                        1 - 1e-16)) for j in range(D)], axis=1)
    assert rel_ok(marg.cpu().numpy(), ref, 1e-5, 1e-5).all()


def test_launch_shape_and_edge_cases(rbp):
    H = W.zsz_2bga("ZSZ-2BGA-156")
    N = H.shape[1]
    code = code_of(rbp, H)
    L = torch.from_numpy(W.awgn_llrs(N, 777, W.awgn_sigma(1.0, 0.5), seed=8)).cuda()
    outs = []
    for waves in (1, 2, 3, 4, 8):
        bits, marg, _ = code.decode_spa(L, rbp.SpaParams(waves_per_shot=waves), marginals=True)
        outs.append((bits.cpu().numpy(), marg.cpu().numpy()))
    for b, m in outs[1:]:
        np.testing.assert_array_equal(b, outs[0][0])
        np.testing.assert_array_equal(m, outs[0][1])
    # one shot, and zero shots (a no-op)
    b1, _, _ = code.decode_spa(L[:1].contiguous(), rbp.SpaParams())
    np.testing.assert_array_equal(b1.cpu().numpy(), outs[0][0][:1])
    code.decode_spa(L[:0].contiguous(), rbp.SpaParams())
    # clipping: LLRs beyond llr_max act as +-llr_max
    big = torch.sign(L) * 1e6
    bb, mb, _ = code.decode_spa(big.contiguous(), rbp.SpaParams(max_iterations=1, stop=False), marginals=True)
    ref = oracle.spa_decode(H, big.cpu().numpy(), max_iterations=1, stop=False, marginals=True, nthreads=8)
    assert rel_ok(mb.cpu().numpy(), ref["marginals"], 1e-5, 1e-5).all()
    # invalid parameters are rejected on the host
    with pytest.raises(rbp.RbpError):
        code.decode_spa(L, rbp.SpaParams(max_iterations=0))
    with pytest.raises(rbp.RbpError):
        code.decode_spa(L, rbp.SpaParams(llr_max=-1.0))


def test_fer_experiment_chunking(rbp):
    """The frame stream is one seeded stream: chunking does not change it, and
    the frame error rate falls with E_b/N_0."""
    from paper_2607_27644_amd import experiments as E
    a = E.awgn_fer(["ZSZ-2BGA-64"], [1.0, 3.0], max_frames=20000, min_errors=10 ** 9, chunk=7000)
    b = E.awgn_fer(["ZSZ-2BGA-64"], [1.0, 3.0], max_frames=20000, min_errors=10 ** 9, chunk=20000)
    pa, pb = a["codes"]["ZSZ-2BGA-64"]["points"], b["codes"]["ZSZ-2BGA-64"]["points"]
    for x, y in zip(pa, pb):
        assert x["frames"] == y["frames"] == 20000
        for key in ("block_errors", "undetected", "nonconverged", "mean_iters"):
            assert x[key] == y[key], key
    assert pa[0]["fer"] > 3 * pa[1]["fer"] > 0
    assert abs(a["shannon_limit_db"] - 0.187) < 0.002
