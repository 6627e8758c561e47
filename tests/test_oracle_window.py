"""Pins of the sliding-window oracle.

* one window covering every round is the global decode, bit for bit;
* the commit masks partition the mechanisms: each column with a detector is
  committed by exactly one window;
* every window of a phenomenological model has rows of degree 0 or >= 2 (the
  decoder's requirement), and its syndrome rows are the model's rows;
* a converged shot leaves no residual syndrome and its correction reproduces
  the syndrome (H e = sigma).
"""
import numpy as np
import pytest

import oracle
from oracle import window as owin
from paper_2607_27644_amd import workloads as W


@pytest.fixture(scope="module")
def model():
    dem = W.phenomenological_dem(W.zsz_lp("ZSZ-LP-60"), 7, 0.02)
    m = dem.M // dem.rounds
    g = oracle.Graph(dem.H, dem.O)
    syn, obs, _ = oracle.sample(g, dem.priors, 300, seed=17)
    return dem, m, syn, obs


def test_single_window_is_the_global_decode(model):
    dem, m, syn, _ = model
    p = oracle.RelayParams(num_sets=20)
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn, p, nthreads=4)
    for w in (dem.rounds, dem.rounds + 3):
        r = owin.decode_windowed(dem.H, dem.O, dem.priors, syn, m, w, 1, p, nthreads=4)
        np.testing.assert_array_equal(r["corrections"], ref["corrections"])
        np.testing.assert_array_equal(r["obs_pred"][:, : ref["obs_pred"].shape[1]], ref["obs_pred"])
        np.testing.assert_array_equal(r["converged"], ref["converged"])


@pytest.mark.parametrize("w,c", [(3, 1), (3, 2), (4, 4), (2, 1)])
def test_windows_partition_and_rows(model, w, c):
    dem, m, _, _ = model
    H = dem.H
    ws = owin.windows(H, m, w, c)
    count = np.zeros(dem.N, dtype=int)
    for s, r, cols, cm in ws:
        count[cols[cm]] += 1
        Hw = H[s * m:(s + r) * m][:, cols]
        deg = Hw.sum(axis=1)
        assert not (deg == 1).any()
        # columns start inside the window
        first = np.array([np.flatnonzero(H[:, j])[0] for j in cols])
        assert ((first >= s * m) & (first < (s + r) * m)).all()
    nonempty = H.any(axis=0)
    assert (count[nonempty] == 1).all() and (count[~nonempty] == 0).all()
    assert ws[-1][0] + ws[-1][1] == dem.rounds


@pytest.mark.parametrize("w,c", [(3, 1), (4, 2)])
def test_converged_shots_explain_the_syndrome(model, w, c):
    dem, m, syn, obs = model
    p = oracle.RelayParams(num_sets=20)
    r = owin.decode_windowed(dem.H, dem.O, dem.priors, syn, m, w, c, p, nthreads=4)
    conv = r["converged"] == 1
    assert conv.mean() > 0.9
    assert not r["residual"][conv].any()
    e = owin._unpack(r["corrections"], dem.N)
    s = (e.astype(np.int64) @ dem.H.T.astype(np.int64)) % 2
    np.testing.assert_array_equal(owin._pack(s.astype(np.uint8))[conv], syn[conv])
    o = (e.astype(np.int64) @ dem.O.T.astype(np.int64)) % 2
    np.testing.assert_array_equal(owin._pack(o.astype(np.uint8)), r["obs_pred"])


# ---------------------------------------------------------------- parallel windows
@pytest.mark.parametrize("core,buffer,gap", [(3, 2, 2), (2, 1, 1), (4, 3, 2)])
def test_parallel_windows_commit_every_column_once(model, core, buffer, gap):
    dem, m, _, _ = model
    A, B = owin.parallel_windows(dem.H, m, core, buffer, gap)
    count = np.zeros(dem.N, dtype=int)
    for rows, cols, cm in A:
        count[cols[cm]] += 1
    for rows, cols, cm, fixed in B:
        count[cols[cm]] += 1
        for i, j in fixed:
            count[j] += 1
            # a fixing row meets exactly one of the gap's columns
            gap_cols = np.concatenate([cols, [f[1] for f in fixed]]).astype(int)
            assert dem.H[i, gap_cols].sum() == 1
    assert (count[dem.H.any(axis=0)] == 1).all()
    # every window row meets at least two window columns (the decoder's requirement)
    for w in A + B:
        deg = dem.H[w[0]][:, w[1]].sum(axis=1)
        assert deg.min() >= 2


def test_one_parallel_window_is_the_global_decode(model):
    dem, m, syn, _ = model
    p = oracle.RelayParams(num_sets=20)
    ref = oracle.decode(oracle.Graph(dem.H, dem.O), dem.priors, syn, p, nthreads=4)
    r = owin.decode_parallel(dem.H, dem.O, dem.priors, syn, m, dem.rounds, 2, 1, p, nthreads=4)
    np.testing.assert_array_equal(r["corrections"], ref["corrections"])
    np.testing.assert_array_equal(r["obs_pred"][:, : ref["obs_pred"].shape[1]], ref["obs_pred"])
    np.testing.assert_array_equal(r["converged"], ref["converged"])


@pytest.mark.parametrize("core,buffer,gap", [(3, 2, 2), (2, 1, 1)])
def test_parallel_converged_shots_explain_the_syndrome(model, core, buffer, gap):
    dem, m, syn, obs = model
    p = oracle.RelayParams(num_sets=20)
    r = owin.decode_parallel(dem.H, dem.O, dem.priors, syn, m, core, buffer, gap, p, nthreads=4)
    conv = r["converged"] == 1
    assert conv.mean() > 0.85
    assert not r["residual"][conv].any()
    e = owin._unpack(r["corrections"], dem.N)
    s = (e.astype(np.int64) @ dem.H.T.astype(np.int64)) % 2
    np.testing.assert_array_equal(owin._pack(s.astype(np.uint8))[conv], syn[conv])


@pytest.mark.parametrize("core,buffer,gap", [(3, 2, 2), (2, 1, 1), (4, 3, 2)])
def test_product_parallel_layout_equals_the_oracles(model, core, buffer, gap):
    """The GPU path's window layout (host code) against the oracle's own
    construction of the same definition, on a phenomenological and a
    circuit-level model."""
    from paper_2607_27644_amd import circuits
    from paper_2607_27644_amd.window import parallel_layout
    dem, m, _, _ = model
    circ = circuits.memory_dem("ZSZ-LP-160", "Z", 2e-3, rounds=4)
    for H, mm in ((dem.H, m), (circ.H, 64)):
        prod = parallel_layout(H, mm, core, buffer, gap)
        orc = owin.parallel_windows(H, mm, core, buffer, gap)
        assert len(prod[0]) == len(orc[0]) and len(prod[1]) == len(orc[1])
        for (rows, cols, cm, _, _), (orows, ocols, ocm) in zip(prod[0], orc[0]):
            np.testing.assert_array_equal(rows, orows)
            np.testing.assert_array_equal(cols, ocols)
            np.testing.assert_array_equal(cm, ocm)
        for (rows, cols, cm, fr, fc), (orows, ocols, ocm, ofixed) in zip(prod[1], orc[1]):
            np.testing.assert_array_equal(rows, orows)
            np.testing.assert_array_equal(cols, ocols)
            np.testing.assert_array_equal(fr, [i for i, _ in ofixed])
            np.testing.assert_array_equal(fc, [j for _, j in ofixed])
