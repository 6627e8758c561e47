"""Relay memory-strength grid search and LER sweep (App. "more numerics",
Table "relay gamma intervals"; Sec. 6.1) on the GPU decoder.

Checks: every interval decodes the same syndromes (a re-run reproduces each
count), the chosen interval is the minimum, an interval without negative
memory strengths fails far more often at p = 1e-2 than the default one, the
LER grows with p, and the sub-threshold fit reproduces its points.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2607_27644_amd import stats  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import experiments
    return experiments


def test_gamma_grid(E):
    r = E.gamma_grid("phen160", 1e-2, [-0.24, 0.0], [0.0, 0.66], 50000, seed=5)
    rows = {(x["gamma_min"], x["gamma_max"]): x for x in r["grid"]}
    assert set(rows) == {(-0.24, 0.0), (-0.24, 0.66), (0.0, 0.0), (0.0, 0.66)}
    best = min(r["grid"], key=lambda x: (x["failures"], x["mean_iters"]))
    assert r["best"] == best
    # paired: the same syndromes give the same counts on a second run
    r2 = E.gamma_grid("phen160", 1e-2, [-0.24], [0.66], 50000, seed=5)
    assert r2["grid"][0]["failures"] == rows[(-0.24, 0.66)]["failures"]
    # negative memory strengths matter at this noise level
    assert rows[(0.0, 0.66)]["failures"] > 4 * max(rows[(-0.24, 0.66)]["failures"], 1)


def test_ler_sweep_and_fit(E):
    ps = [8e-3, 1e-2, 1.2e-2, 1.5e-2]
    r = E.ler_sweep("phen160", ps, 100000, seed=9, p_fit_max=1.5e-2)
    f = [x["failures"] for x in r["points"]]
    assert f[0] < f[-1] and f[1] < f[-1]
    assert all(x["per_qubit_round_ci95"][0] <= x["per_qubit_round"] <= x["per_qubit_round_ci95"][1]
               for x in r["points"])
    assert "fit" in r and r["d_circ"] == 10
    c = r["fit"]["c"]
    for x in r["points"]:
        if x["failures"] >= 20:
            # the fitted curve passes within a factor of two of the well-measured points
            ratio = float(stats.ler_model(x["p"], c, 10)) / x["per_qubit_round"]
            assert 0.5 < ratio < 2.0, (x["p"], ratio)
