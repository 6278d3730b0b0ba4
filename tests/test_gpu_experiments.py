"""Smoke test of the statistical experiments (rank histograms, SIR collapse) at tiny scale:
they run through the batched and single-ensemble paths and return well-formed counts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_rank_histograms_and_sir_collapse_small():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01031_amd import experiments as ex
    r = ex.rank_histograms(torch, n_experiments=3, n_particles=6, da_hours=0.25,
                           forecast_hours=1.0 / 12, spinup_hours=1.0 / 12, batch=2)
    h = np.array(r["hist"])
    assert h.shape == (2, 6, 7) and np.all(h >= 0)
    assert np.all(h.sum(axis=2) == 3)
    assert 0.0 <= r["p_hu"] <= 1.0 and 0.0 <= r["p_hv"] <= 1.0
    s = ex.sir_collapse(torch, n_particles=12, da_hours=0.25, n_drifters=16, max_observed=3,
                        subsets=4)
    for key in ("kept_R", "kept_10R"):
        k = np.array(s[key])
        assert k.shape == (3,) and np.all(k >= 1.0) and np.all(k <= 12.0)
