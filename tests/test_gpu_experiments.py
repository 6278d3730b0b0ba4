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
    assert h.shape == (2, 6, 7) and np.all(h >= 0)  # six probe cells
    assert np.all(h.sum(axis=2) == 3)
    assert 0.0 <= r["p_hu"] <= 1.0 and 0.0 <= r["p_hv"] <= 1.0
    s = ex.sir_collapse(torch, n_particles=12, da_hours=0.25, n_drifters=16, max_observed=3,
                        subsets=4)
    for key in ("kept_R", "kept_10R"):
        k = np.array(s[key])
        assert k.shape == (3,) and np.all(k >= 1.0) and np.all(k <= 12.0)


def test_drift_forecast_error_norms_match_their_definitions():
    """The large-ensemble drift forecast at reduced size (12 particles on the 500x300 grid,
    3 analyses, 2 forecast hours, 4 drifters): the forecast error E(t) (eq.
    errorPerEnsembleDrifter, eq. errorNorm) and the spread RMSE(t) it reports for the plain
    and the surrogate forecast equal the oracle's definitions applied to the returned
    positions (minimum-image distances, 1e-9 relative)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import workloads as W
    from oracle import drifters as odr
    from paper_1910_01031_amd import experiments as ex
    r = ex.drift_forecast(torch, n_particles=12, da_hours=0.25, forecast_hours=2, n_drifters=4,
                          train_steps=5, net_particles=2, keep_positions=True)
    cfg = W.large_ensemble()
    lx, ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    P = r["positions"]
    assert P["truth"].shape == (2, 4, 2) and P["plain"].shape == (2, 12, 4, 2)
    for name in ("plain", "surrogate"):
        for h in range(2):
            e = odr.forecast_error(P[name][h], P["truth"][h], lx, ly)
            rm = odr.forecast_rmse(P[name][h], lx, ly)
            assert abs(r[name]["E"][h] - e) <= 1e-9 * e, (name, h)
            assert abs(r[name]["RMSE"][h] - rm) <= 1e-9 * rm, (name, h)
    # the drifters moved: the forecast is not the release lattice
    assert np.abs(P["plain"][1] - W.drifter_lattice(cfg, 2, 2)[None]).max() > 1.0
