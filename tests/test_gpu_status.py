"""Error semantics of the analysis at the C ABI (eq. betaTwoStage, non-finite values), forced
from the host with valid inputs: an ensemble too wide for its state dimension (beta <= 0)
and a NaN written into one particle's state.  Every kernel still runs to its end; the
analysis kernels read the status words the sync kernel writes and skip their writes.

  beta <= 0               IEWPF_E_BETA with or without stats; the state bit-unchanged
  NaN at an observed cell IEWPF_E_NONFINITE (non-finite c_i); the state bit-unchanged
  NaN elsewhere           IEWPF_E_NONFINITE naming the particle; every other particle equal
                          bit for bit to the analysis of the same ensemble without the NaN
  batched cycle           the same codes after a graph replay, naming the ensemble
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ensemble as oens
from oracle import observe as oobs
from oracle import philox as ophil

pytestmark = pytest.mark.gpu

CELLS = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1910_01031_amd import load
    load()
    return torch, torch.device("cuda:0")


def _bits(t):
    return t.contiguous().view(-1).view(dtype=__import__("torch").int32).cpu().numpy()


def _wide_ensemble(cfg):
    """Particles drawn independently (no common base): their c_i spread more than zeta, so
    beta <= 0 (the input of the beta test of the oracle suite)."""
    ens = W.as_f32(np.stack([oens.init_member(cfg, None, 0, i) for i in range(cfg.n_particles)]))
    truth = oens.init_member(cfg.replace(ensemble_id=77), None, 0, 0)
    y = oobs.mooring_obs(truth, CELLS, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    return ens, y


def _near_ensemble(cfg, spread=0.003):
    base = oens.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=spread)
    ens = W.as_f32(np.stack([oens.init_member(small, base, 1, i)
                             for i in range(cfg.n_particles)]))
    truth = oens.init_member(small.replace(ensemble_id=77), base, 1, 0)
    noise = ophil.normals(8, cfg.seed, 0, ophil.TAG_OBS, 77, 0).reshape(4, 2)
    return ens, oobs.mooring_obs(truth, CELLS, cfg.H, cfg.obs_sigma, noise)


@pytest.mark.parametrize("want_stats", [True, False])
def test_beta_error_leaves_the_state_untouched(torch_dev, want_stats):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context, IewpfError, abi
    _say(f"beta <= 0, stats {want_stats}")
    cfg = W.tiny().replace(n_particles=4)
    ens, y = _wide_ensemble(cfg)
    ctx = Context(cfg, max_obs=8)
    st = torch.from_numpy(ens.copy()).to(dev)
    with pytest.raises(IewpfError) as e:
        ctx.assimilate(st, CELLS, y, analysis_index=0, want_stats=want_stats)
    assert e.value.code == abi.IEWPF_E_BETA
    torch.cuda.synchronize()
    assert np.array_equal(_bits(st), ens.view(np.int32).reshape(-1))
    # the context stays usable: an ensemble near one state passes afterwards
    good, yg = _near_ensemble(cfg)
    st2 = torch.from_numpy(good.copy()).to(dev)
    stats = ctx.assimilate(st2, CELLS, yg, analysis_index=1)
    assert stats["beta"] > 0
    ctx.close()


def test_nan_at_an_observed_cell_leaves_the_state_untouched(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context, IewpfError, abi
    cfg = W.tiny()
    ens, y = _near_ensemble(cfg)
    ens[3, 1, CELLS[2, 1], CELLS[2, 0]] = np.nan  # hu of particle 3 at observation 2
    ctx = Context(cfg, max_obs=8)
    st = torch.from_numpy(ens.copy()).to(dev)
    with pytest.raises(IewpfError) as e:
        ctx.assimilate(st, CELLS, y, analysis_index=0, want_stats=False)
    assert e.value.code == abi.IEWPF_E_NONFINITE
    assert "particle 3" in str(e.value)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(st), ens.view(np.int32).reshape(-1))
    ctx.close()


def test_nan_away_from_observations_is_reported_after_the_update(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context, IewpfError, abi
    cfg = W.tiny()
    ens, y = _near_ensemble(cfg)
    bad = ens.copy()
    bad[6, 0, 16, 3] = np.nan  # eta of particle 6, no observation there
    ctx = Context(cfg, max_obs=8)
    ref = torch.from_numpy(ens.copy()).to(dev)
    ctx.assimilate(ref, CELLS, y, analysis_index=4, want_stats=False)
    st = torch.from_numpy(bad).to(dev)
    with pytest.raises(IewpfError) as e:
        ctx.assimilate(st, CELLS, y, analysis_index=4, want_stats=False)
    assert e.value.code == abi.IEWPF_E_NONFINITE
    assert "particle 6" in str(e.value)
    torch.cuda.synchronize()
    got, want = st.cpu().numpy(), ref.cpu().numpy()
    others = [i for i in range(cfg.n_particles) if i != 6]
    assert np.array_equal(got[others].view(np.int32), want[others].view(np.int32))
    assert np.isnan(got[6, 0, 16, 3])
    ctx.close()


def test_batched_cycle_reports_the_failing_ensemble(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Batch, Context, IewpfError, abi
    cfg0 = W.tiny().replace(ensemble_id=0)
    cfg1 = W.tiny().replace(n_particles=4, ensemble_id=1)
    e0, y0 = _near_ensemble(cfg0)
    e1, y1 = _wide_ensemble(cfg1)
    ctxs = [Context(cfg0, max_obs=8), Context(cfg1, max_obs=8)]
    sts = [torch.from_numpy(e0.copy()).to(dev), torch.from_numpy(e1.copy()).to(dev)]
    # the forecast the failing ensemble must keep: the same model steps on its own context
    fc = torch.from_numpy(e1.copy()).to(dev)
    solo = Context(cfg1, max_obs=8)
    solo.step_ensemble(fc, 2, first_step=0, noise_on_last=False)
    b = Batch(ctxs, sts)
    for e in range(2):
        b.set_cells(e, CELLS)
    for use_graph in (False, True):
        _say(f"batched status, graph {use_graph}")
        for e, src in enumerate((e0, e1)):
            sts[e].copy_(torch.from_numpy(src))
        with pytest.raises(IewpfError) as e:
            b.cycle(2, 0, 0, [y0, y1], use_graph=use_graph)
        assert e.value.code == abi.IEWPF_E_BETA
        assert "ensemble 1" in str(e.value)
        torch.cuda.synchronize()
        assert torch.equal(sts[1], fc)
        assert not torch.equal(sts[0], torch.from_numpy(e0).to(dev))  # ensemble 0 went on
    b.close()
    for c in ctxs + [solo]:
        c.close()
