"""The analysis update's forms give the same state bit for bit, and the form that reaches
the windows through per-lane wrapped offsets matches the FP64 oracle.

The update (eq. optUpdateEquationTwoStage with the pull of eq. detailedOPDUpdate) has two
kernels, one staging the pull windows in LDS and one reading them through the caches; each
takes a window's column either as lane 0's offset (grids at least a window plus a wave
wide) or as the window's first column, wrapped per lane (narrower grids and windows folded
onto the period); every row walks the range of windows that hold it, so the strip height
(rows per wave) does not change the order of any sum.  Every combination must give the same
bits.  Shapes: 200 x 120 (lane-0 offsets), 100 x 92 (per-lane wrap, windows not folded: the
grid is wider than a window but narrower than a window plus a wave), 160 x 48 (windows folded
in y only).  Tolerance against the oracle: float32 state 1e-5 relative per field."""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ensemble as oens
from oracle import iewpf as oiewpf
from oracle import observe as oobs
from oracle import philox as ophil

pytestmark = pytest.mark.gpu
TOL = 1e-5

SHAPES = [(200, 120, 12, (6, 5)), (100, 92, 10, (3, 3)), (160, 48, 8, (5, 2))]


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


def _inputs(nx, ny, ne, lat):
    cfg = W.Config(nx=nx, ny=ny, dx=5e3, dy=5e3, n_sub=2, c_omega=4, n_particles=ne,
                   seed=W.SEED_BASE + 9, init_std=0.05)
    base = oens.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=0.01)
    ens = W.as_f32(np.stack([oens.init_member(small, base, 1, i) for i in range(ne)]))
    truth = oens.init_member(small.replace(ensemble_id=77), base, 1, 0)
    cells = W.buoy_cells(nx, ny, *lat)
    noise = ophil.normals(2 * len(cells), cfg.seed, 0, ophil.TAG_OBS, 77, 0).reshape(-1, 2)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
    return cfg, ens, cells, y


def _analyse(torch, dev, cfg, ens, cells, y, env):
    from paper_1910_01031_amd import Context
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        ctx = Context(cfg, max_obs=len(cells))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    st = torch.from_numpy(ens.copy()).to(dev)
    ctx.assimilate(st, cells, y, analysis_index=3)
    torch.cuda.synchronize()
    out = st.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("nx,ny,ne,lat", SHAPES)
def test_update_forms_bit_identical(torch_dev, nx, ny, ne, lat):
    torch, dev = torch_dev
    cfg, ens, cells, y = _inputs(nx, ny, ne, lat)
    forms = [{}, {"IEWPF_UPD_LDS": "0"}, {"IEWPF_UPD_STRIP": "3"},
             {"IEWPF_UPD_STRIP": "13", "IEWPF_UPD_LDS": "0"}, {"IEWPF_UPD_STRIP": "29"}]
    ref = None
    for env in forms:
        _say(f"{nx}x{ny}: update form {env or 'default'}")
        got = _analyse(torch, dev, cfg, ens, cells, y, env)
        assert np.isfinite(got).all()
        assert not np.array_equal(got, ens)  # the analysis moved the state
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got.view(np.int32), ref.view(np.int32)), env


def test_update_per_lane_wrap_matches_oracle(torch_dev):
    torch, dev = torch_dev
    nx, ny, ne, lat = SHAPES[1]
    cfg, ens, cells, y = _inputs(nx, ny, ne, lat)
    got = _analyse(torch, dev, cfg, ens, cells, y, {}).astype(np.float64)
    ref, _ = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 3, particles=[0, ne - 1])
    for n, i in enumerate((0, ne - 1)):
        for f in range(3):
            err = np.abs(got[i, f] - ref[n, f]).max() / np.abs(ref[n, f]).max()
            _say(f"  particle {i} field {f} rel err {err}")
            assert err < TOL
