"""iewpf_resample_noalloc (residual resampling with its partial results in the library's fixed
device array, no allocation) against iewpf_resample (the context's workspaces): parents
bit-exact and the resampled states bit-exact, on two calls in a row with the second on fewer
particles (the array keeps the first call's contents), plus the oracle's parents from the
same log-weights (Section "Standard particle filter").  Sizes beyond the array and
overlapping states are refused before any launch."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W
from oracle import resample as ores

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_resample_matches_the_context_resample():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1910_01031_amd import Context, abi
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31)
    for ne, aidx in ((41, 3), (17, 4)):  # the second call is smaller
        _say(f"no-alloc resampling: {ne} particles, analysis {aidx}")
        cfg = W.tiny().replace(n_particles=ne, ensemble_id=5)
        ens = W.as_f32(rng.normal(size=(ne, 3, cfg.ny, cfg.nx)))
        lw = rng.normal(scale=2.0, size=ne)
        lw[1] = -np.inf  # zero weight
        lw_t = torch.from_numpy(lw).to(dev)
        ctx = Context(cfg, max_obs=4)
        st = torch.from_numpy(ens.copy()).to(dev)
        par = torch.zeros(ne, dtype=torch.int32, device=dev)
        ctx.resample(st, lw_t, analysis_index=aidx, parents=par)
        inp = torch.from_numpy(ens.copy()).to(dev)
        out = torch.full_like(inp, float("nan"))
        par2 = torch.full((ne,), -1, dtype=torch.int32, device=dev)
        abi.resample_noalloc(lw_t, inp, out, par2, cfg.seed, cfg.ensemble_id, aidx)
        torch.cuda.synchronize()
        assert torch.equal(par2, par)
        assert np.array_equal(out.cpu().numpy().view(np.int32), st.cpu().numpy().view(np.int32))
        assert torch.equal(inp, torch.from_numpy(ens).to(dev))  # input untouched
        u = ores.resample_uniforms(ne, cfg.seed, aidx, cfg.ensemble_id)
        ref, _ = ores.residual_resample(lw, u)
        assert np.array_equal(par2.cpu().numpy(), ref)
        ctx.close()


def test_noalloc_resample_refuses_before_launching():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1910_01031_amd import abi
    lib = abi.load()
    dev = torch.device("cuda:0")
    x = torch.zeros((4, 12), device=dev)
    lw = torch.zeros(4, dtype=torch.float64, device=dev)
    par = torch.zeros(4, dtype=torch.int32, device=dev)
    args = (ctypes.c_uint64(1), ctypes.c_uint32(0), ctypes.c_uint64(0), lw.data_ptr())
    rc = lib.iewpf_resample_noalloc(65536, 12, *args, x.data_ptr(), x.data_ptr() + 4096, par.data_ptr(),
                                    None)
    assert rc == abi.IEWPF_E_CAPACITY
    rc = lib.iewpf_resample_noalloc(4, 12, *args, x.data_ptr(), x.data_ptr() + 16, par.data_ptr(),
                                    None)
    assert rc == abi.IEWPF_E_ARG  # overlapping states
    rc = lib.iewpf_resample_noalloc(4, 10, *args, x.data_ptr(), x.data_ptr(), par.data_ptr(), None)
    assert rc == abi.IEWPF_E_SHAPE
