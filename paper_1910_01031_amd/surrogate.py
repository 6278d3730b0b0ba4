"""Training and evaluation of the learned surrogate forecast on the GPU.

The surrogate maps a state psi_t to psi_{t + 5 min} (ten deterministic model steps of the
finite-volume scheme).  Training pairs come from ensembles on a grid of the target spacing and
scheme step (a 3x3 convolutional network is translation invariant, so it applies to any grid
of that spacing; the states should resemble the ones it will see): each ensemble is drawn
around a balanced base state, spun up with stochastic model steps, and then paired window by
window with its deterministic ten-step forecast.  Every arithmetic step of the method runs in
the library's kernels (ensemble generation, scheme, normalisation statistics, network
forward/backward, Adam); this module orders the calls, slices device buffers and computes the
learning-rate schedule (a scalar per step) and the evaluation RMSEs (torch reductions over
outputs, for reporting).  `python -m paper_1910_01031_amd.surrogate` times the forward pass.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import abi


@dataclass
class PairSet:
    x: "object"        # device float32 [N][3][ny][nx]
    t: "object"        # device float32 [N][3][ny][nx], ten deterministic model steps later
    mu: np.ndarray     # per-channel mean of x
    sigma: np.ndarray  # per-channel standard deviation of x
    scale: np.ndarray  # per-channel standard deviation of t - x


def make_pairs(torch, cfg, n_pairs: int, base: np.ndarray, group: int = 1000,
               spinup_steps: int = 20, windows_per_group: int = 2, window_steps: int = 10,
               stream_base: int = 100) -> PairSet:
    """n_pairs training pairs (x, M^window_steps x) on cfg's grid; base [3][ny][nx] is the
    state the ensembles are drawn around (initial-state covariance of cfg)."""
    dev = torch.device("cuda")
    per = group * windows_per_group
    n_groups = (n_pairs + per - 1) // per
    xs = torch.empty((n_groups * per, 3, cfg.ny, cfg.nx), device=dev)
    ts = torch.empty_like(xs)
    ctx = abi.Context(cfg.replace(n_particles=group))
    d_base = torch.from_numpy(np.ascontiguousarray(base, dtype=np.float32)).to(dev)
    ens = torch.empty((group, 3, cfg.ny, cfg.nx), device=dev)
    try:
        for gi in range(n_groups):
            ctx.init_ensemble(ens, d_base, stream_index=stream_base + gi)
            step = 1_000_000 * (gi + 1)
            ctx.step_ensemble(ens, spinup_steps, first_step=step, noise_on_last=True)
            step += spinup_steps
            for w in range(windows_per_group):
                lo = (gi * windows_per_group + w) * group
                xs[lo:lo + group].copy_(ens)
                for k in range(window_steps):
                    ctx.step_ensemble(ens, 1, first_step=step + k, noise_on_last=False)
                ts[lo:lo + group].copy_(ens)
                # continue the stochastic run from the end of the window
                ctx.perturb(ens, step + window_steps - 1)
                step += window_steps
        torch.cuda.synchronize()
    finally:
        ctx.close()
    xs, ts = xs[:n_pairs].contiguous(), ts[:n_pairs].contiguous()
    mu, sigma, scale = abi.norm_stats(xs, ts)
    return PairSet(xs, ts, mu, sigma, scale)


def init_params(seed: int, last_scale: float = 0.1) -> np.ndarray:
    """He-style initial weights, zero biases, flat in the network's parameter order."""
    rng = np.random.default_rng(seed)
    ch = (3, 48, 48, 48, 48, 48, 3)
    out = []
    for i in range(6):
        std = np.sqrt(2.0 / (9 * ch[i])) * (last_scale if i == 5 else 1.0)
        out.append((rng.normal(size=ch[i + 1] * ch[i] * 9) * std).astype(np.float32))
        out.append(np.zeros(ch[i + 1], np.float32))
    return np.concatenate(out)


def train(net: abi.Net, pairs: PairSet, n_steps: int, batch: int = 64, lr: float = 1e-3,
          lr_final: float = 1e-4, log_every: int = 0, seed: int = 0):
    """n_steps Adam steps on contiguous mini-batches of the pair set (the pairs are already
    in random order across ensembles); cosine decay from lr to lr_final.  Returns the loss
    history sampled every log_every steps (empty when 0)."""
    net.set_norm(pairs.mu, pairs.sigma, pairs.scale)
    n = pairs.x.shape[0]
    nb = max(1, n // batch)
    rng = np.random.default_rng(seed)
    order = rng.permutation(nb)
    hist = []
    for it in range(n_steps):
        b = int(order[it % nb])
        lo = b * batch
        cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * it / max(1, n_steps)))
        want = bool(log_every) and (it % log_every == 0 or it == n_steps - 1)
        loss = net.train_step(pairs.x[lo:lo + batch], pairs.t[lo:lo + batch], float(cur),
                              want_loss=want)
        if want:
            hist.append((it, loss))
    return hist


def evaluate(torch, net: abi.Net, pairs: PairSet, batch: int = 256):
    """Per-channel RMSE of the surrogate against the plain ten-step forecast, and the same
    for persistence (psi_t as forecast) for scale."""
    n = pairs.x.shape[0]
    se = torch.zeros(3, dtype=torch.float64, device=pairs.x.device)
    sp = torch.zeros_like(se)
    out = torch.empty_like(pairs.x[:batch])
    for lo in range(0, n, batch):
        hi = min(n, lo + batch)
        o = out[:hi - lo]
        net.forward(pairs.x[lo:hi], o)
        se += ((o - pairs.t[lo:hi]).double() ** 2).sum(dim=(0, 2, 3))
        sp += ((pairs.x[lo:hi] - pairs.t[lo:hi]).double() ** 2).sum(dim=(0, 2, 3))
    cells = n * pairs.x.shape[2] * pairs.x.shape[3]
    return (torch.sqrt(se / cells).cpu().numpy(), torch.sqrt(sp / cells).cpu().numpy())


def time_forward(torch, batch: int, ny: int, nx: int, reps: int = 5, seed: int = 0):
    """Milliseconds per network forward on `batch` random states of ny x nx (He-initialised
    weights), after two untimed calls."""
    net = abi.Net(batch * ny * nx)
    try:
        net.set_params(init_params(seed))
        net.set_norm(np.zeros(3, np.float32), np.array([0.4, 50.0, 50.0], np.float32),
                     np.array([0.01, 1.0, 1.0], np.float32))
        gen = torch.Generator(device="cuda").manual_seed(seed)
        scale = torch.tensor([0.4, 50.0, 50.0], device="cuda")[None, :, None, None]
        x = torch.randn((batch, 3, ny, nx), device="cuda", generator=gen) * scale
        y = torch.empty_like(x)
        for _ in range(2):
            net.forward(x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            net.forward(x, y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        net.close()


if __name__ == "__main__":
    import argparse
    import json

    import torch

    ap = argparse.ArgumentParser(description="time the surrogate forward pass")
    ap.add_argument("--batch", type=int, default=100)
    ap.add_argument("--ny", type=int, default=300)
    ap.add_argument("--nx", type=int, default=500)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    ms = time_forward(torch, a.batch, a.ny, a.nx, a.reps)
    flop = 171_072 * a.batch * a.ny * a.nx
    print(json.dumps({"forward_ms": ms, "tflops": flop / (ms / 1e3) / 1e12,
                      "shape": [a.batch, 3, a.ny, a.nx]}), flush=True)
