"""GPU parity of the learned surrogate (BF16 MFMA convolutions, backward pass, Adam, mass-drift
guard with plain-solver fallback) against the FP64 oracle on BF16-rounded operands.

Forward pass, layer by layer (the exact check).  Both sides round the same operands to
BF16; they differ only in how the K = 9 C_in products of a pre-activation are summed (FP32 on
the matrix cores, FP64 in the oracle).  Fed the GPU's own BF16 input of a layer, the oracle's
FP64 pre-activation z and the GPU's FP32 one differ by at most (K + 2) 2^-24 (sum |w a| + |b|)
(the standard bound for a K-term floating-point sum).  Rounding to BF16 is monotone, so the
GPU's BF16 output must lie between bf16(relu(z - delta)) and bf16(relu(z + delta)): equal to
the oracle's rounding except where z sits within delta of a rounding boundary, and one of the
two neighbours there.  The rounding of the layer-0 input is replayed in FP32 as the kernel
computes it, so it is compared bit for bit.

Forward pass, end to end.  A boundary case that rounds the other way moves one layer input by
one BF16 ulp (2^-8 relative) and the later layers carry that on; the end-to-end outputs are
therefore compared statistically (99.9 % of them within 2^-6 of the output RMS, all within
2^-4, mean deviation below 2^-11 of it; observed: 99.9 % within 2^-7.8, all within 2^-6.6).

Backward pass, layer by layer (the exact check).  Fed the GPU's own BF16 layer inputs and
pre-activation gradients, every weight and bias gradient lies within the FP32 summation bound
of the oracle's FP64 sum, and every pre-activation gradient between the BF16 roundings of
the bounds of its FP64 value (test_backward_layerwise_exact).

Backward pass, end to end.  The gradients of the whole network are also compared per tensor
in relative Frobenius norm (1e-2): the loss gradient and every pre-activation gradient are
rounded to BF16 on both sides, so the same boundary cases are the only source of difference.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import surrogate as osur

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def _unflat(flat):
    out, off = [], 0
    for i in range(6):
        cin, cout = osur.CHANNELS[i], osur.CHANNELS[i + 1]
        w = flat[off:off + cout * cin * 9].reshape(cout, cin, 3, 3).astype(np.float64)
        off += cout * cin * 9
        b = flat[off:off + cout].astype(np.float64)
        off += cout
        out.append((w, b))
    return out


def _params(seed, last_scale=1.0, bias_std=0.05):
    rng = np.random.default_rng(seed)
    p = osur.init_params(rng, last_scale=last_scale)
    p = [(w, (rng.normal(size=b.shape) * bias_std).astype(np.float32).astype(np.float64))
         for w, b in p]
    return p


def _states(B, H, W, seed):
    cfg = wl.tiny().replace(nx=W, ny=H)
    rng = np.random.default_rng(seed)
    return np.stack([wl.random_state(cfg, rng) for _ in range(B)]).astype(np.float32)


NORM = (np.array([0.0, 0.0, 0.0], np.float32), np.array([0.4, 50.0, 50.0], np.float32),
        np.array([0.01, 1.0, 1.0], np.float32))


def _x_norm(psi):
    mu, sig, _ = NORM
    return (psi.astype(np.float64) - mu[:, None, None]) / sig[:, None, None]


@pytest.mark.parametrize("B,H,W", [(2, 32, 32), (3, 20, 37), (1, 5, 7), (2, 9, 50)])
def test_forward_matches_oracle(B, H, W):
    _need_gpu()
    from paper_1910_01031_amd import Net
    params = _params(11 + H)
    psi = _states(B, H, W, 5 + W)
    net = Net(B * H * W)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    d_in = torch.from_numpy(psi).cuda()
    d_out = torch.empty_like(d_in)
    net.forward(d_in, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy().astype(np.float64)
    s = NORM[2].astype(np.float64)
    for b in range(B):
        y, _ = osur.forward(params, _x_norm(psi[b]))
        want = psi[b].astype(np.float64) + s[:, None, None] * y
        y_gpu = (got[b] - psi[b].astype(np.float64)) / s[:, None, None]
        # the FP32 residual add rounds psi + s y once: compare net outputs through it
        f32_slack = np.abs(want) * 2.0 ** -23 / s[:, None, None]
        rms = np.sqrt(np.mean(y * y))
        err = np.maximum(np.abs(y_gpu - y) - f32_slack, 0.0)
        assert np.quantile(err, 0.999) <= 2.0 ** -6 * rms, (b, np.quantile(err, 0.999), rms)
        assert err.max() <= 2.0 ** -4 * rms, (b, err.max(), rms)
        assert np.mean(err) <= 2.0 ** -11 * rms
    net.close()


def _bf16_bits_to_f64(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("B,H,W", [(2, 32, 32), (3, 20, 37), (1, 5, 7), (2, 9, 50)])
def test_forward_layerwise_exact(B, H, W):
    """Every layer's BF16 output equals the oracle's rounding of its FP64 pre-activation
    (computed from the GPU's own BF16 input), up to the rounding-boundary cases bounded by
    the FP32 summation error; the last layer's FP32 output within that error."""
    _need_gpu()
    from paper_1910_01031_amd import Net
    params = _params(11 + H)
    psi = _states(B, H, W, 5 + W)
    net = Net(B * H * W)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    net.keep_activations(True)  # layer by layer, every hidden activation kept
    d_in = torch.from_numpy(psi).cuda()
    d_out = torch.empty_like(d_in)
    net.forward(d_in, d_out)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy().astype(np.float64)
    cells = B * H * W
    acts = [None] + [_bf16_bits_to_f64(net.read_activation(L, cells)).reshape(B, H, W, 48)
                     .transpose(0, 3, 1, 2) for L in range(1, 6)]
    mu, sig, sc = NORM
    isig = np.float32(1.0) / sig
    x32 = (psi - mu[None, :, None, None]) * isig[None, :, None, None]  # FP32, as the kernel
    a0 = osur.bf16_round(x32)
    n_boundary = 0
    for b in range(B):
        a = a0[b]
        for i, (w, bias) in enumerate(params):
            wq = osur.bf16_round(w)
            z = osur.conv3x3(a, wq, bias)
            K = 9 * a.shape[0]
            delta = (K + 2) * 2.0 ** -24 * osur.conv3x3(np.abs(a), np.abs(wq), np.abs(bias))
            if i < 5:
                lo = osur.bf16_round(np.maximum(z - delta, 0.0))
                hi = osur.bf16_round(np.maximum(z + delta, 0.0))
                got = acts[i + 1][b]
                assert np.all((got >= lo) & (got <= hi)), (b, i)
                n_boundary += int(np.sum(got != osur.bf16_round(np.maximum(z, 0.0))))
                a = got
            else:
                s = sc.astype(np.float64)[:, None, None]
                want = psi[b].astype(np.float64) + s * z
                tol = s * delta + (np.abs(want) + s * np.abs(z)) * 2.0 ** -23
                assert np.all(np.abs(out[b] - want) <= tol), (b, np.max(np.abs(out[b] - want) - tol))
    # boundary cases are rare: a few per million outputs
    assert n_boundary <= max(4, 1e-4 * 5 * 48 * cells), n_boundary
    net.close()


@pytest.mark.parametrize("B,H,W", [(2, 16, 16), (1, 12, 40)])
def test_gradients_match_oracle(B, H, W):
    _need_gpu()
    from paper_1910_01031_amd import Net
    params = _params(3 + W, last_scale=0.5)
    psi = _states(B, H, W, 21)
    tgt = psi + _states(B, H, W, 22) * np.array([0.01, 0.5, 0.5], np.float32)[None, :, None, None]
    net = Net(B * H * W)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    g, loss, y = net.gradients(torch.from_numpy(psi).cuda(), torch.from_numpy(tgt).cuda())
    s = NORM[2].astype(np.float64)
    # oracle over the batch: the loss is the mean over all cells and channels of the batch
    ys, caches = [], []
    for b in range(B):
        yb, cb = osur.forward(params, _x_norm(psi[b]))
        ys.append(yb)
        caches.append(cb)
    yo = np.stack(ys)
    t = (tgt.astype(np.float64) - psi.astype(np.float64)) / s[None, :, None, None]
    loss_o, gout = osur.mse_loss_and_grad(yo, t)
    gsum = None
    for b in range(B):
        gb = osur.backward(params, caches[b], gout[b], round_grads=True)
        fb = np.concatenate([np.concatenate([w.ravel(), bb.ravel()]) for w, bb in gb])
        gsum = fb if gsum is None else gsum + fb
    # network output (cells x channels, NHWC on the GPU)
    y_gpu = y.reshape(B, H, W, 3).transpose(0, 3, 1, 2)
    assert np.max(np.abs(y_gpu - yo)) <= 2.0 ** -7 * np.sqrt(np.mean(yo * yo))
    assert abs(loss - loss_o) <= 1e-3 * loss_o
    off = 0
    for i in range(6):
        cin, cout = osur.CHANNELS[i], osur.CHANNELS[i + 1]
        for n in (cout * cin * 9, cout):
            a, o = g[off:off + n].astype(np.float64), gsum[off:off + n]
            rel = np.linalg.norm(a - o) / max(np.linalg.norm(o), 1e-30)
            assert rel <= 1e-2, (i, n, rel)
            off += n
    net.close()


@pytest.mark.parametrize("B,H,W", [(2, 16, 16), (1, 12, 40), (1, 5, 7)])
def test_backward_layerwise_exact(B, H, W):
    """Every element of the backward pass against the oracle fed the GPU's own BF16
    intermediates (layer inputs and pre-activation gradients), so the only differences left
    are the FP32 summations and the BF16 roundings, each bounded per element:
      loss gradient     bf16 of 2 (y - (target - x)/s) / n, whose FP32 evaluation errs by at
                        most (2/n)(3u|t| + 2u|d|) + 4u|v| (u = 2^-24): the GPU's value lies
                        between the roundings of v -+ that bound;
      weight and bias   sum over cells of dz a (BF16 x BF16 products are exact in FP32): within
      gradients         (cells + 2) 2u sum |dz a| of the FP64 sum;
      input gradient    dz of layer L-1 = bf16(mask * sum_k w dz), the K = 9 C_out term FP32
                        sum within (K + 2) 2u sum |w dz|: between the roundings of the bounds,
                        zero where layer L-1's ReLU output is zero.
    The matrix-core sums are bounded with 2u per addition (an ulp: the bound holds whether
    the hardware rounds to nearest or truncates)."""
    _need_gpu()
    from paper_1910_01031_amd import Net
    u = 2.0 ** -24
    params = _params(5 + W, last_scale=0.5)
    psi = _states(B, H, W, 41 + W)
    tgt = psi + _states(B, H, W, 42) * np.array([0.01, 0.5, 0.5], np.float32)[None, :, None, None]
    net = Net(B * H * W)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    g, loss, y = net.gradients(torch.from_numpy(psi).cuda(), torch.from_numpy(tgt).cuda())
    cells = B * H * W

    def nchw(a, ch):
        return a.reshape(B, H, W, ch).transpose(0, 3, 1, 2)

    acts = [None] + [nchw(_bf16_bits_to_f64(net.read_activation(L, cells)), 48)
                     for L in range(1, 6)]
    mu, sig, sc = NORM
    x32 = (psi - mu[None, :, None, None]) * (np.float32(1.0) / sig)[None, :, None, None]
    acts[0] = osur.bf16_round(x32)
    dz = [nchw(_bf16_bits_to_f64(net.read_gradient_signal(L, cells)), 3 if L == 5 else 48)
          for L in range(6)]
    # loss gradient
    yv = nchw(y.astype(np.float64), 3)
    t = (tgt.astype(np.float64) - psi.astype(np.float64)) / sc.astype(np.float64)[None, :, None, None]
    d = yv - t
    n = 3.0 * cells
    v = 2.0 * d / n
    dv = (2.0 / n) * (3 * u * np.abs(t) + 2 * u * np.abs(d)) + 4 * u * np.abs(v)
    assert np.all((dz[5] >= osur.bf16_round(v - dv)) & (dz[5] <= osur.bf16_round(v + dv)))
    off = 0
    offs = []
    for i in range(6):
        cin, cout = osur.CHANNELS[i], osur.CHANNELS[i + 1]
        offs.append((off, off + cout * cin * 9))
        off += cout * cin * 9 + cout
    n_boundary = 0
    for L in range(5, -1, -1):
        w, bias = params[L]
        wq = osur.bf16_round(w)
        cin, cout = osur.CHANNELS[L], osur.CHANNELS[L + 1]
        gw = sum(osur.conv3x3_weight_grad(dz[L][b], acts[L][b]) for b in range(B))
        gwa = sum(osur.conv3x3_weight_grad(np.abs(dz[L][b]), np.abs(acts[L][b])) for b in range(B))
        gb = dz[L].sum(axis=(0, 2, 3))
        gba = np.abs(dz[L]).sum(axis=(0, 2, 3))
        w0, b0 = offs[L]
        got_w = g[w0:b0].astype(np.float64).reshape(cout, cin, 3, 3)
        got_b = g[b0:b0 + cout].astype(np.float64)
        assert np.all(np.abs(got_w - gw) <= (cells + 2) * 2 * u * gwa), (L, "weights")
        assert np.all(np.abs(got_b - gb) <= (cells + 2) * 2 * u * gba), (L, "biases")
        if L == 0:
            break
        K = 9 * cout
        for b in range(B):
            s_ = osur.conv3x3_input_grad(dz[L][b], wq)
            delta = (K + 2) * 2 * u * osur.conv3x3_input_grad(np.abs(dz[L][b]), np.abs(wq))
            on = acts[L][b] > 0.0
            lo = np.where(on, osur.bf16_round(s_ - delta), 0.0)
            hi = np.where(on, osur.bf16_round(s_ + delta), 0.0)
            got = dz[L - 1][b]
            assert np.all((got >= lo) & (got <= hi)), (L, b)
            n_boundary += int(np.sum(got != np.where(on, osur.bf16_round(s_), 0.0)))
    assert n_boundary <= max(4, 1e-4 * 5 * 48 * cells), n_boundary
    net.close()


def test_adam_step_matches_oracle():
    _need_gpu()
    from paper_1910_01031_amd import Net
    B, H, W = 2, 16, 16
    params = _params(9, last_scale=0.5)
    p0 = _flat(params).astype(np.float32)
    psi = _states(B, H, W, 31)
    tgt = psi + _states(B, H, W, 32) * np.array([0.01, 0.5, 0.5], np.float32)[None, :, None, None]
    net = Net(B * H * W)
    net.set_params(p0)
    net.set_norm(*NORM)
    dx, dt = torch.from_numpy(psi).cuda(), torch.from_numpy(tgt).cuda()
    g, _, _ = net.gradients(dx, dt)
    lr = 1e-3
    net.train_step(dx, dt, lr)          # first Adam step from the same gradients
    g2, _, _ = net.gradients(dx, dt)     # parameters moved: gradients differ
    net.train_step(dx, dt, lr)
    p2 = net.get_params()
    opt = osur.Adam([(p0.astype(np.float64), np.zeros(1))], lr=lr)
    p1o = opt.step([(p0.astype(np.float64), np.zeros(1))], [(g.astype(np.float64), np.zeros(1))])
    p2o = opt.step(p1o, [(g2.astype(np.float64), np.zeros(1))])[0][0]
    # FP32 Adam vs FP64: |p| ~ 0.1, lr = 1e-3; differences are FP32 roundoff except where a
    # gradient is near zero (m / sqrt(v) then depends on the last bits of g)
    big = (np.abs(g) > 1e-3 * np.abs(g).max()) & (np.abs(g2) > 1e-3 * np.abs(g2).max())
    assert np.max(np.abs(p2 - p2o)[big]) <= 1e-6
    assert np.max(np.abs(p2 - p2o)) <= 2.0 * lr + 1e-6
    net.close()


def test_training_reduces_loss():
    _need_gpu()
    from paper_1910_01031_amd import Context, Net
    cfg = wl.tiny().replace(dx=5e3, dy=5e3, n_sub=2, n_particles=16, init_std=0.3)
    ctx = Context(cfg)
    base = torch.from_numpy(wl.jet_state(cfg).astype(np.float32)).cuda()
    x = torch.empty((cfg.n_particles, 3, cfg.ny, cfg.nx), device="cuda")
    ctx.init_ensemble(x, base, stream_index=7)
    t = x.clone()
    for k in range(10):  # ten deterministic model steps (the 5-minute window)
        ctx.step_ensemble(t, 1, first_step=k, noise_on_last=False)
    torch.cuda.synchronize()
    net = Net(cfg.n_particles * cfg.n_cells)
    net.set_params(_flat(_params(1, last_scale=0.1, bias_std=0.0)).astype(np.float32))
    xs = x.cpu().numpy()
    inc = t.cpu().numpy() - xs
    mu = xs.mean(axis=(0, 2, 3))
    sig = xs.std(axis=(0, 2, 3)) + 1e-6
    sc = inc.std(axis=(0, 2, 3)) + 1e-9
    net.set_norm(mu, sig, sc)
    losses = [net.train_step(x, t, 1e-3, want_loss=True) for _ in range(150)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
    net.close()
    ctx.close()


def test_trained_network_beats_persistence_on_held_out_windows():
    """What the learned part adds: after training on windows the solver generates, the
    network's 5-minute forecast of held-out states (another ensemble stream) is much closer
    to the solver's than keeping the state unchanged (persistence)."""
    _need_gpu()
    from paper_1910_01031_amd import Net
    from paper_1910_01031_amd import surrogate as sur
    cfg = wl.tiny().replace(dx=5e3, dy=5e3, n_sub=2, init_std=0.3)
    base = wl.jet_state(cfg)
    train = sur.make_pairs(torch, cfg, 1024, base, group=128, spinup_steps=6, windows_per_group=4,
                           stream_base=300)
    held = sur.make_pairs(torch, cfg, 256, base, group=128, spinup_steps=6, windows_per_group=2,
                          stream_base=900)
    net = Net(64 * cfg.n_cells)
    net.set_params(sur.init_params(5))
    sur.train(net, train, n_steps=400, batch=32, lr=2e-3, lr_final=2e-4, seed=5)
    rmse, persist = sur.evaluate(torch, net, held, batch=64)
    print("held-out RMSE (eta, hu, hv)", rmse, "persistence", persist, flush=True)
    assert np.all(np.isfinite(rmse))
    # the momenta change most over the window; eta only has to stay near persistence
    assert np.all(rmse[1:] < 0.5 * persist[1:]), (rmse, persist)
    assert rmse[0] < 1.5 * persist[0], (rmse, persist)
    net.close()


def _window_setup(n_particles=6):
    from paper_1910_01031_amd import Context, Net
    cfg = wl.tiny().replace(dx=5e3, dy=5e3, n_sub=2, n_particles=n_particles, init_std=0.3)
    ctx = Context(cfg)
    base = torch.from_numpy(wl.jet_state(cfg).astype(np.float32)).cuda()
    x = torch.empty((cfg.n_particles, 3, cfg.ny, cfg.nx), device="cuda")
    ctx.init_ensemble(x, base, stream_index=3)
    net = Net(cfg.n_particles * cfg.n_cells)
    params = _params(4, last_scale=0.2)
    return cfg, ctx, net, params, x


def test_window_without_fallback_is_the_network():
    _need_gpu()
    from paper_1910_01031_amd import surrogate_window
    cfg, ctx, net, params, x = _window_setup()
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    ref = torch.empty_like(x)
    net.forward(x, ref)
    st = x.clone()
    nf, drift = surrogate_window(ctx, net, st, 10, 0, drift_tol=1e30, noise_scale=0.0)
    torch.cuda.synchronize()
    assert nf == 0
    assert torch.equal(st, ref)
    xin, out = x.cpu().numpy().astype(np.float64), st.cpu().numpy().astype(np.float64)
    for i in range(cfg.n_particles):
        assert abs(drift[i] - osur.mass_drift(xin[i], out[i], cfg.H)) <= 1e-12
    net.close()
    ctx.close()


def test_forced_drift_falls_back_to_the_plain_solver():
    """A large bias on the eta output channel forces mass drift; every particle above the
    threshold is re-stepped by the plain solver, the others keep the network output."""
    _need_gpu()
    from paper_1910_01031_amd import surrogate_window
    cfg, ctx, net, params, x = _window_setup()
    plain = x.clone()
    ctx.step_ensemble(plain, 1, first_step=0, noise_on_last=False)
    netout = torch.empty_like(x)
    # all particles drift: bias 1e3 on the eta increment (scale 0.01 -> +10 m of eta)
    w5, b5 = params[5]
    forced = params[:5] + [(w5, b5 + np.array([1e3, 0.0, 0.0]))]
    net.set_params(_flat(forced).astype(np.float32))
    net.set_norm(*NORM)
    net.set_horizon(1)  # the network stands in for one model step here
    st = x.clone()
    nf, drift = surrogate_window(ctx, net, st, 1, 0, drift_tol=1e-4, noise_scale=0.0)
    torch.cuda.synchronize()
    assert nf == cfg.n_particles and np.all(drift > 1e-4)
    assert torch.equal(st, plain)
    # mixed: threshold between the particles' drifts under the unforced network
    net.set_params(_flat(params).astype(np.float32))
    net.forward(x, netout)
    st = x.clone()
    _, d0 = surrogate_window(ctx, net, st, 1, 0, drift_tol=1e30, noise_scale=0.0)
    tol = float(np.median(d0))
    st = x.clone()
    nf, drift = surrogate_window(ctx, net, st, 1, 0, drift_tol=tol, noise_scale=0.0)
    torch.cuda.synchronize()
    flagged = drift > tol
    assert nf == int(flagged.sum()) and 0 < nf < cfg.n_particles
    for i in range(cfg.n_particles):
        assert torch.equal(st[i], plain[i] if flagged[i] else netout[i]), i
    net.close()
    ctx.close()


def _window_tolerances(ctx, net, x):
    """Drift thresholds flagging no particle, about half of them, and all of them."""
    from paper_1910_01031_amd import surrogate_window
    st = x.clone()
    _, d0 = surrogate_window(ctx, net, st, 10, 0, drift_tol=1e30, noise_scale=0.0)
    return [1e30, float(np.median(d0)), 0.0]


@pytest.mark.parametrize("row_form", ["1", "0"])
def test_async_window_equals_the_synchronous_window(row_form, monkeypatch):
    """The window without host waits (masked plain re-steps over all particles) leaves the
    state of the synchronous window (flagged particles packed and re-stepped) bit for bit, and
    reports the same fallback count and drifts, for no, some and all particles flagged; with
    the scheme step in its full-row form (one workgroup per particle strip) and in its strip
    form (one wave per strip), the two places the mask is read."""
    _need_gpu()
    from paper_1910_01031_amd import surrogate_window, surrogate_window_async
    monkeypatch.setenv("IEWPF_SWE_ROW", row_form)
    cfg, ctx, net, params, x = _window_setup()
    monkeypatch.delenv("IEWPF_SWE_ROW")
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    nfd = torch.zeros(1, dtype=torch.int32, device="cuda")
    dd = torch.zeros(cfg.n_particles, dtype=torch.float64, device="cuda")
    for tol in _window_tolerances(ctx, net, x):
        for noise in (0.0, 1.0):
            ref = x.clone()
            nf, drift = surrogate_window(ctx, net, ref, 10, 40, drift_tol=tol, noise_scale=noise)
            st = x.clone()
            surrogate_window_async(ctx, net, st, 10, 40, tol, noise, nfd, dd)
            torch.cuda.synchronize()
            print(f"tol {tol:g} noise {noise}: {nf} re-stepped", flush=True)
            assert int(nfd.item()) == nf
            assert np.array_equal(dd.cpu().numpy(), drift)
            assert torch.equal(st, ref)
    net.close()
    ctx.close()


def test_async_window_replays_in_a_graph():
    """The window without host waits captured once in a graph (about half the particles
    flagged, noise on): every replay, with eager work and synchronisations between the
    replays, equals the eager synchronous window."""
    _need_gpu()
    from paper_1910_01031_amd import surrogate_window, surrogate_window_async
    cfg, ctx, net, params, x = _window_setup()
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    tol = _window_tolerances(ctx, net, x)[1]
    ref = x.clone()
    nf, drift = surrogate_window(ctx, net, ref, 10, 70, drift_tol=tol, noise_scale=1.0)
    assert 0 < nf < cfg.n_particles
    st = x.clone()
    nfd = torch.zeros(1, dtype=torch.int32, device="cuda")
    dd = torch.zeros(cfg.n_particles, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
        surrogate_window_async(ctx, net, st, 10, 70, tol, 1.0, nfd, dd, stream=side)
    for r in range(3):
        st.copy_(x)
        nfd.fill_(-1)
        dd.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"replay {r}: {int(nfd.item())} re-stepped", flush=True)
        assert int(nfd.item()) == nf
        assert np.array_equal(dd.cpu().numpy(), drift)
        assert torch.equal(st, ref)
    del g
    net.close()
    ctx.close()


def test_window_noise_is_one_scaled_model_error_draw():
    _need_gpu()
    from paper_1910_01031_amd import surrogate_window
    cfg, ctx, net, params, x = _window_setup()
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    det = x.clone()
    surrogate_window(ctx, net, det, 10, 20, drift_tol=1e30, noise_scale=0.0)
    ref = det.clone()
    ctx.perturb(ref, 29)
    st = x.clone()
    surrogate_window(ctx, net, st, 10, 20, drift_tol=1e30, noise_scale=1.0)
    torch.cuda.synchronize()
    assert torch.equal(st, ref)
    st3 = x.clone()
    surrogate_window(ctx, net, st3, 10, 20, drift_tol=1e30, noise_scale=3.0)
    torch.cuda.synchronize()
    p1 = (ref - det).double()
    p3 = (st3 - det).double()
    scale = p1.abs().max().item()
    assert scale > 0
    assert (p3 - 3.0 * p1).abs().max().item() <= 1e-3 * scale + 1e-6 * det.abs().max().item()
    net.close()
    ctx.close()


def test_rejects_oversized_and_invalid_calls():
    _need_gpu()
    from paper_1910_01031_amd import IewpfError, Net
    net = Net(100)
    x = torch.zeros((1, 3, 10, 11), device="cuda")
    with pytest.raises(IewpfError):
        net.forward(x, torch.empty_like(x))
    with pytest.raises(IewpfError):
        net.set_params(np.zeros(net.num_params - 1, np.float32))
    with pytest.raises(IewpfError):
        net.set_norm([0, 0, 0], [1, 0, 1], [1, 1, 1])
    with pytest.raises(IewpfError):
        net.set_horizon(0)
    net.close()


def test_window_length_must_match_the_horizon():
    # a network trained for 10-step windows refuses other window lengths, for the window and
    # the drifter forecast alike, and accepts them once its horizon says so
    _need_gpu()
    from paper_1910_01031_amd import IewpfError, forecast_drifters_surrogate, surrogate_window
    from paper_1910_01031_amd import abi
    cfg, ctx, net, params, x = _window_setup(n_particles=2)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    st = x.clone()
    with pytest.raises(IewpfError) as e:
        surrogate_window(ctx, net, st, 5, 0, drift_tol=1e30, noise_scale=0.0)
    assert e.value.code == abi.IEWPF_E_ARG
    p = torch.from_numpy(np.stack([wl.drifter_lattice(cfg, 2, 2)] * 2)).cuda()
    with pytest.raises(IewpfError) as e:
        forecast_drifters_surrogate(ctx, net, st, p, 1, 5, 40, drift_tol=1e30, noise_scale=0.0)
    assert e.value.code == abi.IEWPF_E_ARG
    torch.cuda.synchronize()
    assert torch.equal(st, x)  # nothing ran
    net.set_horizon(5)
    nf, _ = surrogate_window(ctx, net, st, 5, 0, drift_tol=1e30, noise_scale=0.0)
    assert nf == 0
    net.close()
    ctx.close()


def test_surrogate_drifter_forecast_matches_interpolated_heun():
    """Drifters under the surrogate: every window's end state is the network output, and the
    drifters take Heun steps in the states interpolated linearly in time across the window
    (the oracle's Heun step on the same interpolated states)."""
    _need_gpu()
    from oracle import drifters as odr
    from paper_1910_01031_amd import forecast_drifters_surrogate
    cfg, ctx, net, params, x = _window_setup(n_particles=3)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    rng = np.random.default_rng(8)
    pos0 = np.stack([wl.drifter_lattice(cfg, 3, 3) + rng.normal(scale=2e3, size=(9, 2))
                     for _ in range(3)])
    p = torch.from_numpy(pos0.copy()).cuda()
    traj = torch.zeros((21, 3, 9, 2), dtype=torch.float64, device="cuda")
    st = x.clone()
    nf = forecast_drifters_surrogate(ctx, net, st, p, 2, 10, 40, drift_tol=1e30,
                                     noise_scale=0.0, traj=traj)
    assert nf == 0
    e1 = torch.empty_like(x)
    net.forward(x, e1)
    e2 = torch.empty_like(x)
    net.forward(e1, e2)
    torch.cuda.synchronize()
    assert torch.equal(st, e2)
    ends = [x.cpu().numpy().astype(np.float64), e1.cpu().numpy().astype(np.float64),
            e2.cpu().numpy().astype(np.float64)]
    got = traj.cpu().numpy()
    for i in range(3):
        pos = pos0[i].copy()
        for w in range(2):
            a, b = ends[w][i], ends[w + 1][i]
            for s in range(10):
                pa = a + (s / 10.0) * (b - a)
                pb = a + ((s + 1) / 10.0) * (b - a)
                pos = odr.heun_step(pos, pa, pb, cfg, cfg.dt)
                assert np.abs(got[w * 10 + s + 1, i] - pos).max() < 1e-8, (i, w, s)
    assert np.abs(p.cpu().numpy()[i] - pos).max() < 1e-8
    net.close()
    ctx.close()


def test_analysis_runs_on_the_surrogate_output():
    """The IEWPF analysis takes the surrogate's forecast as it is: a guarded window of the
    network followed by an analysis equals the oracle's analysis of the same forecast (1e-5
    per field), with beta within its float32-normals bound and equal realised weights."""
    _need_gpu()
    from oracle import iewpf as oiewpf
    from oracle import observe as oobs
    from paper_1910_01031_amd import Context, surrogate_window
    cfg, ctx, net, params, x = _window_setup(n_particles=8)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    st = x.clone()
    nf, _ = surrogate_window(ctx, net, st, 10, 0, drift_tol=1e30, noise_scale=0.0)
    assert nf == 0
    torch.cuda.synchronize()
    fc = st.cpu().numpy().astype(np.float64)
    acfg = cfg.replace(obs_sigma=20.0)
    actx = Context(acfg, max_obs=4)
    rng = np.random.default_rng(3)
    truth = wl.jet_state(cfg) + 0.1 * wl.random_state(cfg, rng)
    cells = np.array([[5, 6], [21, 9], [12, 25], [28, 28]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, acfg.obs_sigma, np.zeros((4, 2)))
    stats = actx.assimilate(st, cells, y, analysis_index=3)
    sc = actx.particle_scalars()
    got = st.cpu().numpy().astype(np.float64)
    ref, info = oiewpf.analysis(fc, cells, y, acfg, 3)
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        assert err < 1e-5, (f, err)
    assert abs(stats["beta"] - info["beta"]) < 2.0 ** -22 * abs(info["beta"] - 1.0) + 1e-12
    w = oiewpf.realized_weight(sc[:, 3], sc[:, 1], sc[:, 2], stats["beta"], sc[:, 0], acfg.n_psi)
    assert np.abs(w - stats["cbar"]).max() < 1e-9 * acfg.n_psi
    actx.close()
    net.close()
    ctx.close()


def test_normalisation_statistics_match_their_definition():
    """iewpf_norm_stats: per-channel mean and standard deviation (n - 1) of the inputs plus
    1e-6 and of the increments plus 1e-9, against numpy in float64 (1e-10 relative), on a
    ragged size (the workgroups' slices end mid-image)."""
    _need_gpu()
    from paper_1910_01031_amd import abi
    B, H, W = 3, 37, 53
    x = _states(B, H, W, 61)
    t = x + _states(B, H, W, 62) * np.array([0.01, 0.5, 0.5], np.float32)[None, :, None, None]
    mu, sigma, scale = abi.norm_stats(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    x64, d64 = x.astype(np.float64), t.astype(np.float64) - x.astype(np.float64)
    ref_mu = x64.mean(axis=(0, 2, 3))
    ref_sig = x64.std(axis=(0, 2, 3), ddof=1) + 1e-6
    ref_sc = d64.std(axis=(0, 2, 3), ddof=1) + 1e-9
    # the mean to float64 summation error (relative to the largest value), the deviations
    # to 1e-10 relative
    amax = np.abs(x64).max(axis=(0, 2, 3))
    assert np.all(np.abs(mu - ref_mu) <= 1e-12 * amax), (mu, ref_mu)
    for got, ref in ((sigma, ref_sig), (scale, ref_sc)):
        assert np.all(np.abs(got - ref) <= 1e-10 * np.abs(ref)), (got, ref)


@pytest.mark.parametrize("B,H,W", [(2, 37, 70), (1, 5, 9), (1, 300, 500)])
def test_fused_forward_equals_layer_by_layer(B, H, W):
    """The inference forward runs layers 0 and 1 as one fused pass (layer 0's activation kept
    on chip); its output, and the inputs of layers 2..5, equal the layer-by-layer forward bit
    for bit: tiles ragged in both directions (37 x 70 against 14 x 30 tiles), a grid smaller
    than one tile's halo (5 x 9, the halo wraps more than once), and the paper's grid.  After
    the fused forward the input of layer 1 is not kept and reading it is refused."""
    _need_gpu()
    from paper_1910_01031_amd import IewpfError, Net, abi
    params = _params(23 + W, last_scale=0.3)
    psi = _states(B, H, W, 7 + H)
    net = Net(B * H * W)
    net.set_params(_flat(params).astype(np.float32))
    net.set_norm(*NORM)
    d_in = torch.from_numpy(psi).cuda()
    ref = torch.empty_like(d_in)
    got = torch.empty_like(d_in)
    cells = B * H * W
    net.keep_activations(True)
    net.forward(d_in, ref)
    torch.cuda.synchronize()
    kept = {L: net.read_activation(L, cells) for L in (2, 3, 4, 5)}
    net.keep_activations(False)
    got.fill_(float("nan"))
    net.forward(d_in, got)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
    for L in (2, 3, 4, 5):
        assert np.array_equal(net.read_activation(L, cells), kept[L]), L
    for L in (1,):
        with pytest.raises(IewpfError) as e:
            net.read_activation(L, cells)
        assert e.value.code == abi.IEWPF_E_ARG
    net.close()
