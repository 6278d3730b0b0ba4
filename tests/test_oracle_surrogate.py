"""Pins of the surrogate oracle: BF16 rounding, periodic conv3x3 against torch's
circular-padding conv2d, gradients against torch autograd and central finite differences,
Adam against its closed-form first step."""
import numpy as np
import pytest
import torch

from oracle import surrogate as sg


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-6, 6, size=1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.0e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(sg.bf16_round(x), ref)


def test_conv_matches_torch_circular():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(5, 7, 9))
    w = rng.normal(size=(4, 5, 3, 3))
    b = rng.normal(size=4)
    out = sg.conv3x3(x, w, b)
    conv = torch.nn.Conv2d(5, 4, 3, padding=1, padding_mode="circular", dtype=torch.float64)
    with torch.no_grad():
        conv.weight.copy_(torch.from_numpy(w))
        conv.bias.copy_(torch.from_numpy(b))
        ref = conv(torch.from_numpy(x)[None])[0].numpy()
    assert np.abs(out - ref).max() < 1e-12


def _torch_net(params):
    layers = []
    for i, (w, b) in enumerate(params):
        conv = torch.nn.Conv2d(w.shape[1], w.shape[0], 3, padding=1, padding_mode="circular",
                               dtype=torch.float64)
        with torch.no_grad():
            conv.weight.copy_(torch.from_numpy(w))
            conv.bias.copy_(torch.from_numpy(b))
        layers.append(conv)
        if i < 5:
            layers.append(torch.nn.ReLU())
    return torch.nn.Sequential(*layers)


def test_gradients_match_torch_autograd():
    # straight-through BF16: compare with the same network on BF16-rounded weights/inputs
    rng = np.random.default_rng(2)
    params = sg.init_params(rng)
    params = [(sg.bf16_round(w), rng.normal(size=b.shape) * 0.05) for w, b in params]
    x = sg.bf16_round(rng.normal(size=(3, 8, 10)))
    # use inputs whose layer outputs are BF16-exact is impractical: compare with torch on
    # the same per-layer rounding by feeding torch the oracle's cached inputs
    y, cache = sg.forward(params, x)
    gout = rng.normal(size=y.shape)
    grads = sg.backward(params, cache, gout)
    for i in range(6):
        a, wq, z = cache[i]
        at = torch.from_numpy(a).requires_grad_(True)
        wt = torch.from_numpy(wq).requires_grad_(True)
        bt = torch.from_numpy(params[i][1]).requires_grad_(True)
        zt = torch.nn.functional.conv2d(torch.nn.functional.pad(at[None], (1, 1, 1, 1), mode="circular"),
                                        wt, bt)[0]
        assert np.abs(zt.detach().numpy() - z).max() < 1e-10
    # whole-network check in float64 without rounding effects: compare backward with autograd
    # on a network whose operands are BF16-exact and pre-activation rounding is skipped
    net = _torch_net(params)
    xt = torch.from_numpy(x)[None].requires_grad_(True)
    out = net(xt)[0]
    (out * torch.from_numpy(gout)).sum().backward()
    # the oracle rounds hidden activations to BF16; rebuild a rounding-free oracle pass
    a = x
    c2 = []
    for i, (w, b) in enumerate(params):
        z = sg.conv3x3(a, w, b)
        c2.append((a, w, z))
        a = np.maximum(z, 0) if i < 5 else z
    g2 = sg.backward(params, c2, gout)
    for i, conv in enumerate(m for m in net if isinstance(m, torch.nn.Conv2d)):
        assert np.abs(g2[i][0] - conv.weight.grad.numpy()).max() < 1e-9 * max(1, np.abs(g2[i][0]).max())
        assert np.abs(g2[i][1] - conv.bias.grad.numpy()).max() < 1e-9 * max(1, np.abs(g2[i][1]).max())
    assert len(grads) == 6


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 5, 6))
    w = rng.normal(size=(3, 2, 3, 3))
    b = rng.normal(size=3)
    gy = rng.normal(size=(3, 5, 6))
    f = lambda w_, x_: float(np.sum(gy * sg.conv3x3(x_, w_, b)))
    gw = sg.conv3x3_weight_grad(gy, x)
    gx = sg.conv3x3_input_grad(gy, w)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (2, 1, 1, 2), (1, 0, 2, 1)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        assert abs((f(wp, x) - f(wm, x)) / (2 * h) - gw[idx]) < 1e-6 * max(1, abs(gw[idx]))
    for idx in [(0, 0, 0), (1, 4, 5), (0, 2, 3)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        assert abs((f(w, xp) - f(w, xm)) / (2 * h) - gx[idx]) < 1e-6 * max(1, abs(gx[idx]))


def test_adam_first_step_closed_form():
    params = [(np.ones((1, 1, 3, 3)), np.zeros(1))]
    grads = [(np.full((1, 1, 3, 3), 0.5), np.full(1, -2.0))]
    opt = sg.Adam(params, lr=0.01)
    new = opt.step(params, grads)
    # first step: m/(1-b1) = g, v/(1-b2) = g^2 -> p -= lr * g / (|g| + eps)
    assert np.allclose(new[0][0], 1.0 - 0.01 * 0.5 / (0.5 + 1e-8))
    assert np.allclose(new[0][1], 0.0 + 0.01 * 2.0 / (2.0 + 1e-8))


def test_mass_drift():
    a = np.zeros((3, 4, 4))
    b = a.copy()
    b[0, 0, 0] = 0.023 * 16
    assert abs(sg.mass_drift(a, b, 230.0) - 0.023 / 230.0) < 1e-15
