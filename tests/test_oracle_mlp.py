"""Pins of the warm-start network's oracle (oracle/mlp.py) against what fixes
it independently: torch's CPU float64 layers, autograd and Adam, torch's
bfloat16 conversion, central finite differences of the loss, and closed
forms of the profile interpolation."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def _net(dims, seed):
    rng = np.random.default_rng(seed)
    layers = [(rng.normal(0, 1 / np.sqrt(i), (o, i)), rng.normal(0, 0.1, o)) for o, i in M.layer_shapes(dims)]
    norm = {"in_shift": rng.normal(0, 1, dims[0]), "in_scale": rng.uniform(0.5, 2, dims[0]),
            "out_shift": rng.normal(1000, 100, dims[-1]), "out_scale": rng.uniform(50, 200, dims[-1])}
    return M.pack(layers), norm, rng


def test_param_count_and_layout():
    assert M.param_count() == 6 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 100 + 100
    flat = np.arange(M.param_count(), dtype=np.float64)
    layers = M.unpack(flat)
    assert layers[0][0].shape == (256, 6) and layers[3][0].shape == (100, 256)
    assert layers[0][1][0] == 6 * 256 and layers[1][0][0, 0] == 6 * 256 + 256
    np.testing.assert_array_equal(M.pack(layers), flat)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.001953125, 3e38, -3.4e38, 1e-40, np.inf]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = M.bf16(x)
    np.testing.assert_array_equal(got, want)
    assert np.isnan(M.bf16(np.array([np.nan]))[0])


def test_forward_matches_torch_float64():
    flat, norm, rng = _net(M.DIMS, 1)
    x = rng.normal(0, 1, (9, 6))
    layers = M.unpack(flat)
    h = (torch.from_numpy(x) - torch.from_numpy(norm["in_shift"])) * torch.from_numpy(norm["in_scale"])
    for li, (W, b) in enumerate(layers):
        h = torch.nn.functional.linear(h, torch.from_numpy(W.copy()), torch.from_numpy(b.copy()))
        if li < 3:
            h = torch.nn.functional.gelu(h, approximate="none")
    y, _ = M.forward(flat, x, norm)
    np.testing.assert_allclose(y, h.numpy(), rtol=1e-12, atol=1e-12)
    T = M.temperatures(flat, x, norm)
    np.testing.assert_allclose(T, norm["out_shift"] + norm["out_scale"] * h.numpy(), rtol=1e-13)


def test_gradient_matches_torch_autograd():
    flat, norm, rng = _net(M.DIMS, 2)
    x = rng.normal(0, 1, (7, 6))
    T = rng.normal(1000, 150, (7, 100))
    loss, g = M.loss_and_grad(flat, x, T, norm)
    p = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
    off, h = 0, (torch.from_numpy(x) - torch.from_numpy(norm["in_shift"])) * torch.from_numpy(norm["in_scale"])
    shapes = M.layer_shapes()
    for li, (o, i) in enumerate(shapes):
        W = p[off:off + o * i].view(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        h = h @ W.T + b
        if li < len(shapes) - 1:
            h = torch.nn.functional.gelu(h, approximate="none")
    t = (torch.from_numpy(T) - torch.from_numpy(norm["out_shift"])) / torch.from_numpy(norm["out_scale"])
    L = ((h - t) ** 2).mean()
    L.backward()
    assert abs(loss - L.item()) <= 1e-12 * abs(L.item())
    np.testing.assert_allclose(g, p.grad.numpy(), rtol=1e-10, atol=1e-14 * np.abs(p.grad.numpy()).max())


def test_gradient_matches_central_differences():
    dims = (6, 8, 7, 9, 5)
    flat, norm, rng = _net(dims, 3)
    x = rng.normal(0, 1, (4, 6))
    T = rng.normal(1000, 150, (4, 5))
    _, g = M.loss_and_grad(flat, x, T, norm, dims)
    for k in rng.choice(flat.size, 40, replace=False):
        h = 1e-5 * max(1.0, abs(flat[k]))
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        lp, _ = M.loss_and_grad(fp, x, T, norm, dims)
        lm, _ = M.loss_and_grad(fm, x, T, norm, dims)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1e-3, abs(g[k])), (k, fd, g[k])


def test_gelu_and_derivative_limits():
    z = np.array([-40.0, -3.0, 0.0, 3.0, 40.0])
    g = M.gelu(z)
    assert g[0] == 0.0 and g[2] == 0.0 and g[4] == 40.0
    np.testing.assert_allclose(M.gelu_grad(np.array([-40.0, 0.0, 40.0])), [0.0, 0.5, 1.0], atol=1e-15)
    zz = np.linspace(-5, 5, 101)
    fd = (M.gelu(zz + 1e-6) - M.gelu(zz - 1e-6)) / 2e-6
    np.testing.assert_allclose(M.gelu_grad(zz), fd, atol=1e-8)


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    w0 = rng.normal(0, 1, 50)
    p = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        gr = rng.normal(0, 1, 50)
        p.grad = torch.from_numpy(gr.copy())
        opt.step()
        w, m, v = M.adam_step(w, gr, m, v, step, 3e-3)
        np.testing.assert_allclose(w, p.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_warm_profile_interpolation_and_fallback():
    lp_nn = np.linspace(3.0, -6.0, 100) + 6.0  # descending, bottom to top
    T_nn = 1500.0 - 80.0 * (lp_nn - 3.0)
    lp_layers = np.array([9.5, 9.0, 5.3, 0.0, -1.0])  # two below the range, one above
    T, fb = M.warm_profile(lp_nn, T_nn, lp_layers, 1000.0, 10.0, 1e4)
    assert not fb
    lin = 1500.0 - 80.0 * (np.clip(lp_layers, 0.0, 9.0) - 3.0)
    np.testing.assert_allclose(T, lin, rtol=1e-14)
    T, fb = M.warm_profile(lp_nn, T_nn, lp_nn, 1000.0, 10.0, 1e4)
    np.testing.assert_array_equal(T, T_nn)
    bad = T_nn.copy()
    bad[7] = np.nan
    T, fb = M.warm_profile(lp_nn, bad, lp_layers, 1000.0, 10.0, 1e4)
    assert fb and np.all(T == 1000.0)
    bad = T_nn.copy()
    bad[0] = 2e4
    assert M.warm_profile(lp_nn, bad, lp_layers, 1000.0, 10.0, 1e4)[1]


@pytest.mark.parametrize("quant", [False, True])
def test_quantised_network_stays_near_exact(quant):
    """Rounding at the BF16 points moves outputs by about the bfloat16 unit
    roundoff (2^-8) relative to their spread, not more."""
    flat, norm, rng = _net(M.DIMS, 5)
    x = rng.normal(0, 1, (32, 6))
    y0, _ = M.forward(flat, x, norm, quant=False)
    y1, _ = M.forward(flat, x, norm, quant=quant)
    err = np.abs(y1 - y0).max() / np.abs(y0).max()
    assert err < (3e-2 if quant else 1e-15), err
