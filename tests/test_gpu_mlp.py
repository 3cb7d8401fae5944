"""The warm-start network's HIP kernels (BF16 MFMA products, FP32
accumulation) against the FP64 oracle network, through the C ABI.

Tolerances come from the arithmetic.  The oracle is run with ``quant=True``,
rounding to bfloat16 at the same points as the kernels, so the two differ by
FP32-versus-FP64 accumulation (relative 1e-6) plus the rare activation whose
FP32 and FP64 values round to neighbouring bfloat16 numbers (one bfloat16
unit, 2^-8 relative, on that element).  Over three hidden layers of 256 such
flips move an output by far less than 2e-3 of the output range, the bound
used for outputs; gradients, built from the same activations and rounded
errors, are held to 1e-2 norm-wise per layer and the loss to 1e-3.
"""
import os

import numpy as np
import pytest
import torch

from oracle import mlp as M

pytestmark = pytest.mark.gpu

H = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global H
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1606_05474_amd import helios

    H = helios
    H.lib()
    yield


def _random_net(dims, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        o, n = dims[i + 1], dims[i]
        parts += [rng.normal(0, np.sqrt(2.0 / n), o * n), rng.normal(0, 0.1, o)]
    flat = np.concatenate(parts).astype(np.float32).astype(np.float64)
    norm = {"in_shift": rng.normal(0, 1, dims[0]).astype(np.float32).astype(np.float64),
            "in_scale": rng.uniform(0.5, 2, dims[0]).astype(np.float32).astype(np.float64),
            "out_shift": rng.normal(1000, 100, dims[-1]).astype(np.float32).astype(np.float64),
            "out_scale": rng.uniform(50, 200, dims[-1]).astype(np.float32).astype(np.float64)}
    net = H.MLP(dims)
    net.set_norm(norm["in_shift"], norm["in_scale"], norm["out_shift"], norm["out_scale"])
    net.set_params(flat)
    return net, flat, norm, rng


def _x(rng, B, n_in=6):
    return rng.normal(0, 1.5, (B, n_in)).astype(np.float32)


def test_bf16_copy_is_round_to_nearest_even():
    net, flat, _, _ = _random_net((6, 256, 256, 256, 100), 0)
    got = net.params_bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    want = M.bf16(flat)
    np.testing.assert_array_equal(got.view(np.float32).astype(np.float64), want)


@pytest.mark.parametrize("B", [1, 63, 200, 1000])
def test_forward_matches_oracle(B):
    net, flat, norm, rng = _random_net((6, 256, 256, 256, 100), 1)
    x = _x(rng, B)
    T = net.forward(x).cpu().numpy().astype(np.float64)
    Tq = M.temperatures(flat, x.astype(np.float64), norm, quant=True)
    y_ref = (Tq - norm["out_shift"]) / norm["out_scale"]
    y_gpu = (T - norm["out_shift"]) / norm["out_scale"]
    err = np.abs(y_gpu - y_ref).max() / np.abs(y_ref).max()
    assert err < 2e-3, err
    # and within the bfloat16 error of the exact float64 network
    T64 = M.temperatures(flat, x.astype(np.float64), norm, quant=False)
    assert np.abs(T - T64).max() / np.abs(T64 - norm["out_shift"]).max() < 3e-2


@pytest.mark.parametrize("dims", [(6, 256, 256, 256, 100), (5, 40, 40, 17), (6, 70, 3)])
def test_backward_matches_oracle(dims):
    net, flat, norm, rng = _random_net(dims, 2)
    B = 300
    x = _x(rng, B, dims[0])
    T = norm["out_shift"] + norm["out_scale"] * rng.normal(0, 1, (B, dims[-1]))
    xt = torch.as_tensor(x, device="cuda")
    Tt = torch.as_tensor(T.astype(np.float32), device="cuda")
    loss, grad = net.backward(xt, Tt)
    loss, grad = float(loss.item()), grad.cpu().numpy().astype(np.float64)
    l_ref, g_ref = M.loss_and_grad(flat, x.astype(np.float64), T.astype(np.float32).astype(np.float64), norm,
                                   dims, quant=True)
    assert abs(loss - l_ref) <= 1e-3 * l_ref, (loss, l_ref)
    for (gW, gb), (rW, rb) in zip(M.unpack(grad, dims), M.unpack(g_ref, dims)):
        assert np.linalg.norm(gW - rW) <= 1e-2 * np.linalg.norm(rW)
        assert np.linalg.norm(gb - rb) <= 1e-2 * np.linalg.norm(rb)


def test_adam_step_matches_oracle():
    net, flat, _, rng = _random_net((6, 256, 256, 256, 100), 3)
    m = np.zeros(flat.size)
    v = np.zeros(flat.size)
    w = flat.copy()
    for step in range(1, 4):
        g = rng.normal(0, 1e-2, flat.size).astype(np.float32)
        net.adam(torch.as_tensor(g, device="cuda"), lr=1e-3)
        w, m, v = M.adam_step(w, g.astype(np.float64), m, v, step, 1e-3)
    p = net.params.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(p, w, rtol=1e-5, atol=1e-7)
    got = net.params_bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(got.view(np.float32).astype(np.float64), M.bf16(p))


def test_training_on_device_fits_a_smooth_target():
    """A few hundred Adam steps of the device kernels reduce the loss on a
    smooth synthetic mapping by more than an order of magnitude."""
    dims = (6, 256, 256, 256, 100)
    net = H.MLP(dims)
    net.init(seed=7)
    rng = np.random.default_rng(8)
    B = 2048
    x = rng.uniform(-1, 1, (B, 6)).astype(np.float32)
    lp = np.linspace(0, 1, 100)
    T = (1000 + 300 * x[:, :1] * lp + 200 * np.tanh(x[:, 1:2] * 2) * (1 - lp) + 50 * x[:, 2:3]).astype(np.float32)
    net.set_norm(np.zeros(6), np.ones(6), T.mean(0), T.std(0) + 1e-3)
    xt, Tt = torch.as_tensor(x, device="cuda"), torch.as_tensor(T, device="cuda")
    first = float(net.backward(xt, Tt)[0].item())
    for _ in range(300):
        net.train_step(xt, Tt, lr=1e-3)
    last = float(net.backward(xt, Tt)[0].item())
    assert last < first / 10, (first, last)


def test_warm_start_interpolates_and_falls_back():
    from paper_1606_05474_amd import workloads as W

    net, flat, norm, rng = _random_net((6, 64, 64, 100), 4)
    # outputs near 1000 K with a narrow spread, so only the forced cases leave [10, 1e4] K
    net.set_norm(norm["in_shift"], norm["in_scale"], norm["out_shift"], np.full(100, 20.0))
    lp_net = np.log10(W.pressure_centres(100))  # the network's points, bottom to top
    atms = [W.plain_workload(n=n, nb=2)[0] for n in (100, 37, 150, 2)]
    b = H.Batch(atms)
    x = _x(rng, len(atms))
    x[2, 3] = np.nan  # forces a non-finite profile for atmosphere 2
    T_c = torch.zeros(b.total_n, dtype=torch.float64, device="cuda")
    fb = torch.full((len(atms),), -1, dtype=torch.int32, device="cuda")
    H.warm_start(b, net, x, lp_net, T_c, fb, T_iso=1000.0, T_lo=10.0, T_hi=1e4)
    T_net = net.forward(x).cpu().numpy().astype(np.float64)
    fb = fb.cpu().numpy()
    T_c = b.split_layer(T_c.cpu().numpy())
    for a, atm in enumerate(atms):
        want, wfb = M.warm_profile(lp_net, T_net[a], np.log10(atm["P_c"]), 1000.0, 10.0, 1e4)
        assert fb[a] == int(wfb)
        np.testing.assert_allclose(T_c[a], want, rtol=1e-12)
    assert list(fb) == [0, 0, 1, 0]
    # a bound below the profile sends every atmosphere to the isothermal start
    T_c2 = torch.zeros(b.total_n, dtype=torch.float64, device="cuda")
    fb2 = torch.zeros(len(atms), dtype=torch.int32, device="cuda")
    H.warm_start(b, net, x, lp_net, T_c2, fb2, T_iso=900.0, T_lo=10.0, T_hi=float(T_net[np.isfinite(T_net)].min()) - 1)
    assert np.all(fb2.cpu().numpy() == 1) and np.all(T_c2.cpu().numpy() == 900.0)


def test_mlp_errors_are_reported():
    net = H.MLP((6, 32, 10))
    with pytest.raises(H.HeliosError):
        net.forward(np.zeros((0, 6), np.float32))
    bad = H.HeliosMlp(6, 0, 1, 10)
    assert H.lib().helios_mlp_param_count(bad) == 0


WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_1606_05474_amd", "data", "warmstart_mlp.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained warm-start network in the tree")
def test_trained_network_shortens_the_solve():
    """The committed network (trained on the device by these kernels) starts
    held-out atmospheres close to their equilibrium: fewer temperature
    updates to the same tolerance than the isothermal start, and profiles
    within a few tens of kelvin of the converged ones."""
    from paper_1606_05474_amd import warmstart as WS
    from paper_1606_05474_amd import workloads as W

    net = WS.load(WEIGHTS)
    atms, kt = W.learned_workload(40, 24, 100)
    b = H.Batch(atms)
    s = H.Solver(b, H.KTable(kt), prec=H.FP64)
    T0 = np.concatenate([a["T0"] for a in atms])
    s.reset(T0)
    c_iso, it_iso, _ = s.run(400, 10, graph=True)
    T_conv = s.T_c.cpu().numpy().copy()
    x = np.stack([a["params"] for a in atms])
    fb = s.warm_reset(net, x, net.logP)
    T_start = s.T_c.cpu().numpy().copy()
    c_nn, it_nn, rs = s.run(400, 10, graph=True, restart_after=150)
    assert fb.sum() == 0
    both = c_iso & c_nn
    assert both.sum() >= len(atms) // 2
    assert np.median(it_nn[both]) < 0.8 * np.median(it_iso[both]), (np.median(it_nn[both]), np.median(it_iso[both]))
    err = [np.sqrt(np.mean((T_start[b.lay_off[a]:b.lay_off[a + 1]] - T_conv[b.lay_off[a]:b.lay_off[a + 1]]) ** 2))
           for a in np.where(c_iso)[0]]
    assert np.median(err) < 60.0, np.median(err)
