"""FP64 reference of the learned warm start: the multilayer perceptron that
maps six atmosphere parameters to an initial temperature profile, its
gradient, its optimizer step and the interpolation of its profile onto an
atmosphere's layers.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the test suite, the
smoke check and the benchmark's CPU baseline may use it; the product path
never does.  Plain numpy in float64, written out from the definitions; no
code is shared with the GPU kernels.

The paper itself starts every atmosphere from a fixed profile; the network is
an addition to the method.  Its definition:

* layers 6 -> 256 -> 256 -> 256 -> 100, affine maps ``z = W h + b`` with
  ``W`` stored [out][in];
* GELU in the exact (error-function) form after each hidden layer,
  ``gelu(z) = z Phi(z)`` with ``Phi`` the standard normal CDF; linear output;
* inputs normalised as ``(x - in_shift) * in_scale``; outputs are normalised
  temperatures, ``T = out_shift + out_scale * y``;
* loss: mean squared error over batch and outputs in the normalised units;
* optimizer: Adam (Kingma & Ba 2015, Algorithm 1) with bias correction.

``quant=True`` reproduces the points at which a BF16 implementation rounds:
the normalised inputs, the weights, the hidden activations and the
back-propagated errors are rounded to bfloat16 (round to nearest, ties to
even, from the float32 value), everything else stays in float64.  With
``quant=False`` the network is evaluated exactly in float64.

Flat parameter layout (float32 on the device, float64 here): for each layer
in order, ``W`` row-major [out][in] followed by ``b`` [out].
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

DIMS = (6, 256, 256, 256, 100)


# ------------------------------------------------------------ layout
def layer_shapes(dims=DIMS):
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def param_count(dims=DIMS) -> int:
    return sum(o * i + o for o, i in layer_shapes(dims))


def unpack(flat, dims=DIMS):
    """[(W, b)] views of a flat parameter vector."""
    out, off = [], 0
    for o, i in layer_shapes(dims):
        W = flat[off:off + o * i].reshape(o, i)
        off += o * i
        b = flat[off:off + o]
        off += o
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in layers])


# ------------------------------------------------------------ bfloat16
def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) from the float32 value,
    returned as float64.  NaN stays NaN; overflow goes to infinity."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ------------------------------------------------------------ activation
def gelu(z):
    """z * Phi(z), Phi the standard normal CDF."""
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    """d/dz of z * Phi(z) = Phi(z) + z * phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


# ------------------------------------------------------------ network
def forward(flat, x, norm, dims=DIMS, quant=False):
    """Normalised outputs y [B][n_out] and the cache for backward.
    norm = dict(in_shift, in_scale, out_shift, out_scale)."""
    q = bf16 if quant else (lambda v: np.asarray(v, np.float64))
    layers = unpack(np.asarray(flat, np.float64), dims)
    h = q((np.asarray(x, np.float64) - norm["in_shift"]) * norm["in_scale"])
    hs, zs = [h], []
    for li, (W, b) in enumerate(layers):
        z = h @ q(W).T + b
        if li == len(layers) - 1:
            return z, {"h": hs, "z": zs, "layers": layers}
        zs.append(z)
        h = q(gelu(z))
        hs.append(h)
    raise AssertionError("unreachable")


def temperatures(flat, x, norm, dims=DIMS, quant=False):
    y, _ = forward(flat, x, norm, dims, quant)
    return norm["out_shift"] + norm["out_scale"] * y


def loss_and_grad(flat, x, T, norm, dims=DIMS, quant=False):
    """Mean squared error in normalised units and its gradient with respect
    to the flat parameters (back-propagation written out layer by layer)."""
    y, c = forward(flat, x, norm, dims, quant)
    q = bf16 if quant else (lambda v: v)
    t = (np.asarray(T, np.float64) - norm["out_shift"]) / norm["out_scale"]
    r = y - t
    B, n_out = y.shape
    loss = float(np.mean(r * r))
    d = q(2.0 * r / (B * n_out))  # dL/dy
    layers, hs, zs = c["layers"], c["h"], c["z"]
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (d.T @ hs[li], d.sum(axis=0))
        if li > 0:
            d = q((d @ q(W)) * gelu_grad(zs[li - 1]))
    return loss, pack(grads)


def adam_step(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (flat, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------------ warm start
def warm_profile(logP_nn, T_nn, logP_layers, T_iso, T_lo, T_hi):
    """Initial layer temperatures of one atmosphere from the network's profile
    T_nn at log pressures logP_nn: linear in log P between the two nearest
    network points, the end values outside them.  If any of the network's
    values is not finite or outside [T_lo, T_hi], the atmosphere falls back
    to the isothermal start T_iso.  Returns (T, fell_back)."""
    T_nn = np.asarray(T_nn, np.float64)
    if not np.all(np.isfinite(T_nn)) or np.any(T_nn < T_lo) or np.any(T_nn > T_hi):
        return np.full(len(logP_layers), float(T_iso)), True
    lp = np.asarray(logP_nn, np.float64)
    order = np.argsort(lp)
    return np.interp(np.asarray(logP_layers, np.float64), lp[order], T_nn[order]), False
