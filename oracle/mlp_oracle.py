"""FP64 CPU oracle of the surrogate network (test infrastructure only).

Plain NumPy, written from the definitions, layer by layer:
  z_l = h_l W_l^T + b_l,  h_{l+1} = tanh(z_l) for hidden layers, y = z_{L-1};
  loss L = sum (y - t)^2 / (batch * outputs);
  back-propagation by the chain rule: dL/dy = 2 (y - t) / (batch * outputs),
  dL/dW_l = dz_l^T h_l, dL/db_l = sum_b dz_l, dz_{l-1} = (dz_l W_l) (1 - h_l^2);
  Adam (Kingma & Ba, 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  p -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).
Parameters are packed layer by layer: W_l [out][in] row-major, then b_l [out].

``bf16=True`` rounds the operands of every matrix product (inputs,
activations, weights, back-propagated errors) to BF16, round to nearest even,
as the GPU network does, and keeps everything else FP64: the GPU result must
then agree to FP32-accumulation level.  Pinned by tests/test_mlp_oracle_pins.py
(finite differences, a hand-derived one-neuron network, Adam's first step).
Shares no code with the HIP library.
"""

from __future__ import annotations

import numpy as np


def n_params(widths) -> int:
    return int(sum(widths[l + 1] * (widths[l] + 1) for l in range(len(widths) - 1)))


def unpack(params, widths):
    """List of (W [out][in], b [out]) views of the packed parameters."""
    out, o = [], 0
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        W = params[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = params[o:o + n_out]
        o += n_out
        out.append((W, b))
    return out


def init_params(widths, seed=0):
    """Glorot-uniform weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        lim = np.sqrt(6.0 / (n_in + n_out))
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)


def round_bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def _op(a, bf16):
    return round_bf16(a) if bf16 else np.asarray(a, dtype=np.float64)


def forward(params, widths, X, bf16=False):
    """Network output and the list of layer inputs h_0 = X, h_1, ..."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    h = np.asarray(X, dtype=np.float64)
    hs = [h]
    for l, (W, b) in enumerate(layers):
        z = _op(h, bf16) @ _op(W, bf16).T + b
        h = z if l == len(layers) - 1 else np.tanh(z)
        hs.append(h)
    return h, hs


def loss_and_grad(params, widths, X, T, bf16=False):
    """Mean squared error and its gradient (packed like the parameters)."""
    params = np.asarray(params, dtype=np.float64)
    layers = unpack(params, widths)
    y, hs = forward(params, widths, X, bf16)
    T = np.asarray(T, dtype=np.float64)
    n = y.size
    loss = float(np.sum((y - T) ** 2) / n)
    dz = 2.0 * (y - T) / n
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gW = _op(dz, bf16).T @ _op(hs[l], bf16)
        gb = dz.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            dz = (_op(dz, bf16) @ _op(W, bf16)) * (1.0 - hs[l] ** 2)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(params, grad, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (k = 1 for the first); returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    p = params - lr * (m / (1.0 - b1 ** k)) / (np.sqrt(v / (1.0 - b2 ** k)) + eps)
    return p, m, v
