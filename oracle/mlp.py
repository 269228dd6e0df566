"""Plain numpy reference of the surrogate MLP (test infrastructure only).

Forward pass, mean-squared-error loss on the standardised log mu and its
gradient by the textbook chain rule, in float64.  With ``bf16=True`` the
values the device stores in bfloat16 (inputs, weights, hidden activations,
back-propagated errors) are rounded at the same places, so that the device
kernels and this reference differ only in the order and precision of their
float32 accumulation.  Shares nothing with the library.

Parameter layout: for each layer l, W_l^T as [n_out_l][k_l] rows with the
bias in column n_in_l; k_0 = 32 (7 inputs), k_l = hidden + 8 otherwise.
"""
import numpy as np


def bf16_round(x):
    """Round float64/float32 values to bfloat16 (nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, hidden, n_out):
    shapes = [(hidden, 32, 7), (hidden, hidden + 8, hidden),
              (hidden, hidden + 8, hidden), (n_out, hidden + 8, hidden)]
    out, o = [], 0
    for rows, kp, kin in shapes:
        w = np.asarray(params[o:o + rows * kp], dtype=np.float64).reshape(rows, kp)
        out.append((w, kin))
        o += rows * kp
    assert o == len(params)
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, theta, lo, hi, hidden, n_out, bf16=True):
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params, hidden, n_out)
    x = 2.0 * (theta - lo) / (hi - lo) - 1.0
    acts, zs = [], []
    a = np.concatenate([r(x), np.ones((len(x), 1))], axis=1)   # input + bias
    acts.append(a)
    for li, (w, kin) in enumerate(layers):
        W = r(w[:, :kin + 1])            # weights and bias column
        z = a @ W.T
        if li < 3:
            zs.append(z)
            h = r(silu(z))
            a = np.concatenate([h, np.ones((len(h), 1))], axis=1)
            acts.append(a)
        else:
            y = z
    return y, acts, zs


def mse_grad(params, theta, targets, lo, hi, hidden, n_out, bf16=True,
             magnitude=False):
    """Loss mean((y - t)^2) and its gradient w.r.t. the flat parameters.
    With ``magnitude`` also the sum of the absolute values of the terms
    that make up each gradient element, sum_b |dL/dz_b| |a_b|, the scale
    against which a device's rounding of those terms is bounded."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params, hidden, n_out)
    y, acts, zs = forward(params, theta, lo, hi, hidden, n_out, bf16)
    B = len(theta)
    res = y - targets
    loss = float(np.mean(res ** 2))
    delta = r(2.0 * res / (B * n_out))   # dL/dy, stored in bfloat16
    grads, mags = [None] * 4, [None] * 4
    for li in range(3, -1, -1):
        w, kin = layers[li]
        g = np.zeros_like(w)
        g[:, :kin + 1] = delta.T @ acts[li]
        grads[li] = g
        if magnitude:
            a = np.zeros_like(w)
            a[:, :kin + 1] = np.abs(delta).T @ np.abs(acts[li])
            mags[li] = a
        if li > 0:
            W = r(w[:, :kin])
            delta = r((delta @ W) * dsilu(zs[li - 1]))
    flat = np.concatenate([g.ravel() for g in grads])
    if magnitude:
        return loss, flat, np.concatenate([a.ravel() for a in mags])
    return loss, flat
