"""Pins of the numpy reference of the surrogate network (oracle/mlp.py),
which the device's BF16 forward and backward kernels are checked against:
its gradient against central differences of its own loss through the
forward pass, parameter by parameter (a dropped SiLU' factor, a transposed
weight or a missing bias column fails it); its forward pass against a
network built to compute a known function of one input; its bfloat16
rounding against torch's conversion."""
import numpy as np
import pytest
from scipy.special import expit

from oracle import mlp


H, N = 8, 8          # hidden width and outputs of the tiny network


def tiny(seed):
    g = np.random.Generator(np.random.PCG64(seed))
    shapes = [(H, 32, 7), (H, H + 8, H), (H, H + 8, H), (N, H + 8, H)]
    parts = []
    for rows, kp, kin in shapes:
        w = np.zeros((rows, kp))
        w[:, :kin + 1] = g.uniform(-0.9, 0.9, (rows, kin + 1))  # weights, bias
        parts.append(w.ravel())
    lo = np.array([-0.5, -0.5, -0.5, -0.5, 0.0, 0.8, 0.8])
    hi = np.array([0.5, 0.5, 0.5, 0.5, 25.0, 1.2, 1.2])
    th = g.uniform(lo, hi, (5, 7))
    tg = g.standard_normal((5, N))
    return np.concatenate(parts), th, tg, lo, hi


def test_mse_grad_matches_central_differences():
    p, th, tg, lo, hi = tiny(1)
    loss, g = mlp.mse_grad(p, th, tg, lo, hi, H, N, bf16=False)

    def f(q):
        y, _, _ = mlp.forward(q, th, lo, hi, H, N, bf16=False)
        return float(np.mean((y - tg) ** 2))

    assert loss == pytest.approx(f(p), rel=1e-14)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (f(p + e) - f(p - e)) / (2 * h)
    # central differences of a smooth function: truncation O(h^2), rounding
    # O(eps |f| / h); padding columns of the parameter layout have no effect
    scale = np.abs(g).max()
    assert np.max(np.abs(fd - g)) <= 1e-7 * scale, np.argmax(np.abs(fd - g))
    n_live = int(np.count_nonzero(g))
    assert n_live == H * 8 + 2 * H * (H + 1) + N * (H + 1)


def test_gradient_magnitude_bounds_the_gradient():
    p, th, tg, lo, hi = tiny(2)
    _, g, m = mlp.mse_grad(p, th, tg, lo, hi, H, N, bf16=True, magnitude=True)
    _, g2 = mlp.mse_grad(p, th, tg, lo, hi, H, N, bf16=True)
    assert np.array_equal(g, g2)
    assert np.all(np.abs(g) <= m * (1 + 1e-12))


def test_forward_known_function():
    """A network whose only path carries input i through unit 0 of every
    layer computes silu(silu(silu(x_i))) + c with x_i = 2 (t - lo)/(hi - lo)
    - 1: -1 at the box's low edge, 0 at its centre, 1 at its high edge."""
    lo = np.array([-0.5, -0.5, -0.5, -0.5, 0.0, 0.8, 0.8])
    hi = np.array([0.5, 0.5, 0.5, 0.5, 25.0, 1.2, 1.2])
    for i in range(7):
        ws = [np.zeros((H, 32)), np.zeros((H, H + 8)), np.zeros((H, H + 8)),
              np.zeros((N, H + 8))]
        ws[0][0, i] = 1.0
        ws[1][0, 0] = 1.0
        ws[2][0, 0] = 1.0
        ws[3][3, 0] = 1.0
        ws[3][5, H] = 0.25          # bias of output 5
        p = np.concatenate([w.ravel() for w in ws])
        th = np.tile((lo + hi) / 2, (3, 1))
        th[0, i], th[2, i] = lo[i], hi[i]
        y, _, _ = mlp.forward(p, th, lo, hi, H, N, bf16=False)

        def s(z):
            return z * expit(z)

        for r, x in enumerate((-1.0, 0.0, 1.0)):
            assert y[r, 3] == pytest.approx(s(s(s(x))), rel=1e-13, abs=1e-15)
            assert y[r, 5] == 0.25
            assert np.all(y[r, [0, 1, 2, 4, 6, 7]] == 0.0)


def test_bf16_round_matches_torch():
    import torch
    g = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([g.standard_normal(4000) * 10.0 ** g.integers(-6, 6, 4000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16_round(x)
    assert np.array_equal(got, ref)
    assert got[-5] == 1.0 and got[-4] == 1.0 and got[-3] == 1 + 2 ** -6
