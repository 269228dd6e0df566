"""Learned surrogate of the expected spectrum, with a fallback to the exact
method.

An MLP maps theta (7 parameters, normalised over a training box) through
three hidden SiLU layers to the standardised log mu_j of every observed
bin.  Training data come from the batched method; training and inference
run in the library's BF16 matrix-core kernels (forward, backward, Adam, and
an inference kernel that fuses the output layer with exp and the Poisson
deviance).  At evaluation time a fraction of every batch is re-evaluated
exactly; if any spot check misses by more than ``tol`` in -2lnL, the whole
batch is re-evaluated exactly, and points outside the training box always
are.  This module only marshals buffers (torch) and calls the library.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import (Context, eval_nll_multi_dev, nr_eval_mu_batched_dev,
               nr_mlp_create, nr_mlp_destroy, nr_mlp_get_grads,
               nr_mlp_get_params, nr_mlp_nll_dev, nr_mlp_num_params,
               nr_mlp_set_box, nr_mlp_set_output_norm, nr_mlp_set_params,
               nr_mlp_targets_dev, nr_mlp_train_step_dev, nr_mlp_logmu_dev)


def layer_shapes(hidden: int, n_out: int):
    """(rows, padded input width, true input width) of W^T per layer."""
    return [(hidden, 32, 7), (hidden, hidden + 8, hidden),
            (hidden, hidden + 8, hidden), (n_out, hidden + 8, hidden)]


def init_params(hidden: int, n_out: int, seed: int, out_scale: float = 0.1):
    """He-uniform weights, zero biases, zero padding columns."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shapes = layer_shapes(hidden, n_out)
    for li, (rows, kp, kin) in enumerate(shapes):
        w = np.zeros((rows, kp), dtype=np.float32)
        a = math.sqrt(6.0 / kin)
        if li == len(shapes) - 1:
            a *= out_scale
        w[:, :kin] = g.uniform(-a, a, (rows, kin))
        parts.append(w.ravel())
    return np.concatenate(parts)


class Surrogate:
    def __init__(self, n_out: int, lo, hi, hidden: int = 256,
                 device: int = 0, seed: int = 4001):
        self.h = nr_mlp_create(device, hidden, n_out)
        self.n_out, self.hidden, self.device = n_out, hidden, device
        self.dev = torch.device(f"cuda:{device}")
        nr_mlp_set_params(self.h, init_params(hidden, n_out, seed))
        nr_mlp_set_box(self.h, lo, hi)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self._bufs = {}

    def close(self):
        if self.h is not None:
            nr_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- data
    def sample_box(self, n: int, seed: int) -> torch.Tensor:
        g = np.random.Generator(np.random.PCG64(seed))
        th = g.uniform(self.lo, self.hi, (n, 7))
        return torch.tensor(th, dtype=torch.float64, device=self.dev)

    def make_targets(self, ctx: Context, theta: torch.Tensor,
                     chunk: int = 8192, set_norm: bool = True):
        """Expected spectra from the batched method, as standardised log mu
        (FP32 [P, n_out]).  The per-bin mean and spread of log mu are taken
        from the first chunk."""
        P = theta.shape[0]
        stream = torch.cuda.current_stream(self.dev)
        t = torch.empty(P, self.n_out, dtype=torch.float32, device=self.dev)
        mu = torch.empty(min(chunk, P), self.n_out, dtype=torch.float64,
                         device=self.dev)
        for c0 in range(0, P, chunk):
            n = min(chunk, P - c0)
            th = theta[c0:c0 + n].contiguous()
            nr_eval_mu_batched_dev(ctx.h, th.data_ptr(), n, mu.data_ptr(),
                                   stream.cuda_stream)
            if c0 == 0 and set_norm:
                lm = np.log(np.maximum(mu[:n].cpu().numpy(), 1e-300))
                mean = lm.mean(0).astype(np.float32)
                std = np.maximum(lm.std(0), 1e-3).astype(np.float32)
                nr_mlp_set_output_norm(self.h, mean, std)
            nr_mlp_targets_dev(self.h, mu.data_ptr(), n, t[c0:c0 + n].data_ptr(),
                               stream.cuda_stream)
        torch.cuda.synchronize(self.dev)
        return t

    # ---------------------------------------------------------- training
    def train(self, theta: torch.Tensor, targets: torch.Tensor,
              epochs: int = 100, batch: int = 4096, lr_max: float = 2e-3,
              lr_min: float = 2e-5, seed: int = 4003, log_every: int = 0,
              time_limit: float | None = None):
        P = theta.shape[0]
        steps_per_epoch = P // batch
        total = epochs * steps_per_epoch
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(seed)
        stream = torch.cuda.current_stream(self.dev)
        losses = []
        t0 = time.time()
        step = 0
        for ep in range(epochs):
            perm = torch.randperm(P, device=self.dev, generator=gen)
            for b in range(steps_per_epoch):
                idx = perm[b * batch:(b + 1) * batch]
                th = theta.index_select(0, idx)
                tg = targets.index_select(0, idx)
                lr = lr_min + 0.5 * (lr_max - lr_min) * (
                    1 + math.cos(math.pi * step / max(1, total)))
                want = log_every and (step % log_every == 0)
                v = nr_mlp_train_step_dev(self.h, th.data_ptr(), tg.data_ptr(),
                                          batch, lr, bool(want),
                                          stream.cuda_stream)
                if want:
                    losses.append((step, v))
                step += 1
            if time_limit is not None and time.time() - t0 > time_limit:
                break
        torch.cuda.synchronize(self.dev)
        return dict(steps=step, epochs=ep + 1, seconds=time.time() - t0,
                    losses=losses)

    def grads(self):
        return nr_mlp_get_grads(self.h)

    def params(self):
        return nr_mlp_get_params(self.h)

    def set_params(self, p):
        nr_mlp_set_params(self.h, p)

    def save(self, path):
        np.savez(path, params=self.params(), lo=self.lo, hi=self.hi)

    # --------------------------------------------------------- inference
    def logmu(self, theta: torch.Tensor) -> torch.Tensor:
        B = theta.shape[0]
        out = torch.empty(B, self.n_out, dtype=torch.float32, device=self.dev)
        nr_mlp_logmu_dev(self.h, theta.data_ptr(), B, out.data_ptr(),
                         torch.cuda.current_stream(self.dev).cuda_stream)
        return out

    def nll(self, ctx: Context, theta: torch.Tensor):
        B = theta.shape[0]
        nll = torch.empty(B, dtype=torch.float64, device=self.dev)
        outside = torch.empty(B, dtype=torch.int32, device=self.dev)
        nr_mlp_nll_dev(self.h, ctx.h, theta.data_ptr(), B, nll.data_ptr(),
                       outside.data_ptr(),
                       torch.cuda.current_stream(self.dev).cuda_stream)
        return nll, outside

    def _buf(self, key, shape, dtype):
        b = self._bufs.get(key)
        if b is None or b.shape != shape:
            b = torch.empty(shape, dtype=dtype, device=self.dev)
            self._bufs[key] = b
        return b

    def _exact(self, ctx: Context, theta: torch.Tensor, key: str):
        """Exact -2lnL through the batched method, on buffers that stay put
        so the library's cached graph is replayed."""
        n = theta.shape[0]
        th = self._buf(key + "_th", (n, 7), torch.float64)
        out = self._buf(key + "_nll", (n,), torch.float64)
        th.copy_(theta)
        eval_nll_multi_dev([ctx], [th], [out],
                           stream=torch.cuda.current_stream(self.dev))
        return out

    def evaluate(self, ctx: Context, theta: torch.Tensor, tol: float = 0.1,
                 spot_frac: float = 0.01, min_spot: int = 64,
                 seed: int = 0, force_fail: bool = False):
        """-2lnL for a batch with spot checks and fallback.  Returns
        (nll [B], info).  ``force_fail`` perturbs the surrogate values of
        the spot-checked points (test hook for the fallback)."""
        B = theta.shape[0]
        nll, outside = self.nll(ctx, theta)
        n_spot = min(B, max(min_spot, int(math.ceil(spot_frac * B))))
        g = torch.Generator(device=self.dev)
        g.manual_seed(seed)
        idx = torch.randperm(B, device=self.dev, generator=g)[:n_spot]
        exact_spot = self._exact(ctx, theta.index_select(0, idx), "spot")
        sur_spot = nll.index_select(0, idx)
        if force_fail:
            sur_spot = sur_spot + 10.0 * tol
        inbox = outside.index_select(0, idx) == 0
        dev_spot = (sur_spot - exact_spot).abs()
        worst = float(dev_spot[inbox].max().item()) if bool(inbox.any()) else 0.0
        failed = bool((dev_spot > tol)[inbox].any().item()) or force_fail
        if failed:
            out = self._exact(ctx, theta, "all").clone()
            return out, dict(fallback="batch", fallback_fraction=1.0,
                             spot=n_spot, spot_worst=worst)
        out = nll.clone()
        out[idx] = exact_spot
        oi = torch.nonzero(outside != 0).flatten()
        if oi.numel():
            out[oi] = self._exact(ctx, theta.index_select(0, oi), "out")
        return out, dict(fallback="none" if oi.numel() == 0 else "outside",
                         fallback_fraction=float(oi.numel()) / B,
                         spot=n_spot, spot_worst=worst)
