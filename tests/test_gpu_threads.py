"""Distinct contexts driven from different threads at the same time: each
thread runs the plain, batched (with a first-call tuning of its shape
class into a shared cache file) and template forms on its own context;
results agree with the same calls made from one thread and with the
oracle, and the cache file holds both shape classes."""
import json
import sys
import threading

import numpy as np
import pytest

import synth
from problems import gpu_context, inputs

pytestmark = pytest.mark.gpu

SHAPES = [(300, 77, 40, 131), (512, 256, 32, 200)]  # n_t, n_reco, n_e, points


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_forms(ctx, th):
    return (ctx.eval_nll(th[:9]), ctx.eval_nll_batched(th),
            ctx.eval_nll_grad_batched(th[:33]), ctx.eval_nll_templates(th, grad=True))


def test_distinct_contexts_from_two_threads(tmp_path, monkeypatch):
    monkeypatch.delenv("NR_GEMM_CONFIG", raising=False)
    probs, ctxs, ths = [], [], []
    for d, (n_t, n_reco, n_e, P) in enumerate(SHAPES):
        p = inputs(n_t, n_reco, n_e, 100_000, 810 + d, 820 + d)
        probs.append(p)
        ctxs.append(gpu_context(p))
        ths.append(synth.theta_prior(P, 830 + d))
    # one thread first (every buffer sized, tuned into a cache of its own)
    monkeypatch.setenv("NR_AUTOTUNE_CACHE", str(tmp_path / "serial.json"))
    ref = [run_forms(c, th) for c, th in zip(ctxs, ths)]
    # then both contexts at once, tuning again into a fresh shared cache
    cache = tmp_path / "shared.json"
    monkeypatch.setenv("NR_AUTOTUNE_CACHE", str(cache))
    log(f"[gpu] two threads, contexts {SHAPES}")
    got, errs = [None, None], []

    def work(d):
        try:
            for _ in range(3):
                got[d] = run_forms(ctxs[d], ths[d])
        except Exception as e:  # re-raised on the main thread
            errs.append((d, e))

    ts = [threading.Thread(target=work, args=(d,)) for d in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in ts)
    assert not errs, errs
    for d in range(2):
        o = probs[d]["oracle"]
        plain, bat, (bg_n, bg_g), (tp_n, tp_g) = got[d]
        rplain, rbat, (rbg_n, rbg_g), (rtp_n, rtp_g) = ref[d]
        # the plain and template forms do not depend on the tuning: bitwise
        assert np.array_equal(plain, rplain) and np.array_equal(tp_n, rtp_n)
        assert np.array_equal(tp_g, rtp_g)
        # the batched forms may run another tile configuration
        assert np.max(np.abs(bat - rbat)) <= 1e-9 * np.abs(rbat).max()
        assert np.max(np.abs(bg_n - rbg_n)) <= 1e-9 * np.abs(rbg_n).max()
        assert np.max(np.abs(bg_g - rbg_g)) <= 1e-7 * np.abs(rbg_g).max()
        for i in (0, len(ths[d]) // 2, len(ths[d]) - 1):
            assert abs(bat[i] - o.nll(ths[d][i])) <= 1e-3, (d, i)
    saved = json.loads(cache.read_text())
    kinds = sorted(k.split("|")[0] for k in saved)
    assert kinds == ["grad", "grad", "nll", "nll"], saved
    for c in ctxs:
        c.close()
