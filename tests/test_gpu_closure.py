"""The HIP single-point path on the paper's closure problem (Sec. VI.A):
fed the binned SM response of a 7Be line, it must reproduce the oracle's
reweighted prediction, and therefore close against the direct continuum
fold as the paper reports."""
import numpy as np
import pytest

from oracle import closure

pytestmark = pytest.mark.gpu

NSI = np.array([0.1, 0.1, 0, 0, 0, 1, 1.0])
MM = np.array([0, 0, 0, 0, 2.8 ** 2, 1, 1.0])


@pytest.mark.parametrize("n_t", [25, 200])
def test_closure_on_gpu(n_t):
    import paper_2607_00488_amd as nr
    edges = np.arange(0.0, 451.0)
    Rj, pee, tmax = closure.binned_response(n_t, edges)
    m = Rj.sum(1)
    Rc = (Rj / m[:, None]).astype(np.float32)
    ctx = nr.Context(0)
    ctx.set_sources([dict(kind=0, E=[closure.BE7], weight=[1.0], p_ee=[pee],
                          group=0)], n_t, 0.0, tmax)
    ctx.set_response(Rc, m=m)
    nb = len(edges) - 1
    ctx.set_data(np.ones(nb), np.zeros(nb))
    sel = (edges[:-1] >= 50) & (edges[1:] <= 400)
    for th in (NSI, MM):
        mu = ctx.eval_mu(th)[0]
        # the same reweighting with the same FP32 response, in FP64
        w = closure.spectrum(closure.Oracle(), closure.BE7,
                             (np.arange(n_t) + 0.5) * tmax / n_t, th, pee)
        w /= closure.spectrum(closure.Oracle(), closure.BE7,
                              (np.arange(n_t) + 0.5) * tmax / n_t,
                              np.array([0, 0, 0, 0, 0, 1, 1.0]), pee)
        ref = ((m * w)[:, None] * Rc.astype(np.float64)).sum(0)
        assert np.allclose(mu, ref, rtol=1e-10, atol=1e-12 * ref.max())
        direct, _ = closure.predictions(th, n_t, edges)
        integ = abs(mu[sel].sum() - direct[sel].sum()) / direct[sel].sum()
        _, integ_ref = closure.closure(th, n_t)
        # FP32 storage of the conditional response adds < 1e-7
        assert integ == pytest.approx(integ_ref, rel=0.02, abs=2e-7)
    ctx.close()
