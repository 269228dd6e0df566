"""Band skipping in the single-point path: the fold and the adjoint read only
the column bands of R that hold non-zero responses (Sec. II.D: a recoil
electron's light lands within a few resolution widths).  The skipped terms
are exact zeros and no sum changes order, so every result must equal the
full dense read bit for bit; the oracle checks the values themselves."""
import sys

import numpy as np
import pytest

import synth
from problems import config_inputs, gpu_context, inputs, parity_thetas

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both_ways(ctx, th, rows_per_wg=0):
    """(dense, banded) results of the synchronous, gradient, spectrum and
    device entry points."""
    import torch
    dev = torch.device("cuda:0")
    if rows_per_wg:
        ctx.set_fold_tiling(rows_per_wg)
    out = []
    for on in (False, True):
        ctx.set_band_skipping(on)
        tt = torch.tensor(th, dtype=torch.float64, device=dev)
        nl = torch.empty(len(th), dtype=torch.float64, device=dev)
        na = torch.empty(len(th), dtype=torch.float64, device=dev)
        s = torch.cuda.Stream(device=dev)
        ctx.eval_nll_dev(tt, nl, stream=s)
        ctx.eval_nll_dev_noalloc(tt, na, stream=s)
        s.synchronize()
        out.append(dict(nll=ctx.eval_nll(th), grad=ctx.eval_nll_grad(th)[1],
                        mu=ctx.eval_mu(th[:6]), dev=nl.cpu().numpy(),
                        noalloc=na.cpu().numpy()))
    ctx.set_band_skipping(False)
    return out


def assert_same(dense, band, what):
    for k in dense:
        assert np.array_equal(dense[k], band[k]), (what, k,
                                                   np.max(np.abs(dense[k] - band[k])))


def test_band_skipping_config0():
    p = config_inputs(0)
    ctx = gpu_context(p)
    th = parity_thetas(0, 24)
    dense, band = both_ways(ctx, th)
    assert_same(dense, band, "512 x 256")
    o = p["oracle"]
    for i in (0, 5, 20):
        assert abs(band["nll"][i] - o.nll(th[i])) <= 1e-3
    ctx.close()


@pytest.mark.parametrize("n_t,n_reco,rows", [(1000, 1023, 8), (333, 77, 0),
                                              (4096, 2048, 16)])
def test_band_skipping_ragged_and_fine_tiles(n_t, n_reco, rows):
    """Ragged shapes, and 8- or 16-row fold tiles, so that many tiles are
    narrow bands and some are all zero."""
    p = inputs(n_t, n_reco, 64, 200_000, 7301 + n_t, 7302 + n_t)
    ctx = gpu_context(p)
    th = parity_thetas(0, 12)
    log(f"[gpu] band skipping {n_t} x {n_reco}, rows per tile {rows or 'auto'}")
    dense, band = both_ways(ctx, th, rows)
    assert_same(dense, band, f"{n_t} x {n_reco}")
    ctx.close()


def test_band_skipping_zero_rows_and_columns():
    """Rows with no response at all and a block of empty columns."""
    p = inputs(512, 256, 64, 200_000, 7311, 7312)
    R = p["R"].copy()
    R[100:180] = 0.0
    R[:, 200:240] = 0.0
    import paper_2607_00488_amd as nr
    ctx = nr.Context(0)
    ctx.set_sources(p["src"], 512)
    ctx.set_response(R, n_sig=p["n_sig"])
    ctx.set_data(p["n"], p["b"])
    th = parity_thetas(0, 8)
    dense, band = both_ways(ctx, th, 8)
    assert_same(dense, band, "zero rows and columns")
    ctx.close()


def test_band_skipping_needs_a_response():
    import paper_2607_00488_amd as nr
    ctx = nr.Context(0)
    with pytest.raises(nr.NrError) as e:
        ctx.set_band_skipping(True)
    assert e.value.code == nr.NR_ESTATE
    ctx.close()


@pytest.mark.parametrize("cfg", ["0", "1", "2", "3"])
def test_band_skipping_batched(monkeypatch, cfg):
    """The batched forms under band skipping: each GEMM tile reduces only
    over the K-steps where its response entries are not all zero.  With the
    tile configuration pinned, the likelihood, gradient and spectra equal
    the dense ones bit for bit; a grouped launch mixes a banded and a dense
    analysis."""
    monkeypatch.setenv("NR_GEMM_CONFIG", cfg)
    import torch
    import paper_2607_00488_amd as nr
    p = inputs(2048, 1024, 64, 400_000, 7321, 7322)
    q = config_inputs(0)
    ctx, cq = gpu_context(p), gpu_context(q)
    th = parity_thetas(0, 40)
    log(f"[gpu] batched band skipping, tile configuration {cfg}")
    res = []
    for on in (False, True):
        ctx.set_band_skipping(on)
        nl, gr = ctx.eval_nll_grad_batched(th)
        res.append((ctx.eval_nll_batched(th), nl, gr, ctx.eval_mu_batched(th[:5])))
    for a, b in zip(*res):
        assert np.array_equal(a, b), np.max(np.abs(a - b))
    # grouped: the banded analysis beside a dense one, device pointers
    dev = torch.device("cuda:0")
    tt = [torch.tensor(th, dtype=torch.float64, device=dev) for _ in range(2)]
    out = [torch.empty(len(th), dtype=torch.float64, device=dev) for _ in range(2)]
    nr.eval_nll_multi_dev([ctx, cq], tt, out)
    torch.cuda.synchronize()
    assert np.array_equal(out[0].cpu().numpy(), res[0][0])
    assert np.array_equal(out[1].cpu().numpy(), cq.eval_nll_batched(th))
    o = p["oracle"]
    for i in (0, 17, 39):
        assert abs(res[1][0][i] - o.nll(th[i])) <= 1e-3
    ctx.close()
    cq.close()
