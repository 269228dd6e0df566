"""MI355X-native spectrum-reweighting likelihood (arXiv:2607.00488).

Thin ctypes binding over ``libnureweight.so``.  The functions ``nr_*`` carry
the names and arguments of the C ABI declared in ``include/nureweight.h``;
:class:`Context` wraps them for numpy and torch callers.  Every step of the
likelihood runs in the library's HIP kernels; this module only marshals
arguments.  Importing works without a GPU; any call that needs the library
raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._build import LIB as _LIB_PATH

NR_NTHETA = 7
NR_OK, NR_EINVAL, NR_ESTATE, NR_EHIP, NR_ENOMEM = 0, -1, -2, -3, -4
NR_PROBE_CACHED, NR_PROBE_ALTERNATE = 1, 2
NR_NOALLOC_WORKSPACE_BYTES = 16 << 20

# Exported symbols of include/nureweight.h.
EXPORTS = (
    "nr_create", "nr_destroy", "nr_set_sources", "nr_set_response",
    "nr_set_data", "nr_eval_nll", "nr_eval_nll_grad", "nr_eval_mu",
    "nr_eval_nll_dev", "nr_eval_nll_dev_noalloc", "nr_set_band_skipping", "nr_eval_weights", "nr_get_reference", "nr_stream",
    "nr_set_mc_events", "nr_eval_ess", "nr_set_components", "nr_num_theta",
    "nr_time_stage", "nr_set_fold_tiling", "nr_last_error",
    "nr_eval_nll_batched", "nr_eval_nll_grad_batched", "nr_eval_mu_batched",
    "nr_eval_nll_multi", "nr_eval_nll_multi_dev",
    "nr_mlp_create", "nr_mlp_destroy", "nr_mlp_num_params", "nr_mlp_set_params",
    "nr_mlp_get_params", "nr_mlp_get_grads", "nr_mlp_set_box",
    "nr_mlp_set_output_norm", "nr_mlp_targets_dev", "nr_mlp_train_step_dev",
    "nr_mlp_logmu_dev", "nr_mlp_nll_dev", "nr_eval_mu_batched_dev",
    "nr_build_templates", "nr_eval_nll_templates", "nr_eval_mu_templates",
    "nr_eval_nll_templates_dev", "nr_probe_mfma_f64", "nr_probe_hbm_read",
    "nr_probe_read",
)


class NrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nureweight error {code}: {msg}")
        self.code = code


class nr_source(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int),
                ("E", C.POINTER(C.c_double)),
                ("weight", C.POINTER(C.c_double)),
                ("p_ee", C.POINTER(C.c_double)), ("group", C.c_int)]


class nr_physics(C.Structure):
    _fields_ = [("me", C.c_double), ("gf", C.c_double), ("sw2", C.c_double),
                ("alpha_em", C.c_double), ("tau_frac", C.c_double)]


class nr_components(C.Structure):
    _fields_ = [("n_comp", C.c_int), ("comp_of_source", C.POINTER(C.c_int)),
                ("hist", C.POINTER(C.c_float)),
                ("comp_mask", C.POINTER(C.c_double)),
                ("scale", C.POINTER(C.c_double)),
                ("rate_sm", C.POINTER(C.c_double)), ("n_bkg", C.c_int),
                ("bkg_pdf", C.POINTER(C.c_double)),
                ("bkg_rate", C.POINTER(C.c_double)),
                ("mask", C.POINTER(C.c_double)), ("exposure", C.c_double)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load the built library; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: when PyTorch is importable, let its
    # bundled runtime be the one the library binds to (same soname).
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is not built; run __graft_entry__.build() or "
            "python -m paper_2607_00488_amd._build")
    L = C.CDLL(_LIB_PATH)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    pD = C.POINTER(C.c_double)
    L.nr_create.argtypes = [I, C.POINTER(P)]
    L.nr_destroy.argtypes = [P]
    L.nr_destroy.restype = None
    L.nr_set_sources.argtypes = [P, C.POINTER(nr_source), I, I, D, D,
                                 C.POINTER(nr_physics)]
    L.nr_set_response.argtypes = [P, C.POINTER(C.c_float), I, I, pD, D]
    L.nr_set_data.argtypes = [P, pD, pD, I, pD, pD]
    L.nr_eval_nll.argtypes = [P, pD, I, pD]
    L.nr_eval_nll_grad.argtypes = [P, pD, I, pD, pD]
    L.nr_eval_mu.argtypes = [P, pD, I, pD]
    L.nr_eval_weights.argtypes = [P, pD, I, pD]
    L.nr_set_mc_events.argtypes = [P, pD, I]
    L.nr_set_components.argtypes = [P, C.POINTER(nr_components), I]
    L.nr_num_theta.argtypes = [P]
    L.nr_eval_ess.argtypes = [P, pD, I, pD]
    L.nr_eval_nll_dev.argtypes = [P, P, I, P, P, P]
    L.nr_eval_nll_dev_noalloc.argtypes = [P, P, I, P, P, P]
    L.nr_set_band_skipping.argtypes = [P, I]
    L.nr_get_reference.argtypes = [P, pD, pD]
    L.nr_stream.argtypes = [P]
    L.nr_stream.restype = P
    L.nr_time_stage.argtypes = [P, I, I, pD]
    L.nr_set_fold_tiling.argtypes = [P, I, I]
    L.nr_last_error.restype = C.c_char_p
    L.nr_eval_nll_batched.argtypes = [P, pD, I, pD]
    L.nr_eval_nll_grad_batched.argtypes = [P, pD, I, pD, pD]
    L.nr_eval_mu_batched.argtypes = [P, pD, I, pD]
    L.nr_eval_nll_multi.argtypes = [C.POINTER(P), I, C.POINTER(pD),
                                    C.POINTER(I), C.POINTER(pD)]
    L.nr_eval_nll_multi_dev.argtypes = [C.POINTER(P), I, C.POINTER(P),
                                        C.POINTER(I), C.POINTER(P),
                                        C.POINTER(P), P]
    pF = C.POINTER(C.c_float)
    L.nr_mlp_create.argtypes = [I, I, I, C.POINTER(P)]
    L.nr_mlp_destroy.argtypes = [P]
    L.nr_mlp_destroy.restype = None
    L.nr_mlp_num_params.argtypes = [P]
    L.nr_mlp_num_params.restype = C.c_long
    L.nr_mlp_set_params.argtypes = [P, pF, C.c_long]
    L.nr_mlp_get_params.argtypes = [P, pF, C.c_long]
    L.nr_mlp_get_grads.argtypes = [P, pF, C.c_long]
    L.nr_mlp_set_box.argtypes = [P, pD, pD]
    L.nr_mlp_set_output_norm.argtypes = [P, pF, pF]
    L.nr_mlp_targets_dev.argtypes = [P, P, I, P, P]
    L.nr_mlp_train_step_dev.argtypes = [P, P, P, I, C.c_float, pD, P]
    L.nr_mlp_logmu_dev.argtypes = [P, P, I, P, P]
    L.nr_mlp_nll_dev.argtypes = [P, P, P, I, P, P, P]
    L.nr_eval_mu_batched_dev.argtypes = [P, P, I, P, P]
    L.nr_build_templates.argtypes = [P]
    L.nr_eval_nll_templates.argtypes = [P, pD, I, pD, pD]
    L.nr_eval_mu_templates.argtypes = [P, pD, I, pD]
    L.nr_eval_nll_templates_dev.argtypes = [P, P, I, P, P, P]
    L.nr_probe_mfma_f64.argtypes = [I, I, I, pD]
    L.nr_probe_hbm_read.argtypes = [I, C.c_longlong, I, pD]
    L.nr_probe_read.argtypes = [I, C.c_longlong, I, I, pD]
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("nr_destroy", "nr_stream", "nr_last_error",
                        "nr_mlp_destroy", "nr_mlp_num_params"):
            fn.restype = C.c_int
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise NrError(rc, load().nr_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ----------------------------------------------------------- C-ABI names
def nr_create(device: int = 0):
    h = C.c_void_p()
    _check(load().nr_create(int(device), C.byref(h)))
    return h


def nr_destroy(h):
    load().nr_destroy(h)


def nr_set_sources(h, sources, n_t, t_lo=0.0, t_hi=16.0, physics=None):
    keep = []
    arr = (nr_source * len(sources))()
    for i, s in enumerate(sources):
        E, w, p = (_f64(s["E"]), _f64(s["weight"]), _f64(s["p_ee"]))
        keep += [E, w, p]
        arr[i] = nr_source(int(s["kind"]), len(E), _dp(E), _dp(w), _dp(p),
                           int(s["group"]))
    ph = None
    if physics is not None:
        ph = C.byref(nr_physics(*[float(x) for x in physics]))
    _check(load().nr_set_sources(h, arr, len(sources), int(n_t), float(t_lo),
                                 float(t_hi), ph))


def nr_set_response(h, R, m=None, n_sig=1.0e4):
    R = np.ascontiguousarray(R, dtype=np.float32)
    pm = None
    if m is not None:
        m = _f64(m)
        pm = _dp(m)
    _check(load().nr_set_response(h, R.ctypes.data_as(C.POINTER(C.c_float)),
                                  R.shape[0], R.shape[1], pm, float(n_sig)))


def nr_num_theta(h) -> int:
    return int(load().nr_num_theta(h))


def nr_set_data(h, n, b, pull_mean=None, pull_sigma=None):
    n = _f64(n)
    pb = None
    if b is not None:
        b = _f64(b)
        pb = _dp(b)
    pm = ps = None
    if pull_mean is not None:
        k = nr_num_theta(h)
        pmv, psv = _f64(pull_mean), _f64(pull_sigma)
        if pmv.shape != (k,) or psv.shape != (k,):
            raise ValueError(f"pulls need {k} entries each")
        pm, ps = _dp(pmv), _dp(psv)
    _check(load().nr_set_data(h, _dp(n), pb, len(n), pm, ps))


def nr_set_components(h, comp_of_source, hist, scale, rate_sm, bkg_pdf=None,
                      bkg_rate=None, comp_mask=None, mask=None, exposure=1.0):
    """hist: [K, n_t, n_reco] float32; bkg_pdf: [B, n_reco]."""
    hist = np.ascontiguousarray(hist, dtype=np.float32)
    K, n_t, n_reco = hist.shape
    cs = np.ascontiguousarray(comp_of_source, dtype=np.int32)
    sc, rs = _f64(scale), _f64(rate_sm)
    if sc.shape != (K,) or rs.shape != (K,):
        raise ValueError("scale and rate_sm need one entry per component")
    B = 0 if bkg_pdf is None else int(np.shape(bkg_pdf)[0])
    keep = [hist, cs, sc, rs]
    st = nr_components()
    st.n_comp = K
    st.comp_of_source = cs.ctypes.data_as(C.POINTER(C.c_int))
    st.hist = hist.ctypes.data_as(C.POINTER(C.c_float))
    st.scale, st.rate_sm = _dp(sc), _dp(rs)
    st.n_bkg = B
    if B:
        bp, br = _f64(bkg_pdf), _f64(bkg_rate)
        if bp.shape != (B, n_reco) or br.shape != (B,):
            raise ValueError("bkg_pdf is [B, n_reco], bkg_rate [B]")
        keep += [bp, br]
        st.bkg_pdf, st.bkg_rate = _dp(bp), _dp(br)
    if comp_mask is not None:
        cm = _f64(comp_mask)
        if cm.shape != (K, n_reco):
            raise ValueError("comp_mask is [K, n_reco]")
        keep.append(cm)
        st.comp_mask = _dp(cm)
    if mask is not None:
        m = _f64(mask)
        if m.shape != (n_reco,):
            raise ValueError("mask is [n_reco]")
        keep.append(m)
        st.mask = _dp(m)
    st.exposure = float(exposure)
    _check(load().nr_set_components(h, C.byref(st), n_reco))
    del keep


def nr_eval_nll(h, theta):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty(th.shape[0])
    _check(load().nr_eval_nll(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_eval_nll_grad(h, theta):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty(th.shape[0])
    g = np.empty((th.shape[0], NR_NTHETA))
    _check(load().nr_eval_nll_grad(h, _dp(th), th.shape[0], _dp(out), _dp(g)))
    return out, g


def nr_eval_mu(h, theta, n_reco):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty((th.shape[0], n_reco))
    _check(load().nr_eval_mu(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_set_mc_events(h, n_events):
    ev = _f64(n_events)
    _check(load().nr_set_mc_events(h, _dp(ev), int(ev.shape[0])))


def nr_eval_ess(h, theta, n_reco):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty((th.shape[0], n_reco))
    _check(load().nr_eval_ess(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_eval_weights(h, theta, n_t):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty((th.shape[0], n_t))
    _check(load().nr_eval_weights(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_eval_nll_dev(h, d_theta_ptr, n_pts, d_nll_ptr, d_grad_ptr=None,
                    stream_ptr=None):
    _check(load().nr_eval_nll_dev(h, C.c_void_p(d_theta_ptr), int(n_pts),
                                  C.c_void_p(d_nll_ptr),
                                  C.c_void_p(d_grad_ptr or 0),
                                  C.c_void_p(stream_ptr or 0)))


def nr_set_band_skipping(h, on):
    _check(load().nr_set_band_skipping(h, 1 if on else 0))


def nr_eval_nll_dev_noalloc(h, d_theta_ptr, n_pts, d_nll_ptr, d_grad_ptr=None,
                            stream_ptr=None):
    _check(load().nr_eval_nll_dev_noalloc(h, C.c_void_p(d_theta_ptr), int(n_pts),
                                          C.c_void_p(d_nll_ptr),
                                          C.c_void_p(d_grad_ptr or 0),
                                          C.c_void_p(stream_ptr or 0)))


def nr_build_templates(h):
    _check(load().nr_build_templates(h))


def nr_eval_nll_templates(h, theta, grad=False):
    nt = nr_num_theta(h)
    th = _f64(theta, (-1, nt))
    out = np.empty(th.shape[0])
    g = np.empty((th.shape[0], nt)) if grad else None
    _check(load().nr_eval_nll_templates(h, _dp(th), th.shape[0], _dp(out),
                                        _dp(g) if grad else None))
    return (out, g) if grad else out


def nr_eval_mu_templates(h, theta, n_reco):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty((th.shape[0], n_reco))
    _check(load().nr_eval_mu_templates(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_eval_nll_templates_dev(h, d_theta_ptr, n_pts, d_nll_ptr, d_grad_ptr=None,
                              stream_ptr=None):
    _check(load().nr_eval_nll_templates_dev(h, C.c_void_p(d_theta_ptr), int(n_pts),
                                            C.c_void_p(d_nll_ptr),
                                            C.c_void_p(d_grad_ptr or 0),
                                            C.c_void_p(stream_ptr or 0)))


def nr_probe_mfma_f64(device=0, blocks=8192, iters=16):
    """Sustained FP64 matrix-core TFLOP/s of the device (register-only
    stream of independent MFMA instructions)."""
    out = np.zeros(1)
    rc = load().nr_probe_mfma_f64(int(device), int(blocks), int(iters), _dp(out))
    if rc != 0:
        raise NrError(rc, "nr_probe_mfma_f64 failed")
    return float(out[0])


def nr_probe_hbm_read(device=0, nbytes=2 << 30, reps=10):
    """Sustained HBM read GB/s of the device (streaming sum over a buffer
    much larger than the caches)."""
    out = np.zeros(1)
    rc = load().nr_probe_hbm_read(int(device), int(nbytes), int(reps), _dp(out))
    if rc != 0:
        raise NrError(rc, "nr_probe_hbm_read failed")
    return float(out[0])


def nr_probe_read(device=0, nbytes=2 << 30, reps=10, flags=0):
    """Read GB/s of the same streaming sum with ordinary loads
    (NR_PROBE_CACHED) and/or passes alternating in direction
    (NR_PROBE_ALTERNATE); flags=0 is nr_probe_hbm_read."""
    out = np.zeros(1)
    rc = load().nr_probe_read(int(device), int(nbytes), int(reps), int(flags), _dp(out))
    if rc != 0:
        raise NrError(rc, "nr_probe_read failed")
    return float(out[0])


def nr_get_reference(h, n_t):
    s = np.empty(n_t)
    m = np.empty(n_t)
    _check(load().nr_get_reference(h, _dp(s), _dp(m)))
    return s, m


def nr_stream(h):
    return load().nr_stream(h)


def nr_time_stage(h, stage, iters):
    v = C.c_double()
    _check(load().nr_time_stage(h, int(stage), int(iters), C.byref(v)))
    return v.value


def nr_set_fold_tiling(h, rows_per_wg=0, use_graph=-1):
    _check(load().nr_set_fold_tiling(h, int(rows_per_wg), int(use_graph)))


def nr_eval_nll_batched(h, theta):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty(th.shape[0])
    _check(load().nr_eval_nll_batched(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_eval_nll_grad_batched(h, theta):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty(th.shape[0])
    g = np.empty((th.shape[0], NR_NTHETA))
    _check(load().nr_eval_nll_grad_batched(h, _dp(th), th.shape[0], _dp(out),
                                           _dp(g)))
    return out, g


def nr_eval_mu_batched(h, theta, n_reco):
    th = _f64(theta, (-1, nr_num_theta(h)))
    out = np.empty((th.shape[0], n_reco))
    _check(load().nr_eval_mu_batched(h, _dp(th), th.shape[0], _dp(out)))
    return out


def nr_eval_nll_multi(handles, thetas):
    n = len(handles)
    ths = [_f64(t, (-1, nr_num_theta(h))) for h, t in zip(handles, thetas)]
    outs = [np.empty(t.shape[0]) for t in ths]
    H = (C.c_void_p * n)(*[h.value if hasattr(h, "value") else h
                            for h in handles])
    pD = C.POINTER(C.c_double)
    TH = (pD * n)(*[_dp(t) for t in ths])
    NP = (C.c_int * n)(*[t.shape[0] for t in ths])
    OUT = (pD * n)(*[_dp(o) for o in outs])
    _check(load().nr_eval_nll_multi(H, n, TH, NP, OUT))
    return outs


def nr_eval_nll_multi_dev(handles, theta_ptrs, n_pts, nll_ptrs,
                          grad_ptrs=None, stream_ptr=None):
    n = len(handles)
    H = (C.c_void_p * n)(*[h.value if hasattr(h, "value") else h
                            for h in handles])
    TH = (C.c_void_p * n)(*theta_ptrs)
    NP = (C.c_int * n)(*[int(x) for x in n_pts])
    OUT = (C.c_void_p * n)(*nll_ptrs)
    GR = None if grad_ptrs is None else (C.c_void_p * n)(*grad_ptrs)
    _check(load().nr_eval_nll_multi_dev(H, n, TH, NP, OUT, GR,
                                        C.c_void_p(stream_ptr or 0)))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def nr_mlp_create(device, hidden, n_out):
    h = C.c_void_p()
    _check(load().nr_mlp_create(int(device), int(hidden), int(n_out),
                                C.byref(h)))
    return h


def nr_mlp_destroy(h):
    load().nr_mlp_destroy(h)


def nr_mlp_num_params(h):
    return int(load().nr_mlp_num_params(h))


def nr_mlp_set_params(h, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(load().nr_mlp_set_params(h, _fp(p), p.size))


def nr_mlp_get_params(h):
    p = np.empty(nr_mlp_num_params(h), dtype=np.float32)
    _check(load().nr_mlp_get_params(h, _fp(p), p.size))
    return p


def nr_mlp_get_grads(h):
    p = np.empty(nr_mlp_num_params(h), dtype=np.float32)
    _check(load().nr_mlp_get_grads(h, _fp(p), p.size))
    return p


def nr_mlp_set_box(h, lo, hi):
    lo, hi = _f64(lo), _f64(hi)
    _check(load().nr_mlp_set_box(h, _dp(lo), _dp(hi)))


def nr_mlp_set_output_norm(h, mean, std):
    m = np.ascontiguousarray(mean, dtype=np.float32)
    s_ = np.ascontiguousarray(std, dtype=np.float32)
    _check(load().nr_mlp_set_output_norm(h, _fp(m), _fp(s_)))


def nr_mlp_targets_dev(h, d_mu, P, d_t, stream=None):
    _check(load().nr_mlp_targets_dev(h, C.c_void_p(d_mu), int(P),
                                     C.c_void_p(d_t), C.c_void_p(stream or 0)))


def nr_mlp_train_step_dev(h, d_theta, d_t, B, lr, want_loss=False,
                          stream=None):
    loss = C.c_double(float("nan"))
    _check(load().nr_mlp_train_step_dev(
        h, C.c_void_p(d_theta), C.c_void_p(d_t), int(B), float(lr),
        C.byref(loss) if want_loss else None, C.c_void_p(stream or 0)))
    return loss.value


def nr_mlp_logmu_dev(h, d_theta, B, d_logmu, stream=None):
    _check(load().nr_mlp_logmu_dev(h, C.c_void_p(d_theta), int(B),
                                   C.c_void_p(d_logmu),
                                   C.c_void_p(stream or 0)))


def nr_mlp_nll_dev(h, ctx_h, d_theta, B, d_nll, d_outside=None, stream=None):
    _check(load().nr_mlp_nll_dev(h, ctx_h, C.c_void_p(d_theta), int(B),
                                 C.c_void_p(d_nll),
                                 C.c_void_p(d_outside or 0),
                                 C.c_void_p(stream or 0)))


def nr_eval_mu_batched_dev(ctx_h, d_theta, n_pts, d_mu, stream=None):
    _check(load().nr_eval_mu_batched_dev(ctx_h, C.c_void_p(d_theta),
                                         int(n_pts), C.c_void_p(d_mu),
                                         C.c_void_p(stream or 0)))


def nr_last_error():
    return load().nr_last_error().decode()


# --------------------------------------------------------------- wrapper
class Context:
    """One analysis bound to one device (numpy / torch convenience)."""

    def __init__(self, device: int = 0):
        self.h = nr_create(device)
        self.device = device
        self.n_t = self.n_reco = None

    def close(self):
        if self.h is not None:
            nr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_sources(self, sources, n_t, t_lo=0.0, t_hi=16.0, physics=None):
        nr_set_sources(self.h, sources, n_t, t_lo, t_hi, physics)
        self.n_t = int(n_t)

    def set_response(self, R, m=None, n_sig=1.0e4):
        nr_set_response(self.h, R, m, n_sig)
        self.n_t, self.n_reco = int(R.shape[0]), int(R.shape[1])

    def set_components(self, comp_of_source, hist, scale, rate_sm, **kw):
        """Multi-component form; hist [K, n_t, n_reco]; keywords as in
        nr_set_components.  The data must be set again afterwards."""
        nr_set_components(self.h, comp_of_source, hist, scale, rate_sm, **kw)
        self.n_reco = int(np.shape(hist)[2])

    @property
    def n_theta(self) -> int:
        return nr_num_theta(self.h)

    def set_data(self, n, b, pull_mean=None, pull_sigma=None):
        nr_set_data(self.h, n, b, pull_mean, pull_sigma)

    def eval_nll(self, theta):
        return nr_eval_nll(self.h, theta)

    def eval_nll_grad(self, theta):
        return nr_eval_nll_grad(self.h, theta)

    def eval_mu(self, theta):
        return nr_eval_mu(self.h, theta, self.n_reco)

    def eval_weights(self, theta):
        return nr_eval_weights(self.h, theta, self.n_t)

    def set_mc_events(self, n_events):
        nr_set_mc_events(self.h, n_events)

    def eval_ess(self, theta):
        return nr_eval_ess(self.h, theta, self.n_reco)

    def reference(self):
        return nr_get_reference(self.h, self.n_t)

    def stream(self):
        return nr_stream(self.h)

    def time_stage(self, stage, iters=100):
        return nr_time_stage(self.h, stage, iters)

    def set_band_skipping(self, on=True):
        """Read only the non-zero column bands of R in the single-point
        path (bitwise the same results)."""
        nr_set_band_skipping(self.h, on)

    def set_fold_tiling(self, rows_per_wg=0, use_graph=-1):
        nr_set_fold_tiling(self.h, rows_per_wg, use_graph)

    def eval_nll_batched(self, theta):
        return nr_eval_nll_batched(self.h, theta)

    def eval_nll_grad_batched(self, theta):
        return nr_eval_nll_grad_batched(self.h, theta)

    def eval_mu_batched(self, theta):
        return nr_eval_mu_batched(self.h, theta, self.n_reco)

    def _dev_args(self, theta_t, nll_t, grad_t):
        assert theta_t.dtype == nll_t.dtype and str(theta_t.dtype).endswith("float64")
        assert theta_t.is_contiguous() and nll_t.is_contiguous()
        if theta_t.dim() != 2 or theta_t.shape[1] != self.n_theta:
            raise ValueError(f"theta must be [P, {self.n_theta}]")
        if nll_t.numel() < theta_t.shape[0] or (
                grad_t is not None and grad_t.numel() < self.n_theta * theta_t.shape[0]):
            raise ValueError("output tensors are too small")
        if grad_t is not None:
            assert grad_t.dtype == nll_t.dtype and grad_t.is_contiguous()

    def eval_nll_dev(self, theta_t, nll_t, grad_t=None, stream=None):
        """torch tensors on this device: theta [P, n_theta] f64, nll [P]
        f64, grad [P, 7] f64 or None; enqueued on `stream` (a torch stream,
        or None for the HIP default stream)."""
        self._dev_args(theta_t, nll_t, grad_t)
        sp = None if stream is None else stream.cuda_stream
        nr_eval_nll_dev(self.h, theta_t.data_ptr(), theta_t.shape[0],
                        nll_t.data_ptr(),
                        None if grad_t is None else grad_t.data_ptr(), sp)

    def eval_nll_dev_noalloc(self, theta_t, nll_t, grad_t=None, stream=None):
        """As eval_nll_dev, through the entry point that allocates nothing
        (the library's static per-device workspace)."""
        self._dev_args(theta_t, nll_t, grad_t)
        sp = None if stream is None else stream.cuda_stream
        nr_eval_nll_dev_noalloc(self.h, theta_t.data_ptr(), theta_t.shape[0],
                                nll_t.data_ptr(),
                                None if grad_t is None else grad_t.data_ptr(), sp)

    def build_templates(self):
        nr_build_templates(self.h)

    def eval_nll_templates(self, theta, grad=False):
        return nr_eval_nll_templates(self.h, theta, grad)

    def eval_mu_templates(self, theta):
        return nr_eval_mu_templates(self.h, theta, self.n_reco)

    def eval_nll_templates_dev(self, theta_t, nll_t, grad_t=None, stream=None):
        """The template form on torch tensors, as eval_nll_dev."""
        self._dev_args(theta_t, nll_t, grad_t)
        sp = None if stream is None else stream.cuda_stream
        nr_eval_nll_templates_dev(self.h, theta_t.data_ptr(), theta_t.shape[0],
                                  nll_t.data_ptr(),
                                  None if grad_t is None else grad_t.data_ptr(), sp)


def eval_nll_multi(contexts, thetas):
    """Grouped batched evaluation over several Contexts (host arrays)."""
    return nr_eval_nll_multi([c.h for c in contexts], thetas)


def eval_nll_multi_dev(contexts, theta_ts, nll_ts, grad_ts=None, stream=None):
    """Grouped batched evaluation on torch tensors (one per context)."""
    nr_eval_nll_multi_dev(
        [c.h for c in contexts], [t.data_ptr() for t in theta_ts],
        [t.shape[0] for t in theta_ts], [t.data_ptr() for t in nll_ts],
        None if grad_ts is None else [g.data_ptr() for g in grad_ts],
        None if stream is None else stream.cuda_stream)
