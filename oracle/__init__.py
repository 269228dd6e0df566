"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never loads it, and it shares no
code with the HIP path: the C source in this folder is its own, and this
wrapper only marshals arguments through ctypes.

See ``oracle.c`` for the passage of the paper each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

THETA_SM = np.array([0, 0, 0, 0, 0, 1, 1], dtype=np.float64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no contraction, no fast-math,
    OpenMP over independent bins only."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c99", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        F = C.POINTER(C.c_float)
        L.or_create.restype = P
        L.or_destroy.argtypes = [P]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_set_physics.argtypes = [P] + [C.c_double] * 5
        L.or_add_source.argtypes = [P, C.c_int, C.c_int, D, D, D, C.c_int]
        L.or_add_source.restype = C.c_int
        L.or_set_grid.argtypes = [P, C.c_int, C.c_double, C.c_double]
        L.or_set_grid.restype = C.c_int
        L.or_set_response.argtypes = [P, F, C.c_int, C.c_int, D, C.c_double]
        L.or_set_response.restype = C.c_int
        L.or_set_data.argtypes = [P, D, D, C.c_int, D, D]
        L.or_set_data.restype = C.c_int
        L.or_dsigma.argtypes = [P, C.c_int, C.c_double, C.c_double, D]
        L.or_dsigma.restype = C.c_double
        for name in ("or_spectrum", "or_weights", "or_mu", "or_row_factors"):
            fn = getattr(L, name)
            fn.restype = C.c_int
        L.or_spectrum.argtypes = [P, D, D]
        L.or_weights.argtypes = [P, D, D]
        L.or_mu.argtypes = [P, D, D]
        L.or_row_factors.argtypes = [P, D]
        L.or_nll.argtypes = [P, D]
        L.or_nll.restype = C.c_double
        L.or_nll_grad.argtypes = [P, D, D]
        L.or_nll_grad.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def set_threads(n: int):
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


class Oracle:
    """One analysis: sources, recoil grid, response and data."""

    def __init__(self, physics=None):
        self._L = _load()
        self._c = self._L.or_create()
        self._keep = []
        if physics is not None:
            self._L.or_set_physics(self._c, *[float(x) for x in physics])

    def close(self):
        if self._c:
            self._L.or_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_source(self, kind, E, weight, p_ee, group=0):
        E, pE = _d(E)
        w, pw = _d(weight)
        p, pp = _d(p_ee)
        rc = self._L.or_add_source(self._c, int(kind), len(E), pE, pw, pp,
                                   int(group))
        assert rc == 0, rc

    def set_sources(self, sources, n_t, t_lo=0.0, t_hi=16.0):
        for s in sources:
            self.add_source(s["kind"], s["E"], s["weight"], s["p_ee"],
                            s["group"])
        assert self._L.or_set_grid(self._c, int(n_t), float(t_lo),
                                   float(t_hi)) == 0
        self.n_t = int(n_t)

    def set_response(self, R, m=None, n_sig=1.0e4):
        R = np.ascontiguousarray(R, dtype=np.float32)
        pm = None
        if m is not None:
            m, pm = _d(m)
        rc = self._L.or_set_response(
            self._c, R.ctypes.data_as(C.POINTER(C.c_float)), R.shape[0],
            R.shape[1], pm, float(n_sig))
        assert rc == 0, rc
        self.n_reco = R.shape[1]

    def set_data(self, n, b, pull_mean=None, pull_sigma=None):
        n, pn = _d(n)
        b, pb = _d(b)
        pm = ps = None
        if pull_mean is not None:
            pmv, pm = _d(pull_mean)
            psv, ps = _d(pull_sigma)
            self._keep += [pmv, psv]
        rc = self._L.or_set_data(self._c, pn, pb, len(n), pm, ps)
        assert rc == 0, rc

    def dsigma(self, flavour, E, T, theta):
        th, pth = _d(theta)
        return self._L.or_dsigma(self._c, int(flavour), float(E), float(T), pth)

    def spectrum(self, theta):
        th, pth = _d(theta)
        out = np.empty(self.n_t)
        assert self._L.or_spectrum(self._c, pth, _d(out)[1]) == 0
        return out

    def weights(self, theta):
        th, pth = _d(theta)
        out = np.empty(self.n_t)
        assert self._L.or_weights(self._c, pth, _d(out)[1]) == 0
        return out

    def row_factors(self):
        out = np.empty(self.n_t)
        assert self._L.or_row_factors(self._c, _d(out)[1]) == 0
        return out

    def mu(self, theta):
        th, pth = _d(theta)
        out = np.empty(self.n_reco)
        assert self._L.or_mu(self._c, pth, _d(out)[1]) == 0
        return out

    def nll(self, theta):
        th, pth = _d(theta)
        return float(self._L.or_nll(self._c, pth))

    def nll_grad(self, theta):
        th, pth = _d(theta)
        g = np.empty(7)
        v = self._L.or_nll_grad(self._c, pth, _d(g)[1])
        return float(v), g
