"""The template form's FP64 logarithm (plain arithmetic, atanh series),
built for the host from the same header the device code includes, against
the C library's log over log-uniform arguments, arguments near 1 and the
range Poisson expectations take."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2607_00488_amd", "csrc")

HARNESS = r"""
#include "lnpos.h"
extern "C" void ln_pos_many(const double* x, double* y, long n) {
    for (long i = 0; i < n; ++i) y[i] = nr::ln_pos(x[i]);
}
"""


# The reciprocal estimate of the quotient (m - 1) / (m + 1): exact on the
# host by default; the second build starts the Newton steps from an
# estimate off by 2^-13 relative, coarser than a hardware estimate needs to
# be for the same two steps of an IEEE division.
SEEDS = {"exact": [], "coarse": ["-DNR_LNPOS_SEED(d)=((1.0/(d))*(1.0+0x1p-13))"]}


@pytest.fixture(scope="module", params=sorted(SEEDS))
def ln_pos(tmp_path_factory, request):
    d = tmp_path_factory.mktemp("lnpos")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    so = d / "libh.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                    "-D__host__=", "-D__device__=", *SEEDS[request.param],
                    "-I", CSRC, str(src), "-o", str(so)],
                   check=True)
    lib = C.CDLL(str(so))
    lib.ln_pos_many.argtypes = [C.c_void_p, C.c_void_p, C.c_long]

    def f(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        lib.ln_pos_many(x.ctypes.data, y.ctypes.data, x.size)
        return y
    return f


def test_against_libm(ln_pos):
    g = np.random.default_rng(20261)
    xs = [np.exp(g.uniform(-700, 700, 400_000)),        # log-uniform, whole range
          1.0 + g.uniform(-1e-3, 1e-3, 100_000),         # near 1
          g.uniform(1e-3, 1e5, 400_000),                 # expected counts per bin
          np.array([0.5, 1.0, 2.0, 0.70710678118654752, 0.7071067811865476,
                    np.nextafter(1.0, 0), np.nextafter(1.0, 2), 5e-324, 2.2250738585072014e-308,
                    1.7976931348623157e308, 3.0, 10.0])]
    x = np.concatenate(xs)
    y = ln_pos(x)
    ref = np.log(x)
    err = np.abs(y - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 4e-16, (err.max(), x[np.argmax(err)])
    # relative accuracy where the value is small (x near 1)
    near = np.abs(ref) < 1e-2
    rel = np.abs(y[near] - ref[near]) / np.maximum(np.abs(ref[near]), 1e-300)
    assert rel.max() <= 8e-16
    assert ln_pos(np.array([1.0]))[0] == 0.0


def test_special_values(ln_pos):
    y = ln_pos(np.array([np.inf, np.nan]))
    assert y[0] == np.inf and np.isnan(y[1])
