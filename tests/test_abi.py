"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(nr_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("nr_set_sources", "nr_set_response", "nr_set_data",
              "nr_eval_nll", "nr_eval_nll_grad"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2607_00488_amd as nr
    path = nr.library_path()
    if not os.path.exists(path):
        pytest.fail(f"{path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(nr.EXPORTS) <= declared_functions()
    assert declared_functions() <= set(nr.EXPORTS)


def test_binding_has_the_same_names():
    import paper_2607_00488_amd as nr
    for n in declared_functions():
        assert hasattr(nr, n), n


def test_probe_rejects_bad_arguments_without_a_device():
    """Argument checks of the matrix-core and read probes return before any
    device call (so they run here without a GPU)."""
    import numpy as np
    import paper_2607_00488_amd as nr
    lib = nr.load()
    out = np.zeros(1)
    for blocks, iters in ((0, 1), (1, 0), (1 << 17, 1)):
        assert lib.nr_probe_mfma_f64(0, blocks, iters, nr._dp(out)) == nr.NR_EINVAL
    assert lib.nr_probe_mfma_f64(0, 1, 1, None) == nr.NR_EINVAL
    for nbytes, reps in ((1 << 19, 1), ((1 << 20) + 8, 1), (1 << 20, 0), (1 << 37, 1)):
        assert lib.nr_probe_hbm_read(0, nbytes, reps, nr._dp(out)) == nr.NR_EINVAL
        assert lib.nr_probe_read(0, nbytes, reps, 3, nr._dp(out)) == nr.NR_EINVAL
    for flags in (-1, 4, 7):
        assert lib.nr_probe_read(0, 1 << 20, 1, flags, nr._dp(out)) == nr.NR_EINVAL
    assert lib.nr_probe_read(0, 1 << 20, 1, 0, None) == nr.NR_EINVAL


def test_header_constants_match_the_binding():
    """Every integer #define of the header (status codes, parameter counts,
    probe flags) has the same value in the Python binding."""
    import paper_2607_00488_amd as nr
    text = open(os.path.join(ROOT, "include", "nureweight.h")).read()
    found = dict(re.findall(r"#define\s+(NR_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text))
    assert {"NR_OK", "NR_EINVAL", "NR_PROBE_CACHED", "NR_PROBE_ALTERNATE"} <= set(found)
    for name, value in found.items():
        assert hasattr(nr, name), name
        assert getattr(nr, name) == int(value), (name, getattr(nr, name), value)
