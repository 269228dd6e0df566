"""The boundary from C: the header compiles as strict C11 and a C program
(tests/c/abi_driver.c) linked against the library runs sources, response,
data, the plain and template evaluations with gradients, and invalid calls
through the C ABI alone; its results are checked against the oracle."""
import os
import struct
import subprocess
import sys

import numpy as np
import pytest

from problems import inputs, parity_thetas

HERE = os.path.dirname(os.path.abspath(__file__))
INCLUDE = os.path.join(HERE, "..", "include")
DRIVER = os.path.join(HERE, "c", "abi_driver.c")


def build_driver(tmp):
    import paper_2607_00488_amd as nr
    lib = nr.library_path()
    if not os.path.exists(lib):
        pytest.fail(f"{lib} is not built (run __graft_entry__.build())")
    libdir = os.path.dirname(os.path.abspath(lib))
    exe = os.path.join(str(tmp), "abi_driver")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", INCLUDE, DRIVER, "-L", libdir, "-lnureweight",
                    f"-Wl,-rpath,{libdir}", "-lm", "-o", exe], check=True)
    return exe


def test_header_is_c11_and_a_c_program_links(tmp_path):
    assert os.path.exists(build_driver(tmp_path))


def write_problem(path, p, th):
    with open(path, "wb") as f:
        f.write(struct.pack("<4i", len(p["src"]), p["n_t"], p["n_reco"], len(th)))
        f.write(struct.pack("<3d", 0.0, p["t_hi"], p["n_sig"]))
        for s in p["src"]:
            f.write(struct.pack("<3i", s["kind"], len(s["E"]), s["group"]))
            for key in ("E", "weight", "p_ee"):
                f.write(np.ascontiguousarray(s[key], dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(p["R"], dtype="<f4").tobytes())
        for a in (p["n"], p["b"], th):
            f.write(np.ascontiguousarray(a, dtype="<f8").tobytes())


@pytest.mark.gpu
def test_c_caller_against_oracle(tmp_path):
    import paper_2607_00488_amd as nr
    p = inputs(333, 77, 37, 200_000, 91, 92)
    o = p["oracle"]
    th = parity_thetas(0, 8)
    exe = build_driver(tmp_path)
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_problem(fin, p, th)
    print(f"[gpu] C driver over {len(th)} points ({p['n_t']} x {p['n_reco']})", flush=True)
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=180)
    sys.stdout.write(r.stdout + r.stderr)
    assert r.returncode == 0
    P = len(th)
    raw = open(fout, "rb").read()
    d = np.frombuffer(raw[:8 * (16 * P)], dtype="<f8")
    nll, grad = d[:P], d[P:8 * P].reshape(P, 7)
    nll_t, grad_t = d[8 * P:9 * P], d[9 * P:16 * P].reshape(P, 7)
    codes = struct.unpack("<7i", raw[8 * 16 * P:])
    assert codes == (nr.NR_ESTATE, nr.NR_EINVAL, 1, nr.NR_EINVAL, nr.NR_EINVAL,
                     1, nr.NR_ESTATE)
    for i in range(P):
        v, rg = o.nll_grad(th[i])
        scale = np.maximum(np.abs(rg), 1e-3 * np.abs(rg).max())
        for got, g in ((nll[i], grad[i]), (nll_t[i], grad_t[i])):
            assert abs(got - v) <= 1e-3, (i, got, v)
            assert np.all(np.abs(g - rg) <= 1e-4 * scale + 1e-6), (i, g, rg)
