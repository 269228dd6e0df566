"""The library's host code under AddressSanitizer: the ASan build
(libnureweight_asan.so, device code unchanged) driven from C by
tests/c/host_asan_stress.c through most entry points on the GPU; any
invalid host memory access fails the run."""
import os
import subprocess
import sys

import pytest

from problems import inputs, parity_thetas
from test_c_abi import write_problem

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
INCLUDE = os.path.join(HERE, "..", "include")
DRIVER = os.path.join(HERE, "c", "host_asan_stress.c")
CLANG = "/opt/rocm/llvm/bin/clang"


def test_host_code_under_asan(tmp_path):
    import glob
    from paper_2607_00488_amd import _build
    lib = _build.ASAN_LIB
    if not os.path.exists(lib):
        pytest.fail(f"{lib} is not built (run __graft_entry__.build())")
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    assert rt, "clang's shared ASan runtime is missing"
    libdir = os.path.dirname(lib)
    exe = str(tmp_path / "stress")
    subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fsanitize=address", "-shared-libasan",
                    "-fno-omit-frame-pointer", "-I", INCLUDE, DRIVER, "-L", libdir,
                    "-l:libnureweight_asan.so", f"-Wl,-rpath,{libdir}",
                    f"-Wl,-rpath,{os.path.dirname(rt[0])}", "-lm", "-o", exe], check=True)
    fin = str(tmp_path / "in.bin")
    write_problem(fin, inputs(333, 77, 37, 200_000, 91, 92), parity_thetas(0, 48))
    print("[gpu] host ASan stress run (333 x 77, 81 points, no single-point spectra)", flush=True)
    # the HIP runtime's own allocations outlive the process, so no leak check
    env = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=0")
    r = subprocess.run([exe, fin], capture_output=True, text=True, timeout=240, env=env)
    sys.stdout.write(r.stdout[-2000:] + r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr
    assert r.returncode == 0 and "stress ok" in r.stdout
