"""The library's host code under AddressSanitizer on the CPU: every
source built host-only (no device code) against tests/c/mock_hip.cpp, a
stand-in for the HIP runtime that keeps device memory in host memory and
runs no kernel, then driven through call sequences by
tests/host_mock_sequence.py -- among them, at 16384 x 4096, the sequence
of the skipped paper-scale GPU test (67 likelihoods, then the spectra of 4
points).  The values are meaningless; a host-side access out of bounds, a
copy larger than its buffer or a use after free fails the run."""
import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.join(HERE, "..")
CSRC = os.path.join(ROOT, "paper_2607_00488_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
         "-fsanitize=address", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include")]


@pytest.fixture(scope="module")
def mock_lib(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang's shared ASan runtime is missing")
    d = tmp_path_factory.mktemp("mock")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [str(d / (os.path.basename(s)[:-4] + ".o")) for s in srcs]
    procs = [subprocess.Popen([HIPCC] + FLAGS + ["-c", s, "-o", o],
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
             for s, o in zip(srcs, objs)]
    for p, s in zip(procs, srcs):
        out = p.communicate()[0].decode()
        assert p.returncode == 0, f"host-only build of {s} failed:\n{out}"
    # each object names its (absent) device image; give them storage
    names = set()
    for o in objs:
        nm = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        names |= {ln.split()[-1] for ln in nm.stdout.splitlines() if "__hip_fatbin_" in ln}
    fat = d / "fatbins.c"
    fat.write_text("".join(f"char {n}[64];\n" for n in sorted(names)))
    fat_o = str(d / "fatbins.o")
    subprocess.run([CLANGXX, "-x", "c", "-fPIC", "-c", str(fat), "-o", fat_o], check=True)
    libs = {}
    for tag, extra in (("", []), ("_short", ["-DMOCK_SHORT_ALLOC"])):
        mock_o = str(d / f"mock_hip{tag}.o")
        subprocess.run([HIPCC] + FLAGS + extra + ["-c", os.path.join(HERE, "c", "mock_hip.cpp"),
                                                  "-o", mock_o], check=True, capture_output=True)
        lib = str(d / f"libnureweight_mock{tag}.so")
        # -Bsymbolic: the library's own HIP calls bind to the stand-in
        subprocess.run([CLANGXX, "-shared", "-fsanitize=address", "-shared-libasan",
                        "-Wl,-Bsymbolic", "-o", lib] + objs + [mock_o, fat_o], check=True)
        libs[tag] = lib
    return libs, rt[0]


def run_sequence(lib, rt, which):
    env = dict(os.environ, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23")
    return subprocess.run([sys.executable, os.path.join(HERE, "host_mock_sequence.py"), lib,
                           which], capture_output=True, text=True, timeout=600, env=env)


@pytest.mark.parametrize("which", ["broad", "paper"])
def test_host_code_on_cpu_stand_in(mock_lib, which):
    libs, rt = mock_lib
    r = run_sequence(libs[""], rt, which)
    sys.stdout.write(r.stdout[-3000:] + r.stderr[-6000:])
    assert "AddressSanitizer" not in r.stderr
    assert r.returncode == 0 and "mock sequence done" in r.stdout


def test_stand_in_reports_a_short_buffer(mock_lib):
    """The harness is live: with device allocations 8 bytes short, the
    first upload into one is reported."""
    libs, rt = mock_lib
    r = run_sequence(libs["_short"], rt, "broad")
    assert r.returncode == 23, r.stdout[-2000:] + r.stderr[-2000:]
    assert "AddressSanitizer: heap-buffer-overflow" in r.stderr
