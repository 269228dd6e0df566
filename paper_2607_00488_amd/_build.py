"""Build of the HIP library for gfx950 (in-tree, no JIT cache)."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libnureweight.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # code-object v5: loadable by the HIP runtime that PyTorch bundles
    "-mcode-object-version=5",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix instructions accumulate in ordinary vector registers: with the
    # accumulation registers the compiler carried the accumulators across
    # the GEMM's K loop in vector registers and copied them over and back
    # every step (96 moves per 32 MFMAs in the 64 x 128 tile)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source of the library into libnureweight.so."""
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + sources() + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


ASAN_LIB = os.path.join(HERE, "libnureweight_asan.so")


def build_asan() -> str:
    """The same library with AddressSanitizer on its host code only (the
    device code is not instrumented), for the host-side sanitizer test: a C
    program linked against it with clang's shared ASan runtime."""
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + [
        "-O1", "-g", "-Xarch_host", "-fsanitize=address",
        "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libasan"]
    tmp = ASAN_LIB + ".tmp"
    res = subprocess.run([hipcc] + flags + sources() + ["-o", tmp],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc (host ASan) failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_asan())
