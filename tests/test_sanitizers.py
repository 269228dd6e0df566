"""The FP64 oracle built with the address and undefined-behaviour
sanitizers (gcc, host only) and driven through every entry point by
tests/c/oracle_checked.c: a bad access, leak or undefined operation fails
the run."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(HERE, "..", "oracle", "oracle.c")
DRIVER = os.path.join(HERE, "c", "oracle_checked.c")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_checked")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    ORACLE_C, DRIVER, "-lm", "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle checked run" in r.stdout
