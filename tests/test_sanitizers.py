"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the host code
(CPU only; no GPU code is built with a sanitizer):

- the library's host setup (host_setup.cpp, partition.cpp, cinv.cpp,
  cheb.cpp) compiled with g++ -fsanitize=address,undefined next to a driver
  (tests/sanitize/host_driver.cpp) that runs every host-build path on small
  matrices and the input checks on bad input; leak checking on;
- the oracle compiled with the same sanitizers and driven through its Python
  binding (tests/sanitize/oracle_workflow.py) with libasan preloaded.

Any sanitizer report stops the program with a nonzero status."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1505_04341_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


pytestmark = pytest.mark.skipif(runtime("libasan.so") is None, reason="no AddressSanitizer runtime")


def test_host_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    srcs = [os.path.join(HERE, "sanitize", "host_driver.cpp")] + [
        os.path.join(CSRC, f) for f in ("host_setup.cpp", "partition.cpp", "cinv.cpp", "cheb.cpp")]
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", exe],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    lib = oracle.build(True, str(tmp_path / "libddlr_oracle_san.so"), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=runtime("libasan.so"), ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitize", "oracle_workflow.py"), lib],
                       capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]
