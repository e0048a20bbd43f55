"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code.

Two drivers under tests/sanitize/ are compiled with gcc / g++ and
-fsanitize=address,undefined (no recovery, leak checks on) and run:
oracle_driver.c exercises every exported function of the CPU oracle on small
isolated, MPE, APE-with-columns, 3P, 2P1I and 1P2I trees (walks, columns,
the adaptive block update, the Ewald series and table, HEALPix, the network);
topology_driver.cpp runs the library's host-side topology builder on seeded
random AMR grids and on invalid ones.  A first test checks that the
sanitizer build reports a planted out-of-bounds read, so a clean run means
something.  CPU only.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="8")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="gcc / g++ not available")


def _build_run(cmd, exe, timeout=600):
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=timeout)


def test_sanitizer_reports_a_planted_overflow(tmp_path):
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\nint main(int c, char **v) { int *a = malloc(4 * sizeof(int));"
                   " int r = a[c + 3]; free(a); return r & 1; }\n")
    r = _build_run(["gcc", *SAN, str(src)], str(tmp_path / "oob"))
    # UBSan's object-size check or ASan's shadow check, whichever sees it first
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr)


def test_oracle_under_sanitizers(tmp_path):
    o = os.path.join(ROOT, "oracle")
    srcs = [os.path.join(o, f) for f in ("octoracle.c", "ewald.c", "columns.c", "mlp.c", "mlpwalk.c")]
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", *SAN,
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), *srcs, "-lm"]
    r = _build_run(cmd, str(tmp_path / "oracle_driver"))
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr


def test_topology_under_sanitizers(tmp_path):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.isdir(os.path.join(rocm, "include", "hip")):
        pytest.skip("HIP headers not available")
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"), *SAN,
           os.path.join(ROOT, "tests", "sanitize", "topology_driver.cpp"),
           os.path.join(ROOT, "paper_1708_06142_amd", "csrc", "topology.cpp")]
    r = _build_run(cmd, str(tmp_path / "topology_driver"))
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr
