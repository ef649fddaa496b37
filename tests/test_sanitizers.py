"""Host memory checks: the oracle (gcc, AddressSanitizer + UBSan) and the
library's host code (hipcc, AddressSanitizer on the host side only) are
built with sanitizers and run through their own host tests in a child
process that preloads the sanitizer runtime.  Any sanitizer report fails
the child and this test.  CPU only; the sanitizer builds go to _build/."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")


def run_child(env_extra, tests):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *tests], env=env, cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                       timeout=1200)
    log = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, log
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "LeakSanitizer"):
        assert marker not in r.stdout + r.stderr, log
    return r.stdout


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    from oracle import solver as S
    lib = S.build_sanitized(os.path.join(OUT, "liboracle_asan.so"))
    out = run_child(dict(LD_PRELOAD=S.sanitizer_runtime(), PD_ORACLE_LIB=lib),
                    ["tests/test_oracle_solver.py", "tests/test_oracle_adjoint.py"])
    assert " passed" in out


def test_library_host_code_under_address_sanitizer():
    from paper_2212_04415_amd import build as PB
    lib = PB.build_sanitized(os.path.join(OUT, "libpdmi_asan.so"))
    out = run_child(dict(LD_PRELOAD=PB.sanitizer_runtime(), PDMI_LIB=lib), ["tests/test_library_host.py"])
    assert " passed" in out


def test_the_child_process_reports_a_planted_overflow(tmp_path):
    """Negative control: a one-element heap overflow in a throw-away C
    function, built and loaded the way the oracle's sanitizer build is, is
    reported by the child (so a clean run above means no report)."""
    from oracle import solver as S
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\nint oob(int n) { int *a = malloc(sizeof(int) * n); a[n] = 1; "
                   "int v = a[0]; free(a); return v; }\n")
    lib = str(tmp_path / "liboob.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address", "-fPIC", "-shared", "-o", lib, str(src)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", LD_PRELOAD=S.sanitizer_runtime())
    r = subprocess.run([sys.executable, "-c", f"import ctypes; ctypes.CDLL({lib!r}).oob(4)"], env=env,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
