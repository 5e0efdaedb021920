"""The oracle's own pins, re-run against a host AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle (CPU only).

The oracle is loaded by ctypes into an uninstrumented Python, so the child
process preloads the sanitizer runtimes.  Any out-of-bounds access, use after
free or undefined behaviour inside the oracle aborts the child and fails this
test.  A planted out-of-bounds read, compiled with the same flags, shows the
sanitizer is armed.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["test_oracle_pins.py", "test_oracle_planted.py", "test_oracle_sparse.py", "test_oracle_fsp.py",
             "test_oracle_typed.py", "test_oracle_refine_grid.py"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def env():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    from oracle import oracle as orc
    orc.build(sanitized=True)
    e = dict(os.environ)
    e.update(LD_PRELOAD=f"{asan} {ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
             UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ARAULLO_ORACLE_SANITIZED="1",
             PYTHONPATH=ROOT)
    return e


def test_sanitizer_is_armed(env, tmp_path):
    from oracle import oracle as orc
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\nint main(void){int *a=malloc(4*sizeof(int));"
                   "volatile int i=4;int x=a[i];free(a);return x;}\n")
    exe = tmp_path / "oob"
    subprocess.run(["gcc", *orc.SANITIZE_FLAGS, str(src), "-o", str(exe)], check=True)
    e = {k: v for k, v in env.items() if k != "LD_PRELOAD"}
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=e)
    # either runtime reports it first: ASan's heap-buffer-overflow or UBSan's
    # object-size check
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr), r.stderr


def test_oracle_pins_under_sanitizers(env):
    probe = ("from oracle import oracle as o; o.lib(); "
             "print(any('liboracle_sanitized.so' in l for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip() == "True", r.stderr[-2000:]
    files = [os.path.join(ROOT, "tests", f) for f in PIN_FILES]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *files], capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
