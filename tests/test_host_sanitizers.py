"""Host-side sanitizer runs, on the CPU: the oracle built with AddressSanitizer
and UndefinedBehaviorSanitizer runs its pins, and the library built with both
sanitizers on its host side (device code unchanged) runs the argument checks of
the C ABI and the clean-up of creations that fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _env(**extra):
    env = dict(os.environ)
    # Python itself is not instrumented and keeps its objects to the end, so
    # leak reports would be its own; every other finding stops the run
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.update(extra)
    return env


def _gcc_asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path):
        pytest.skip("gcc has no shared ASan runtime")
    return path


def _check_clean(r):
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]


def test_sanitizer_runtime_is_live(tmp_path):
    # the preloaded runtime reports a heap overflow in an instrumented library
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "int planted(int i) { int* a = malloc(4 * sizeof(int)); a[i] = 1;"
                   " int v = a[0]; free(a); return v; }\n")
    so = tmp_path / "libplanted.so"
    subprocess.run(["gcc", "-shared", "-fPIC", "-g", "-fsanitize=address", str(src), "-o", str(so)],
                   check=True)
    code = f"import ctypes; ctypes.CDLL({str(so)!r}).planted(4)"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       env=_env(LD_PRELOAD=_gcc_asan_runtime()))
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


def test_oracle_pins_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    so = tmp_path / "liboracle_asan.so"
    subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-ffp-contract=off", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(so), "-lm"], check=True)
    env = _env(LD_PRELOAD=_gcc_asan_runtime(), ORACLE_LIB=str(so))
    probe = ("import oracle.oracle as O; O._load(); "
             "print(any('liboracle_asan' in l for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True,
                       timeout=120, env=env, cwd=ROOT)
    _check_clean(r)
    assert r.stdout.strip() == "True"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    _check_clean(r)
    assert " passed" in r.stdout


def test_abi_checks_under_host_asan_ubsan(tmp_path):
    from paper_2305_15693_amd import build as B
    if not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc")
    lib = B.build_host_sanitized(str(tmp_path))
    env = _env(LD_PRELOAD=B.host_sanitizer_runtime(), FRESCO_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), "-k",
                        "invalid or validation or exports or releases"],
                       capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    _check_clean(r)
    assert "4 passed" in r.stdout
