"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle pin suites run against a sanitized build of the oracle (gcc,
libasan preloaded), and any sanitizer report fails the test.  The host part
of the HIP library's argument checks runs under the same runtime."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def sanitized_env(lib: str) -> dict:
    import oracle
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = oracle.asan_runtime()
    # CPython itself leaks by design; memory errors and UB stay fatal
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    import oracle
    lib = oracle.build_sanitized()
    suites = ["tests/test_oracle_pins.py", "tests/test_oracle_peeksort.py", "tests/test_oracle_mergesorts.py",
              "tests/test_oracle_comparisons.py", "tests/test_oracle_galloping.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", "-k",
                        "not printed_in_sec4", *suites], cwd=ROOT, env=sanitized_env(lib),
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout


@pytest.mark.slow
def test_sanitizer_catches_a_planted_overflow(tmp_path):
    """The sanitized build does report errors: an out-of-bounds write planted
    in a copy of the oracle (one element past the merge buffer) aborts."""
    import oracle
    src = open(os.path.join(ROOT, "oracle", "powersort_oracle.c")).read()
    a = "        memcpy(tk + o * ks, A->key + src * ks, ks);"
    assert a in src
    bad = tmp_path / "bad.c"
    bad.write_text(src.replace(a, a + "\n        if (o + 1 == hi - lo) memcpy(tk + (o + 1) * ks, A->key + src * ks, ks);"))
    lib = str(tmp_path / "liboracle_bad.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", *oracle.SANITIZE_FLAGS, "-o", lib,
                           str(bad)])
    code = "import numpy as np, oracle\noracle.powersort(np.r_[np.arange(40), np.arange(27)].astype(np.int32))\n"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=sanitized_env(lib), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]


@pytest.mark.slow
def test_abi_host_checks_under_asan_and_ubsan():
    """tests/test_abi_host.py (exports, argument checks, status strings,
    workspace sizes, tuning, pool limit) against a build of the library
    whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer."""
    from paper_1805_04154_amd import build
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env["POWERSORT_HIP_LIB"] = lib
    env["LD_PRELOAD"] = build.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                        "tests/test_abi_host.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
