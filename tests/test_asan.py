"""The host code under AddressSanitizer (CPU only).

The HIP library's host half (argument validation, handle set-up paths that
run without a GPU, the exported ABI) and the FP64 oracle are rebuilt with
AddressSanitizer, and the ABI tests and the oracle pins run again in a
child process with the matching sanitizer runtime preloaded: clang's for
the library (hipcc is clang), gcc's for the oracle.  An invalid read or
write, a use after free or a double free in that code fails the test.
"""
import glob
import os
import subprocess
import sys

import pytest

from tests.conftest import ROOT

PKG = os.path.join(ROOT, "paper_2605_08528_amd")
ASAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1"}


def stale(lib, sources):
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(s) for s in sources)


@pytest.fixture(scope="module")
def libsf_asan():
    from paper_2605_08528_amd import build as B
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + [os.path.join(ROOT, "include", "sf.h")]
    if stale(B.ASAN_LIB, srcs):
        B.build(sanitize=True)
    return B.ASAN_LIB, B.asan_runtime()


@pytest.fixture(scope="module")
def liboracle_asan():
    from oracle import oracle as O
    lib = os.path.join(ROOT, "oracle", "liboracle_asan.so")
    if stale(lib, [O.SRC]):
        O.build(sanitize=True)
    runtime = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    return lib, runtime


def run_under(runtime, env_extra, args):
    env = dict(os.environ, LD_PRELOAD=runtime, **ASAN_ENV, **env_extra)
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)


def test_sanitized_library_is_the_one_loaded(libsf_asan):
    lib, runtime = libsf_asan
    code = ("from paper_2605_08528_amd import sf; sf.lib(); "
            "m = open('/proc/self/maps').read(); "
            "print('libsf_asan.so' in m, 'asan' in m.split('libsf_asan.so')[0] or 'asan-x86_64' in m)")
    r = run_under(runtime, {"SF_LIBRARY": lib}, ["-c", code])
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.split() == ["True", "True"], r.stdout


def test_abi_tests_pass_under_asan(libsf_asan):
    lib, runtime = libsf_asan
    r = run_under(runtime, {"SF_LIBRARY": lib},
                  ["-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"])
    assert r.returncode == 0 and "AddressSanitizer" not in r.stderr, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout


def test_oracle_pins_pass_under_asan(liboracle_asan):
    lib, runtime = liboracle_asan
    r = run_under(runtime, {"SF_ORACLE_LIBRARY": lib},
                  ["-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_oracle_pins.py"])
    assert r.returncode == 0 and "AddressSanitizer" not in r.stderr, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout
