"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
oracle test runs again, in a child process, against a build of the oracle
with both sanitizers (every report fatal), so an out-of-bounds access, a
use after free or undefined behaviour anywhere in the checker fails here.
A planted out-of-bounds read (a volume buffer shorter than its grid) shows
that the sanitizer build reports it."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def sanitized_env(tmp_path_factory):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    import oracle
    lib = oracle.build_sanitized(str(tmp_path_factory.mktemp("asan") / "libmpm_oracle_asan.so"))
    env = dict(os.environ, LD_PRELOAD=rt, MPM_ORACLE_LIB=lib, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",  # the interpreter itself holds memory at exit
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return env


def test_planted_out_of_bounds_read_is_reported(sanitized_env):
    code = ("import numpy as np, oracle\n"
            "lib = oracle._load()\n"
            "sp = oracle.make_spaces([{'dims': (5, 4, 3), 'affine': np.hstack([np.eye(3), np.zeros((3, 1))])}])\n"
            "vol, out = np.zeros(10), np.zeros(60)  # the grid needs 60 values\n"
            "lib.orc_pull(oracle._dims((5, 4, 3)), sp, oracle._ptr(vol), oracle._ptr(out))\n")
    r = subprocess.run([sys.executable, "-c", code], env=sanitized_env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


def test_oracle_suite_is_clean_under_sanitizers(sanitized_env):
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + files,
                       env=sanitized_env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    print(r.stdout[-600:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
