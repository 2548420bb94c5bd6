"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only): oracle.c is built with -fsanitize=address,undefined (aborting on the
first report) and the oracle's own pin tests run against that build in a
child process, so an out-of-bounds access or undefined operation in the oracle
fails here instead of going unseen."""
import os
import pathlib
import shutil
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
SUITES = ["tests/test_oracle_eft.py", "tests/test_oracle_split.py", "tests/test_oracle_gemm.py",
          "tests/test_oracle_certify.py", "tests/test_oracle_lu.py", "tests/test_oracle_ds.py"]


def test_oracle_suites_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", str(lib), str(ROOT / "oracle" / "oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib), LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *SUITES],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (out.stdout + out.stderr)[-3000:]
    assert out.returncode == 0, tail
    assert "passed" in out.stdout and "ERROR: AddressSanitizer" not in out.stderr, tail
