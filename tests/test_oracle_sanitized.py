"""The oracle's C sources built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven through the ordinary Python binding in a child process (the sanitizer runtime
preloaded, since the interpreter is not instrumented): every oracle entry point, over
burns that succeed, fail, retry and meet a non-finite input, must run clean and give
bitwise the results of the ordinary build.  CPU only."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
SOURCES = ["net.c", "lu.c", "bdf.c", "radau.c", "rkc.c"]
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import oracle_exercise  # noqa: E402


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan runtime")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", lib]
                   + [os.path.join(ORACLE, s) for s in SOURCES] + ["-lm"], check=True)
    out = str(tmp_path / "san.npz")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", ZB_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_exercise.py"), out],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    san = np.load(out)
    plain = oracle_exercise.run()
    assert sorted(san.files) == sorted(plain)
    for k, v in plain.items():
        assert np.array_equal(san[k], v, equal_nan=True), k
