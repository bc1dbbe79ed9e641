"""Host-side logic of the runtime built for the CPU alone, under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU, no HIP): the context's slot rotation, the burn server's
scheduling policy on a fake device, the series logarithm of the rate evaluation, the
refinements of the step control and the autotuner's JSON file."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_06466_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host")


def _build_and_run(src, tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not found")
    exe = str(tmp_path / "prog")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(HERE, src), "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_slot_rotation_waits_for_the_previous_user(tmp_path):
    out = _build_and_run("slots_test.cpp", tmp_path)
    assert "slots ok" in out



def test_server_scheduling_on_a_fake_device(tmp_path):
    out = _build_and_run("sched_test.cpp", tmp_path)
    for part in ("arena ok", "plan ok", "simulation ok", "failures ok", "threads ok", "sched ok"):
        assert part in out


def test_series_logarithm_is_within_1_2_ulp(tmp_path):
    out = _build_and_run("log_test.cpp", tmp_path)
    assert "log ok" in out


def test_step_control_refinements_are_within_1_ulp(tmp_path):
    out = _build_and_run("stepmath_test.cpp", tmp_path)
    assert "stepmath ok" in out


def test_tuning_file_reads_back_and_refuses_malformed_input(tmp_path):
    out = _build_and_run("tunecache_test.cpp", tmp_path)
    for part in ("round trip ok", "reordered ok", "refusals ok", "tunecache ok"):
        assert part in out
