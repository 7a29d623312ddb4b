"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the CPU code: the
oracle (oracle/oracle.c) and the library's host setup (assembly, orderings,
permutation, threaded ILUT), built here with gcc/g++ and run on small
problems of every kind.  A sanitizer report or a failed check fails the
test.  No device code is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert out.strip().splitlines()[-1].endswith("OK") or "OK" in out, out[-2000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=gnu11", "-ffp-contract=off"] + SAN + [
        os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    print(_build_and_run(cmd, exe, tmp_path))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_1901_01685_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-ffp-contract=off"] + SAN + [
        os.path.join(HERE, "host_driver.cpp"), os.path.join(csrc, "setup_assembly.cpp"),
        os.path.join(csrc, "setup_ilut.cpp"), "-lpthread", "-o", exe]
    print(_build_and_run(cmd, exe, tmp_path))
