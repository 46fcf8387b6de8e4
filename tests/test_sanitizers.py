"""CPU sanitizer builds: the oracle (driven by tests/oracle_selftest.c), the
device modular arithmetic built for the host (tests/host_modarith.cpp) and
the library's host-side number theory and table builder
(tests/host_tables.cpp), each compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (no recovery) and run to completion."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, exe, args=(), timeout=600):
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + list(args), stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=timeout, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_selftest")
    _run(["gcc"] + SAN + ["-fopenmp", "-o", exe, os.path.join(ROOT, "tests", "oracle_selftest.c"),
                          os.path.join(ROOT, "oracle", "oracle.c")], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_device_arithmetic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_modarith")
    _run(["g++"] + SAN + ["-std=c++17", "-o", exe, os.path.join(ROOT, "tests", "host_modarith.cpp")], exe, ["50000"])


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_tables")
    _run(["g++"] + SAN + ["-std=c++17", "-o", exe, os.path.join(ROOT, "tests", "host_tables.cpp")], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_tables_optimised(tmp_path):
    exe = str(tmp_path / "host_tables_o2")
    _run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(ROOT, "tests", "host_tables.cpp")], exe)
