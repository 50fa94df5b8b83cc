"""Host-only tests of the survey server's scheduling policy (sched.hpp):
every request sees each segment of a pass exactly once whenever it joins,
slot limits, memory admission, queue order and capacity, percentiles."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2107_12330_amd", "csrc")


import pytest

SANITIZERS = {
    "plain": [],
    "address_undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "thread": ["-fsanitize=thread"],
}


@pytest.mark.parametrize("sanitize", sorted(SANITIZERS))
def test_scheduler_policy(tmp_path, sanitize):
    """The policy checks, plain and under AddressSanitizer with
    UndefinedBehaviorSanitizer, and under ThreadSanitizer (whose threaded
    section drives the objects from several threads)."""
    exe = tmp_path / "sched_driver"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-pthread", *SANITIZERS[sanitize], "-I", CSRC,
                           os.path.join(HERE, "native", "sched_driver.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout and r.stdout.strip().endswith("PASSED")
    assert "Sanitizer" not in r.stderr
