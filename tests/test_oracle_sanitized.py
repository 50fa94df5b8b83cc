"""The oracle's C code built under AddressSanitizer and
UndefinedBehaviorSanitizer (with OpenMP), run on small inputs whose results
the mathematics fixes (tests/native/oracle_sanitize.c): memory errors,
undefined behaviour or a wrong count fail the test."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Wno-unused-function",
                           os.path.join(HERE, "native", "oracle_sanitize.c"), "-o", str(exe)])
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout and r.stdout.strip().endswith("PASSED")
    assert "Sanitizer" not in r.stderr
