"""The C parts of the test infrastructure (the Wilson oracle, the seeded input
generator) built with AddressSanitizer and UndefinedBehaviorSanitizer and run
on small lattices of odd, ragged and single-site extents
(tests/sanitize_driver.c): no out-of-bounds access, no undefined behaviour."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_and_generator_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitize_driver")
    flags = ["-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"]
    srcs = [os.path.join(ROOT, "oracle", "wilson.c"), os.path.join(ROOT, "qcd_inputs", "gen.c"),
            os.path.join(ROOT, "tests", "sanitize_driver.c")]
    build = subprocess.run(["gcc", *flags, "-o", exe, *srcs, "-lm"], capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in (build.stderr or ""):
        pytest.skip("gcc without sanitizer runtimes: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr
    assert "0 failed checks" in run.stdout
