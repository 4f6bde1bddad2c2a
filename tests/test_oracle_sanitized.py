"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/sanitize/oracle_driver.c runs the 2-D and 3-D oracle through time steps
on small grids -- every side kind including an inflow segment, V/W/F cycles,
both transfer pairs, red-black smoothing, grids that do not coarsen evenly --
and the explicit reference solver.  It is built with gcc and the two
sanitizers (leak checking on); any invalid access, leak or undefined
operation ends the run with an error.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_runs_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    srcs = [os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "m1_oracle.c"),
            os.path.join(ROOT, "oracle", "m1_oracle3.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-o", exe, *srcs, "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    # verify_asan_link_order=0: the process may have other libraries preloaded ahead of the ASan runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ERROR" not in run.stderr and "runtime error" not in run.stderr, run.stderr
