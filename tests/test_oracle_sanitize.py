"""The FP64 oracle is the reference of every parity claim, and it indexes and allocates by
hand: build it with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) and run oracle/sanitize_driver.c, which calls every entry
point that allocates or indexes on small molecules, including adaptive
screens with seeded budgets, antithetic rounds, pair indices outside the
library and the refused parameters."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    flags = ["-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    build = subprocess.run([gcc, *flags, "-o", exe, os.path.join(ORACLE, "sanitize_driver.c"),
                            os.path.join(ORACLE, "shape_oracle.c"), "-lm"],
                           capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("sanitizer runtime not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    # other libraries the environment preloads may precede the sanitizer's
    # runtime: the link-order check is relaxed for that, nothing else
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    report = run.stdout[-2000:] + run.stderr[-4000:]
    assert run.returncode == 0, report
    assert "runtime error" not in run.stderr, report
    assert "AddressSanitizer" not in run.stderr, report
    assert "sanitize driver ok" in run.stdout
