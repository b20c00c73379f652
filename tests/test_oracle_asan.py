"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): oracle/asan_check.c drives every entry point of oracle.h on
small dense and CSR problems, ragged and degenerate shapes, every inner rule
and flag, replays, a save and a resume, non-finite error scales and invalid
inputs; any out-of-bounds access, use after free, leak or undefined
operation aborts the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
           "-Wall", "-Wextra", "-Werror", "-o", exe,
           os.path.join(ORACLE, "oracle.c"), os.path.join(ORACLE, "asan_check.c"), "-lm"]
    built = subprocess.run(cmd, capture_output=True, text=True)
    assert built.returncode == 0, built.stderr
    # The environment is passed on unchanged apart from the sanitizer options
    # (a library preloaded by the environment may come before the sanitizer
    # runtime, which its link-order check would otherwise refuse).
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip() == "ok"
    assert "Sanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr
