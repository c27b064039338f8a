"""The oracle's C code under the host AddressSanitizer and
UndefinedBehaviorSanitizer: oracle/selftest.c drives every function over
small and edge-case inputs (empty documents and queries, out-of-range ids and
codes, format overflow and subnormals) and checks values fixed by the
definitions; any out-of-bounds access, leak or undefined operation aborts the
run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_selftest_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_selftest")
    cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-ffp-contract=off", os.path.join(ROOT, "oracle", "maxsim_oracle.c"),
           os.path.join(ROOT, "oracle", "selftest.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle selftest: ok" in r.stdout
