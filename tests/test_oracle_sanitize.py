"""The CPU oracle built with the compiler's address and undefined-behaviour
checks (gcc -fsanitize=address,undefined, every finding fatal) runs small
cells of every problem variant clean; its forward runs agree bit for bit on
1 and 4 threads and its checkpointed adjoint equals the stored-states one
(tests/sanitize/oracle_driver.c)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_checks(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm", "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all ok" in out.stdout
