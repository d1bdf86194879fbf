"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (oracle/sanitize_check.c) compiled with gcc on the host sweeps every
Hamiltonian, scheme and RK order on tiny grids; an invalid access or an
undefined operation aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-std=c99", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE]
    cs = str(tmp_path / "hjxo_cs.o")
    subprocess.run(["gcc", *flags, "-DHJXO_CSTEP", "-c", os.path.join(ORACLE, "hjxo.c"), "-o", cs], check=True)
    subprocess.run(["gcc", *flags, os.path.join(ORACLE, "sanitize_check.c"), cs, "-o", exe, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitized run: ok" in r.stdout
    assert "runtime error" not in r.stderr
