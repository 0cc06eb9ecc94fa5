"""The C ABI driven from C alone: tests/abi_c/kin_abi_check.c links libkin.so, advances a
two-species isomerisation whose backward-Euler step has a closed form (Sec. 3.2) and exits
non-zero on any mismatch.  The program is built by the build entry point."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "abi_c", "kin_abi_check")


@pytest.mark.gpu
def test_c_program_closed_form():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: run the build entry point first")
    p = subprocess.run([EXE], capture_output=True, text=True, timeout=100)
    print(p.stdout, p.stderr)
    assert p.returncode == 0, p.stdout + p.stderr
    assert p.stdout.strip().endswith("ok")
