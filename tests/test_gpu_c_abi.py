"""The C ABI used from a plain C program (tests/c/hm_example.c, built by
__graft_entry__.build()): operator build, product, GMRES solve and one
interface-law step, without Python in the process."""
import os
import re
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "hm_example")


def test_c_program_builds_applies_solves_and_updates():
    assert os.path.exists(EXE), "tests/c/hm_example is not built (run __graft_entry__.build())"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    err = float(re.search(r"relative error ([0-9.e+-]+)", r.stdout).group(1))
    assert err <= 1e-7, err
    m = re.search(r"modes (-?\d+) (-?\d+), shear tractions ([0-9.e+-]+) ([0-9.e+-]+)", r.stdout)
    # element 0 stays elastic: 1 MPa + k_s * 10 um; element 1 slides on f * 10 MPa
    assert (int(m.group(1)), int(m.group(2))) == (0, 1)
    assert float(m.group(3)) == pytest.approx(1e6 + 3.2e10 * 1e-5, rel=1e-12)
    assert float(m.group(4)) == pytest.approx(0.6 * 10e6, rel=1e-12)
