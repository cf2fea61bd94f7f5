"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/oracle_sanitize_driver.c calls every oracle entry point once (neighbour list,
evaluation with the descriptor dumps, per-atom outputs, sampled evaluation, NVE and NPT
MD) on two small systems: the 8-molecule water of the tiny model in a box smaller than
2 rc (self images) and a triclinic copy of it.  The driver is built from the oracle's
own source with both sanitizers and must exit cleanly with no report, and its energy
must equal the ctypes oracle's.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I
from oracle.oracle import Oracle
from conftest import tiny_water

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    out = str(tmp_path_factory.mktemp("asan") / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-std=c11",
           "-o", out, os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "dp_oracle.c"), "-lm"]
    subprocess.check_call(cmd)
    return out


def _write_system(path, c, t, b, masses):
    with open(path, "wb") as f:
        f.write(np.int64(len(t)).tobytes())
        f.write(np.ascontiguousarray(c, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(b, dtype=np.float64).reshape(9).tobytes())
        f.write(np.ascontiguousarray(t, dtype=np.int32).tobytes())
        f.write(np.int64(len(masses)).tobytes())
        f.write(np.ascontiguousarray(masses, dtype=np.float64).tobytes())


@pytest.mark.parametrize("case", ["cubic_self_images", "triclinic"])
def test_oracle_clean_under_sanitizers(driver, tiny_model, tmp_path, case):
    c, t, b = tiny_water(11, 2, 6.3)
    if case == "triclinic":
        tric = np.array([[6.6, 0.0, 0.0], [1.3, 6.4, 0.0], [-0.9, 0.7, 6.5]])
        c, b = c @ np.linalg.inv(b) @ tric, tric
    sysf = str(tmp_path / "system.bin")
    _write_system(sysf, c, t, b, [I.MASS["O"], I.MASS["H"]])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([driver, tiny_model, sysf], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-3000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-3000:]
    E_drv = float(r.stdout.split()[1])
    E_ref = Oracle(tiny_model).eval(c, t, b)["E"]
    assert abs(E_drv - E_ref) <= 1e-12 * abs(E_ref)
