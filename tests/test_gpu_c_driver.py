"""The plain C client (tests/c/abi_driver.c) solves a small MLCC2 problem on
the GPU through the C ABI alone; its ground-state energy and three lowest
excitation energies match the FP64 oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import mlcc as om
from paper_2006_05226_amd.synth import gen_inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client_end_to_end(tmp_path):
    O, V, J, o, v = 6, 30, 60, 3, 12
    inp = gen_inputs(O, V, J, o, v, seed=21)
    path = str(tmp_path / "inputs.bin")
    with open(path, "wb") as f:
        f.write(np.array([O, V, J, o, v], dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(inp.L, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(inp.eps, dtype=np.float64).tobytes())
    pkg = os.path.join(ROOT, "paper_2006_05226_amd")
    exe = str(tmp_path / "abi_driver")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "c", "abi_driver.c"),
                    f"-L{pkg}", "-lmlcc", f"-Wl,-rpath,{pkg}", "-lm", "-o", exe],
                   check=True, capture_output=True, text=True)
    print("c client: MLCC2 6/30/60 active 3/12", flush=True)
    r = subprocess.run([exe, "gpu", path], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    e, *w = [float(x) for x in r.stdout.split()]
    OP = om.Problem(inp.L, inp.eps, om.Dims(O, V, o, v), "mlcc2")
    g = om.ground_state(OP, tol=1e-11)
    ref = om.davidson(OP, g["t1"], g["x2"], 3, tol=1e-9)["omega"]
    assert abs(e - g["energy"]) < 1e-10
    assert np.abs(np.array(w) - ref).max() < 1e-8
