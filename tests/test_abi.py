"""The C-ABI library loads and exports every function include/*.h declares
(CPU only: no device call is made)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2006_05226_amd import mlcc


def header_functions(root):
    names = set()
    for h in sorted(glob.glob(os.path.join(root, "include", "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(mlcc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol(root):
    names = header_functions(root)
    assert len(names) >= 18
    lib = ctypes.CDLL(mlcc.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(mlcc.EXPORTS) == names


def test_binding_declares_signatures():
    lib = mlcc.load()
    for n in mlcc.EXPORTS:
        assert getattr(lib, n).argtypes is not None


def test_create_error_without_gpu_is_reported():
    """Without a device the context call fails with a status, never a crash."""
    import torch
    if torch.cuda.is_available():
        return
    lib = mlcc.load()
    h = ctypes.c_void_p()
    st = lib.mlcc_context_create(0, None, 0, ctypes.byref(h))
    assert st < 0
    assert len(lib.mlcc_last_error(None)) > 0


def test_tile_override_arguments():
    """mlcc_gemm_tile is per context: without one it is refused, never a crash."""
    lib = mlcc.load()
    last = (ctypes.c_int32 * 2)()
    assert lib.mlcc_gemm_tile(None, 128, 96, last) == mlcc.E_ARG
    assert lib.mlcc_gemm_tile(None, -1, 32, None) == mlcc.E_ARG


def test_noalloc_engine_arguments():
    """mlcc_gemm_noalloc refuses a NULL context without touching a device, and
    its scratch size is the one the header states."""
    lib = mlcc.load()
    s4 = (ctypes.c_int64 * 4)(1, 1, 0, 0)
    s3 = (ctypes.c_int64 * 3)(1, 1, 0)
    assert lib.mlcc_gemm_noalloc(None, mlcc.FP64, 1, 1, 1, 1, 1, 1.0, None, s4, None, s4, 0.0,
                                 None, s3, None) == mlcc.E_ARG
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "include", "mlcc_engine.h")).read()
    m = re.search(r"#define MLCC_NOALLOC_SCRATCH_BYTES \(\(uint64_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == mlcc.NOALLOC_SCRATCH_BYTES


def test_cnto_argument_checks():
    """Entry points added with the orbital selection refuse NULL handles
    without touching a device."""
    lib = mlcc.load()
    assert lib.mlcc_cnto(None, 1, None, None, 0, 0, None, None, None, None, None, None) == mlcc.E_ARG


def test_problem_descriptor_layout_matches_header():
    """The binding's mlcc_problem_desc has the header's members in the
    header's order (names and C types), so the structure layouts agree."""
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "include", "mlcc.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} mlcc_problem_desc;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    members = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(const\s+)?(\w+)\s*(\*?)\s*(.*)", decl)
        ctype = m.group(2) + m.group(3)
        for name in m.group(4).split(","):
            members.append((name.strip().lstrip("*"), "ptr" if ("*" in ctype or "*" in name)
                            else ctype))
    ct = {"int32_t": ctypes.c_int32, "uint32_t": ctypes.c_uint32, "uint64_t": ctypes.c_uint64,
          "ptr": ctypes.c_void_p}
    fields = mlcc.ProblemDesc._fields_
    assert [n for n, _ in members] == [f[0] for f in fields]
    assert all(ct[t] is f[1] for (_, t), f in zip(members, fields))
    assert mlcc.MODEL["mlccsd3"] == int(re.search(r"#define MLCC_MLCCSD3 (\d+)", text).group(1))
    for name in ("SYNTH_L", "INPUT_ON_DEVICE", "DETERMINISTIC"):
        value = int(re.search(r"#define MLCC_%s (\d+)u" % name, text).group(1))
        assert getattr(mlcc, name) == value, name
    flags = [getattr(mlcc, n) for n in ("SYNTH_L", "INPUT_ON_DEVICE", "DETERMINISTIC")]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == 3  # distinct bits


def test_plain_c_client(tmp_path):
    """include/mlcc.h compiles as C99 with warnings as errors, and a C client
    linked against the library gets the documented argument errors and
    footprint estimates without a device (tests/c/abi_driver.c)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2006_05226_amd")
    exe = str(tmp_path / "abi_driver")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    f"-I{os.path.join(root, 'include')}", os.path.join(root, "tests", "c", "abi_driver.c"),
                    f"-L{pkg}", "-lmlcc", f"-Wl,-rpath,{pkg}", "-lm", "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
