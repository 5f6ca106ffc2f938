"""The C-ABI library loads and exports every entry point include/bgktgs.h declares.

CPU-only: loads the shared library with ctypes (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2608_19150_amd", "libbgktgs.so")
HDR = os.path.join(ROOT, "include", "bgktgs.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("build_mesh_dag", "tgs_sweep", "moments", "maxwellian", "bgk_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_last_error_is_callable_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.bgk_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.bgk_last_error(), bytes)


_NOMEM_SCRIPT = r'''
import ctypes as C, resource, sys
import numpy as np
lib = C.CDLL(sys.argv[1])
lib.bgk_last_error.restype = C.c_char_p


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("order", C.c_int), ("n_vert", C.c_int64),
                ("vert", C.c_void_p), ("n_cells", C.c_int64), ("cells", C.c_void_p)]


class VGridDesc(C.Structure):
    _fields_ = [("n_v", C.c_int), ("v", C.c_void_p), ("w", C.c_void_p), ("n_1d", C.c_int),
                ("nodes_1d", C.c_void_p), ("weights_1d", C.c_void_p), ("L", C.c_double),
                ("dg_cells", C.c_int)]


# a valid structured mesh of the unit square: n x n squares, two triangles each
n = 1500
g = np.linspace(0.0, 1.0, n + 1)
X, Y = np.meshgrid(g, g, indexing="ij")
vert = np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], 1))
i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
a = (i * (n + 1) + j).ravel()
cells = np.concatenate([np.stack([a, a + n + 1, a + n + 2], 1),
                        np.stack([a, a + n + 2, a + 1], 1)]).astype(np.int32)
v = np.array([[1.0, 0.5], [-0.5, 1.0]])
w = np.ones(2)
md = MeshDesc(2, 1, vert.shape[0], vert.ctypes.data, cells.shape[0], cells.ctypes.data)
vd = VGridDesc(2, v.ctypes.data, w.ctypes.data, 0, None, None, 1.0, 0)
vm = [int(l.split()[1]) for l in open("/proc/self/status") if l.startswith("VmSize")][0] * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (96 << 20), resource.RLIM_INFINITY))
h = C.c_void_p()
rc = lib.build_mesh_dag(C.byref(md), C.byref(vd), None, None, C.byref(h))
print("RC", rc, lib.bgk_last_error().decode())
'''


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_allocation_failure_is_an_error_code(tmp_path):
    """A host allocation failure inside an entry point comes back as
    BGK_E_NOMEM with a message; no C++ exception crosses the C ABI (which
    would abort the process).  The address space of a child process is
    capped just above its current size and build_mesh_dag is given a mesh of
    4.5 million triangles, whose host tables do not fit; it fails before
    any GPU call."""
    import subprocess
    import sys
    script = tmp_path / "nomem.py"
    script.write_text(_NOMEM_SCRIPT)
    r = subprocess.run([sys.executable, str(script), LIB], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RC")][-1]
    assert line.split()[1] == "-3", line
    assert "alloc" in line
