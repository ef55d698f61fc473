"""CPU checks of the C ABI boundary: the built library loads, exports every
function declared in include/tlfea.h, agrees with the header on the
descriptor layout, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlfea.h")


@pytest.fixture(scope="module")
def native():
    from paper_2604_10357_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        from paper_2604_10357_amd import build as B
        B.build(verbose=False)
    return N


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tlfea_\w+)\s*\(", text)))


def test_every_declared_function_is_exported(native):
    decl = declared_functions()
    assert len(decl) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in decl if f not in exported]
    assert not missing, missing
    # and nothing else leaks out of the library
    extra = sorted(e for e in exported if e.startswith("tlfea_") and e not in decl)
    assert not extra, extra
    assert sorted(native.EXPORTED) == decl
    L = native.lib()
    for f in decl:
        assert hasattr(L, f)


def test_descriptor_layout_matches_header(native, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "tlfea.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(tlfea_mesh_desc),"
        " offsetof(tlfea_mesh_desc, n_coef), offsetof(tlfea_mesh_desc, h_conn), offsetof(tlfea_mesh_desc, gl),"
        " offsetof(tlfea_mesh_desc, thickness), offsetof(tlfea_mesh_desc, params),"
        " offsetof(tlfea_mesh_desc, kv_lambda), offsetof(tlfea_mesh_desc, precision),"
        " offsetof(tlfea_mesh_desc, width));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    D = native.MeshDesc
    want = [ctypes.sizeof(D), D.n_coef.offset, D.h_conn.offset, D.gl.offset, D.thickness.offset, D.params.offset,
            D.kv_lambda.offset, D.precision.offset, D.width.offset]
    assert got == want


def test_gather_shape_layout_matches_header(native, tmp_path):
    src = tmp_path / "shape.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "tlfea.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu\\n\", sizeof(tlfea_gather_shape),"
        " offsetof(tlfea_gather_shape, waves), offsetof(tlfea_gather_shape, range_tasks),"
        " offsetof(tlfea_gather_shape, range_values));return 0;}\n")
    exe = tmp_path / "shape"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    G = native.GatherShape
    assert got == [ctypes.sizeof(G), G.waves.offset, G.range_tasks.offset, G.range_values.offset]


def test_status_strings_and_version(native):
    L = native.lib()
    assert L.tlfea_version() >= 100
    for code in range(-7, 1):
        s = native.status_string(code)
        assert s and s != "unknown status"
    assert native.status_string(-99) == "unknown status"


def _desc(native, elem_type=1, n_coef=10, n_elem=1, conn=None, X=None, material=1, params=(1e7, 0.3, 0.0),
          precision=0, gl=(0, 0, 0), thickness=0.0):
    d = native.MeshDesc()
    d.elem_type = elem_type
    d.n_coef = n_coef
    d.n_elem = n_elem
    keep = []
    if conn is not None:
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        keep.append(conn)
        d.h_conn = conn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if X is not None:
        X = np.ascontiguousarray(X, dtype=np.float64)
        keep.append(X)
        d.h_X = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.gl = (ctypes.c_int32 * 3)(*gl)
    d.thickness = thickness
    d.material = material
    d.params = (ctypes.c_double * 3)(*params)
    d.precision = precision
    return d, keep


def test_argument_validation_needs_no_gpu(native):
    """Every one of these is rejected by host-side checks before any HIP call."""
    L = native.lib()
    h = ctypes.c_void_p()
    assert L.tlfea_mesh_create(None, ctypes.byref(h)) == native.TLFEA_OK - 1
    assert L.tlfea_mesh_create(None, None) == -1
    X = np.zeros((10, 3))
    conn = np.arange(10)[None, :]
    d, keep = _desc(native, elem_type=7, conn=conn, X=X)
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -2 and not h.value
    d, keep = _desc(native, conn=np.array([[0, 1, 2, 3, 4, 5, 6, 7, 8, 10]]), X=X)   # id out of range
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -1
    d, keep = _desc(native, conn=conn, X=X, material=9)
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -2
    d, keep = _desc(native, conn=conn, X=X, params=(1e7, 0.5, 0.0))              # nu = 0.5
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -1
    d, keep = _desc(native, conn=conn, X=X, precision=5)
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -1
    d, keep = _desc(native, elem_type=2, n_coef=16, conn=np.arange(4)[None, :], X=np.zeros((16, 3)), gl=(2, 2, 2),
                    thickness=0.1)
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -2            # rule not offered
    d, keep = _desc(native, elem_type=2, n_coef=16, conn=np.arange(4)[None, :], X=np.zeros((16, 3)), gl=(3, 3, 2),
                    thickness=0.0)
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -1            # no thickness
    Xnan = X.copy()
    Xnan[3, 1] = np.nan
    d, keep = _desc(native, conn=conn, X=Xnan)
    assert L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)) == -1
    # null handles
    assert L.tlfea_mesh_destroy(None) == 0
    assert L.tlfea_internal_force(None, None, None, None, None) == -1
    assert L.tlfea_tangent(None, None, None, 1.0, None, None) == -1
    assert L.tlfea_assemble(None, None, None, 1.0, None, None, None) == -1
    assert L.tlfea_assemble_accumulate(None, None, None, 1.0, 1.0, None, None, None) == -1
    assert L.tlfea_internal_force_vjp(None, None, None, None, None, None, None, None) == -1
    assert L.tlfea_build_csr_pattern(None, None) == -1
    assert L.tlfea_get_runtime_flags(None, None) == -1
    assert L.tlfea_mesh_info(None, None, None, None, None, None) == -1
    assert L.tlfea_batch_create(None, 0, ctypes.byref(h)) == -1
    assert L.tlfea_batch_destroy(None) == 0
    sh = native.GatherShape(4, 768, 4096)
    assert L.tlfea_mesh_set_gather_shape(None, ctypes.byref(sh)) == -1
    assert L.tlfea_mesh_get_gather_shape(None, ctypes.byref(sh), None) == -1
    assert L.tlfea_mesh_autotune(None, None, None, 1.0, None, None, 5, None, None, None) == -1
    assert L.tlfea_batch_set_gather_shape(None, ctypes.byref(sh)) == -1
    assert L.tlfea_batch_get_gather_shape(None, ctypes.byref(sh), None) == -1
    assert L.tlfea_batch_autotune(None, None, None, None, None, None, 5, None, None, None) == -1
    assert L.tlfea_build_mass(None, 1000.0) == -1
    assert L.tlfea_get_mass(None, None, None) == -1
    assert L.tlfea_assemble_newton(None, None, None, 1e-3, None, None, None) == -1
    assert L.tlfea_newton_gradient(None, None, None, None, None, 1e-3, None, None) == -1
    assert L.tlfea_build_upper_pattern(None, None) == -1
    assert L.tlfea_get_csr_pattern_upper(None, None, None, 0, None) == -1
    assert L.tlfea_assemble_upper(None, None, None, 1.0, 0.0, None, None, None) == -1
    assert L.tlfea_adamw_solve(None, None, 1e-3, None, None, None, None, None, None, 10, 5, 0.0, 0.0, None, None,
                               None) == -1
