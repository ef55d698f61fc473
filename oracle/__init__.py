"""ctypes front end of the FP64 CPU oracle (plain C, ``tlfea_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The HIP library never imports,
links or executes anything here, and nothing here imports the library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tlfea_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
SRC_OMP = os.path.join(HERE, "tlfea_oracle_omp.c")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

T10 = 1
ANCF3443 = 2
ANCF3243 = 3
SVK = 1
MR = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (single-threaded FP64 C, -O2, no fast-math),
    and its timing-only OpenMP form (the same source plus a threaded loop)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    newest = max(os.path.getmtime(SRC), os.path.getmtime(SRC_OMP))
    if force or not os.path.exists(LIB_OMP) or os.path.getmtime(LIB_OMP) < newest:
        tmp = LIB_OMP + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp, SRC_OMP,
                               "-lm"])
        os.replace(tmp, LIB_OMP)
    return LIB


class _Material(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_double * 3),
                ("eta", ctypes.c_double), ("lam_v", ctypes.c_double)]


class _Mesh(ctypes.Structure):
    _fields_ = [("elem_type", ctypes.c_int), ("n_coef", ctypes.c_int), ("n_elem", ctypes.c_int),
                ("conn", ctypes.POINTER(ctypes.c_int)), ("X", ctypes.POINTER(ctypes.c_double)),
                ("gl", ctypes.c_int * 3), ("thickness", ctypes.c_double), ("width", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_quadrature.argtypes = [ctypes.c_int, ip, dp, dp]
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_t10_shape.argtypes = [dp, dp, dp]
        L.orc_t10_shape.restype = None
        L.orc_ancf3443_shape.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_ancf3243_shape.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_energy_density.argtypes = [ctypes.POINTER(_Material), dp]
        L.orc_energy_density.restype = ctypes.c_double
        L.orc_pk1.argtypes = [ctypes.POINTER(_Material), dp, dp, dp]
        L.orc_pk1.restype = None
        L.orc_tangent.argtypes = [ctypes.POINTER(_Material), dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_tangent.restype = None
        L.orc_element_geometry.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_int, dp, dp]
        L.orc_element.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Material), ctypes.c_int, dp, dp,
                                  ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_csr_build.argtypes = [ctypes.POINTER(_Mesh), ip, ip]
        L.orc_csr_build.restype = ctypes.c_longlong
        L.orc_assemble.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Material), dp, dp, ctypes.c_double,
                                   ctypes.c_double, ip, ctypes.c_int, dp, ip, ip, dp]
        L.orc_slot_map.argtypes = [ctypes.POINTER(_Mesh), ip, ip, ctypes.c_int, ctypes.c_int, ip]
        L.orc_vjp.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Material), dp, dp, dp, dp, dp, dp]
        L.orc_energy.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Material), dp]
        L.orc_energy.restype = ctypes.c_double
        L.orc_element_mass.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_int, ctypes.c_double, dp]
        L.orc_mass_assemble.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_double, ip, ip, dp]
        L.orc_gradient.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp, dp, dp, ctypes.c_double, dp]
        L.orc_gradient.restype = None
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def material(kind, params, eta=0.0, lam_v=0.0) -> _Material:
    p = list(params) + [0.0] * (3 - len(params))
    return _Material(int(kind), (ctypes.c_double * 3)(*p[:3]), float(eta), float(lam_v))


def material_of(m) -> _Material:
    """From a ``workloads.Material``-like object."""
    return material(m.kind, m.params, m.kv_eta, m.kv_lambda)


class Mesh:
    """Keeps the numpy arrays alive for the C struct."""

    def __init__(self, elem_type, X, conn, gl=(0, 0, 0), thickness=0.0, width=0.0):
        self.X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.elem_type = int(elem_type)
        self.n_elem = int(self.conn.shape[0])
        self.n_coef = int(self.X.shape[0])
        self.n_en = {T10: 10, ANCF3443: 16, ANCF3243: 8}[self.elem_type]
        self.s = _Mesh(self.elem_type, self.n_coef, self.n_elem, _ip(self.conn), _dp(self.X),
                       (ctypes.c_int * 3)(*gl), float(thickness), float(width))

    @classmethod
    def of(cls, m):
        return cls(m.elem_type, m.X, m.conn, m.gl, m.thickness, getattr(m, "width", 0.0))

    @property
    def n_dof(self):
        return 3 * self.n_coef

    @property
    def n_qp(self):
        if self.elem_type == T10:
            return 5
        g = self.s.gl
        return g[0] * g[1] * g[2]


def _chk(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def quadrature(elem_type, gl=(0, 0, 0)):
    pts = np.zeros((128, 3))
    w = np.zeros(128)
    n = lib().orc_quadrature(int(elem_type), (ctypes.c_int * 3)(*gl), _dp(pts), _dp(w))
    _chk(0 if n > 0 else n, "quadrature")
    return pts[:n].copy(), w[:n].copy()


def gauss_legendre(n):
    x = np.zeros(8)
    w = np.zeros(8)
    k = lib().orc_gauss_legendre(int(n), _dp(x), _dp(w))
    _chk(0 if k > 0 else k, "gauss_legendre")
    return x[:k].copy(), w[:k].copy()


def t10_shape(xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    N = np.zeros(10)
    dN = np.zeros((10, 3))
    lib().orc_t10_shape(_dp(xi), _dp(N), _dp(dN))
    return N, dN


def ancf3443_shape(xi, lx, ly, H):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    S = np.zeros(16)
    dS = np.zeros((16, 3))
    _chk(lib().orc_ancf3443_shape(_dp(xi), lx, ly, H, _dp(S), _dp(dS)), "ancf3443_shape")
    return S, dS


def energy_density(mat, Hd):
    Hd = np.ascontiguousarray(Hd, dtype=np.float64).reshape(9)
    return lib().orc_energy_density(ctypes.byref(mat), _dp(Hd))


def pk1(mat, Hd, Fdot=None):
    Hd = np.ascontiguousarray(Hd, dtype=np.float64).reshape(9)
    Fd = np.zeros(9) if Fdot is None else np.ascontiguousarray(Fdot, dtype=np.float64).reshape(9)
    P = np.zeros(9)
    lib().orc_pk1(ctypes.byref(mat), _dp(Hd), _dp(Fd), _dp(P))
    return P.reshape(3, 3)


def tangent(mat, Hd, Fdot=None, alpha=1.0, beta=0.0):
    Hd = np.ascontiguousarray(Hd, dtype=np.float64).reshape(9)
    Fd = np.zeros(9) if Fdot is None else np.ascontiguousarray(Fdot, dtype=np.float64).reshape(9)
    A = np.zeros(81)
    lib().orc_tangent(ctypes.byref(mat), _dp(Hd), _dp(Fd), alpha, beta, _dp(A))
    return A.reshape(3, 3, 3, 3)


def element_geometry(mesh: Mesh, e):
    dV = np.zeros(mesh.n_qp)
    g = np.zeros((mesh.n_qp, mesh.n_en, 3))
    _chk(lib().orc_element_geometry(ctypes.byref(mesh.s), int(e), _dp(dV), _dp(g)), "element_geometry")
    return dV, g


def ancf3243_shape(xi, L, W, H):
    S = np.zeros(8)
    dS = np.zeros((8, 3))
    _chk(lib().orc_ancf3243_shape(_dp(np.ascontiguousarray(xi, dtype=np.float64)), L, W, H, _dp(S), _dp(dS)),
         "ancf3243_shape")
    return S, dS


def element(mesh: Mesh, mat, e, q, qdot=None, alpha=1.0, beta=0.0, want_K=True):
    nd = 3 * mesh.n_en
    fe = np.zeros(nd)
    Ke = np.zeros((nd, nd)) if want_K else None
    q = np.ascontiguousarray(q, dtype=np.float64)
    qd = None if qdot is None else np.ascontiguousarray(qdot, dtype=np.float64)
    _chk(lib().orc_element(ctypes.byref(mesh.s), ctypes.byref(mat), int(e), _dp(q), _dp(qd), alpha, beta,
                           _dp(fe), _dp(Ke)), "element")
    return fe, Ke


def csr_pattern(mesh: Mesh):
    nnz = lib().orc_csr_build(ctypes.byref(mesh.s), None, None)
    _chk(0 if nnz >= 0 else int(nnz), "csr count")
    row_off = np.zeros(mesh.n_dof + 1, dtype=np.int32)
    cols = np.zeros(max(nnz, 1), dtype=np.int32)
    n2 = lib().orc_csr_build(ctypes.byref(mesh.s), _ip(row_off), _ip(cols))
    assert n2 == nnz
    return row_off, cols[:nnz]


def assemble(mesh: Mesh, mat, q, qdot=None, alpha=1.0, beta=0.0, elems=None, pattern=None,
             want_f=True, want_K=True):
    """Returns (f, vals); vals is None unless want_K.  ``elems`` restricts the
    sum to a subset of elements (used for sampled parity at full size)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    qd = None if qdot is None else np.ascontiguousarray(qdot, dtype=np.float64)
    f = np.zeros(mesh.n_dof) if want_f else None
    vals = None
    row_off = cols = None
    if want_K:
        if pattern is None:
            pattern = csr_pattern(mesh)
        row_off, cols = pattern
        vals = np.zeros(cols.shape[0])
    el = None if elems is None else np.ascontiguousarray(elems, dtype=np.int32)
    n_list = 0 if el is None else int(el.shape[0])
    _chk(lib().orc_assemble(ctypes.byref(mesh.s), ctypes.byref(mat), _dp(q), _dp(qd), alpha, beta,
                            _ip(el), n_list, _dp(f), _ip(row_off), _ip(cols), _dp(vals)), "assemble")
    return f, vals


def element_mass(mesh: Mesh, e, rho):
    """Consistent element mass m_ab = int rho N_a N_b dV (n_en x n_en), Sec. 4.1."""
    n = mesh.n_en
    m = np.zeros((n, n))
    _chk(lib().orc_element_mass(ctypes.byref(mesh.s), int(e), float(rho), _dp(m)), "element_mass")
    return m


def mass_csr(mesh: Mesh, rho, pattern=None):
    """DOF-level CSR values of M = [m_ab I_3] on the mesh pattern."""
    if pattern is None:
        pattern = csr_pattern(mesh)
    row_off, cols = pattern
    vals = np.zeros(cols.shape[0])
    _chk(lib().orc_mass_assemble(ctypes.byref(mesh.s), float(rho), _ip(row_off), _ip(cols), _dp(vals)),
         "mass_assemble")
    return vals


def gradient(pattern, mvals, v, v_prev, f_int, f_ext, h):
    """g = M (v - v_prev) / h + f_int - f_ext (Sec. 4.4.1, Eq. grad_L, no constraints)."""
    row_off, cols = pattern
    n = row_off.shape[0] - 1
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (mvals, v, v_prev, f_int)]
    fe = None if f_ext is None else np.ascontiguousarray(f_ext, dtype=np.float64)
    g = np.zeros(n)
    lib().orc_gradient(n, _ip(row_off), _ip(cols), _dp(arr[0]), _dp(arr[1]), _dp(arr[2]), _dp(arr[3]), _dp(fe),
                       float(h), _dp(g))
    return g


def slot_map(mesh: Mesh, pattern, e0=0, ne=None):
    row_off, cols = pattern
    if ne is None:
        ne = mesh.n_elem - e0
    nd = 3 * mesh.n_en
    out = np.zeros((ne, nd, nd), dtype=np.int32)
    _chk(lib().orc_slot_map(ctypes.byref(mesh.s), _ip(row_off), _ip(cols), int(e0), int(ne), _ip(out)),
         "slot_map")
    return out


def vjp(mesh: Mesh, mat, q, qdot, w):
    q = np.ascontiguousarray(q, dtype=np.float64)
    qd = np.ascontiguousarray(qdot, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    gq = np.zeros(mesh.n_dof)
    gqd = np.zeros(mesh.n_dof)
    gp = np.zeros(5)
    _chk(lib().orc_vjp(ctypes.byref(mesh.s), ctypes.byref(mat), _dp(q), _dp(qd), _dp(w), _dp(gq), _dp(gqd),
                       _dp(gp)), "vjp")
    return gq, gqd, gp


def energy(mesh: Mesh, mat, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().orc_energy(ctypes.byref(mesh.s), ctypes.byref(mat), _dp(q))


_lib_omp = None


def assemble_omp(mesh: Mesh, mat, q, qdot, alpha, beta, pattern):
    """Timing-only OpenMP form of the fused f + K (atomic scatter over threads);
    returns (f, vals, threads used)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(LIB_OMP):
            build(force=False)
        L = ctypes.CDLL(LIB_OMP)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_assemble_omp.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Material), dp, dp, ctypes.c_double,
                                       ctypes.c_double, dp, ip, ip, dp]
        L.orc_assemble_omp.restype = ctypes.c_int
        L.orc_omp_threads.restype = ctypes.c_int
        _lib_omp = L
    q = np.ascontiguousarray(q, dtype=np.float64)
    qd = None if qdot is None else np.ascontiguousarray(qdot, dtype=np.float64)
    row_off, cols = pattern
    f = np.zeros(mesh.n_dof)
    vals = np.zeros(cols.shape[0])
    _chk(_lib_omp.orc_assemble_omp(ctypes.byref(mesh.s), ctypes.byref(mat), _dp(q), _dp(qd), alpha, beta, _dp(f),
                                   _ip(row_off), _ip(cols), _dp(vals)), "assemble_omp")
    return f, vals, int(_lib_omp.orc_omp_threads())


def adamw_solve(mesh: Mesh, mat, pattern, mvals, q_n, v_n, f_ext, v0, h, lr, beta1, beta2, eps, wd, iters):
    """The first-order inner solver of a time step (Sec. 4.5, Alg. 2) without
    constraint terms, as a plain loop: AdamW with decoupled weight decay on
    g(v) = M (v - v_n)/h + f_int(q_n + h v, v) - f_ext, starting from
    g = m = s = 0; ``iters`` inner iterations, no early exit.  Returns (v, q, g)."""
    v = np.array(v0, dtype=np.float64, copy=True)
    n = v.shape[0]
    g = np.zeros(n)
    m = np.zeros(n)
    s = np.zeros(n)
    q = np.array(q_n, dtype=np.float64, copy=True)
    for l in range(1, iters + 1):
        m = beta1 * m + (1.0 - beta1) * g
        s = beta2 * s + (1.0 - beta2) * g * g
        m_hat = m / (1.0 - beta1 ** l)
        s_hat = s / (1.0 - beta2 ** l)
        v = (1.0 - lr * wd) * v - lr * m_hat / (np.sqrt(s_hat) + eps)
        q = q_n + h * v
        f, _ = assemble(mesh, mat, q, v, 1.0, 0.0, pattern=pattern, want_K=False)
        g = gradient(pattern, mvals, v, v_n, f, f_ext, h)
    return v, q, g
