"""Torch-facing wrappers over the C ABI.  PyTorch only provides device memory
and the current stream; every step of the computation runs in the HIP kernels
of ``libtlfea.so``."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N
from .workloads import Material, Mesh

_PREC = {"fp64": N.TLFEA_FP64, "mixed": N.TLFEA_MIXED}


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor], dtype=torch.float64, n: Optional[int] = None) -> Optional[ctypes.c_void_p]:
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor, got {t.dtype} on {t.device}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class TLMesh:
    """One mesh handle: reference geometry, material, CSR pattern and slot map on the GPU."""

    def __init__(self, mesh: Mesh, material: Material, precision: str = "fp64"):
        if not torch.cuda.is_available():
            raise RuntimeError("TLMesh needs a HIP device")
        L = N.lib()
        conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
        X = np.ascontiguousarray(mesh.X, dtype=np.float64)
        d = N.MeshDesc()
        d.elem_type = mesh.elem_type
        d.n_coef = mesh.n_coef
        d.n_elem = mesh.n_elem
        d.h_conn = conn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.h_X = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.gl = (ctypes.c_int32 * 3)(*mesh.gl)
        d.thickness = mesh.thickness
        d.width = getattr(mesh, "width", 0.0)
        d.material = material.kind
        p = list(material.params) + [0.0] * (3 - len(material.params))
        d.params = (ctypes.c_double * 3)(*p[:3])
        d.kv_eta = material.kv_eta
        d.kv_lambda = material.kv_lambda
        d.precision = _PREC[precision]
        h = ctypes.c_void_p()
        N.check(L.tlfea_mesh_create(ctypes.byref(d), ctypes.byref(h)), "tlfea_mesh_create")
        self._h = h
        self.mesh = mesh
        self.material = material
        self.precision = precision
        self.n_dof = mesh.n_dof
        self.n_elem = mesh.n_elem
        self.n_en = {N.TLFEA_T10: 10, N.TLFEA_ANCF3443: 16, N.TLFEA_ANCF3243: 8}[mesh.elem_type]
        self.nnz = -1

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            N.lib().tlfea_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- configuration
    def set_material(self, material: Material):
        p = list(material.params) + [0.0] * (3 - len(material.params))
        arr = (ctypes.c_double * 3)(*p[:3])
        N.check(N.lib().tlfea_mesh_set_material(self._h, material.kind, arr, material.kv_eta, material.kv_lambda),
                "tlfea_mesh_set_material")
        self.material = material

    def set_precision(self, precision: str):
        N.check(N.lib().tlfea_mesh_set_precision(self._h, _PREC[precision]), "tlfea_mesh_set_precision")
        self.precision = precision

    def info(self):
        """Sizes of the mesh: n_dof, n_elem, nnz (-1 before the pattern), n_en, n_qp."""
        n_dof, n_el, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        n_en, n_qp = ctypes.c_int32(), ctypes.c_int32()
        N.check(N.lib().tlfea_mesh_info(self._h, ctypes.byref(n_dof), ctypes.byref(n_el), ctypes.byref(nnz),
                                        ctypes.byref(n_en), ctypes.byref(n_qp)), "tlfea_mesh_info")
        return dict(n_dof=n_dof.value, n_elem=n_el.value, nnz=nnz.value, n_en=n_en.value, n_qp=n_qp.value)

    # -- pattern
    def build_pattern(self) -> int:
        """Build the CSR pattern, slot map and node ranges once (tlfea_build_csr_pattern); returns nnz."""
        nnz = ctypes.c_int64()
        N.check(N.lib().tlfea_build_csr_pattern(self._h, ctypes.byref(nnz)), "tlfea_build_csr_pattern")
        self.nnz = nnz.value
        return self.nnz

    def csr_pattern(self, on_device: bool = True):
        """(row_offsets, col_indices) of the pattern, int32, on the device or the host."""
        dev = "cuda" if on_device else "cpu"
        ro = torch.empty(self.n_dof + 1, dtype=torch.int32, device=dev)
        cols = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)[: self.nnz]
        N.check(N.lib().tlfea_get_csr_pattern(self._h, ctypes.c_void_p(ro.data_ptr()),
                                              ctypes.c_void_p(cols.data_ptr()), int(on_device), _stream()),
                "tlfea_get_csr_pattern")
        return ro, cols

    def slot_map(self, e0: int = 0, ne: Optional[int] = None, on_device: bool = True):
        """CSR position of every entry of the element matrices of elements [e0, e0 + ne), (ne, 3 n_en, 3 n_en) int32."""
        ne = self.n_elem - e0 if ne is None else ne
        nd = 3 * self.n_en
        dev = "cuda" if on_device else "cpu"
        out = torch.empty((ne, nd, nd), dtype=torch.int32, device=dev)
        N.check(N.lib().tlfea_get_slot_map(self._h, e0, ne, ctypes.c_void_p(out.data_ptr()), int(on_device),
                                           _stream()), "tlfea_get_slot_map")
        return out

    # -- compute
    def internal_force(self, q, qdot=None, out=None):
        """f_int(q, qdot) (qdot may be None: zero velocity), float64, n_dof."""
        out = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if out is None else out
        N.check(N.lib().tlfea_internal_force(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                             _ptr(out, n=self.n_dof), _stream()), "tlfea_internal_force")
        return out

    def internal_force_noalloc(self, q, qdot=None, out=None):
        """f_int(q, qdot) through the allocation-free entry point (the library
        allocates nothing; its fixed per-GPU work area is shared by every such
        call on the GPU, so overlapping calls race).  ``out`` is required."""
        if out is None:
            raise ValueError("internal_force_noalloc needs a caller-allocated output")
        N.check(N.lib().tlfea_internal_force_noalloc(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                                     _ptr(out, n=self.n_dof), _stream()),
                "tlfea_internal_force_noalloc")
        return out

    def tangent(self, q, qdot=None, h: float = 1.0, out=None, alpha=None, beta=None):
        """CSR values of alpha df/dq + beta df/dqdot, (alpha, beta) = (h, 1) unless given."""
        out = torch.empty(self.nnz, dtype=torch.float64, device=q.device) if out is None else out
        a = h if alpha is None else alpha
        b = 1.0 if beta is None else beta
        N.check(N.lib().tlfea_tangent_ex(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof), float(a),
                                         float(b), _ptr(out, n=self.nnz), _stream()), "tlfea_tangent_ex")
        return out

    def assemble(self, q, qdot=None, alpha: float = 1.0, beta: float = 1.0, f=None, vals=None):
        """f_int and the CSR values of alpha df/dq + beta df/dqdot in one call."""
        f = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if f is None else f
        vals = torch.empty(self.nnz, dtype=torch.float64, device=q.device) if vals is None else vals
        N.check(N.lib().tlfea_assemble_ex(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof), float(alpha),
                                          float(beta), _ptr(f, n=self.n_dof), _ptr(vals, n=self.nnz), _stream()),
                "tlfea_assemble_ex")
        return f, vals

    def assemble_accumulate(self, q, qdot=None, alpha: float = 1.0, beta: float = 1.0, f=None, vals=None):
        """As assemble, adding onto f and vals instead of overwriting them."""
        N.check(N.lib().tlfea_assemble_accumulate(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                                  float(alpha), float(beta), _ptr(f, n=self.n_dof),
                                                  _ptr(vals, n=self.nnz), _stream()), "tlfea_assemble_accumulate")
        return f, vals

    def assemble_points(self, q, qdot=None, alpha: float = 1.0, beta: float = 1.0, want_tangent: bool = True):
        """Pass 1 alone: the per-element work of an assembly into the mesh's work buffer."""
        N.check(N.lib().tlfea_assemble_points(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                              float(alpha), float(beta), int(want_tangent), _stream()),
                "tlfea_assemble_points")

    def assemble_nodes(self, f=None, vals=None, accumulate: bool = False):
        """Pass 2 alone: f and / or the CSR values from what the last pass 1 left."""
        N.check(N.lib().tlfea_assemble_nodes(self._h, _ptr(f, n=self.n_dof), _ptr(vals, n=self.nnz),
                                             int(accumulate), _stream()), "tlfea_assemble_nodes")
        return f, vals

    def vjp(self, q, qdot, w, want_q=True, want_qdot=True, want_params=True):
        """(df/dq)^T w, (df/dqdot)^T w and d(w.f)/d(p0, p1, p2, kv_eta, kv_lambda), float64."""
        dev = q.device
        gq = torch.empty(self.n_dof, dtype=torch.float64, device=dev) if want_q else None
        gqd = torch.empty(self.n_dof, dtype=torch.float64, device=dev) if want_qdot else None
        gp = torch.empty(5, dtype=torch.float64, device=dev) if want_params else None
        N.check(N.lib().tlfea_internal_force_vjp(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                                 _ptr(w, n=self.n_dof), _ptr(gq), _ptr(gqd), _ptr(gp), _stream()),
                "tlfea_internal_force_vjp")
        return gq, gqd, gp

    def internal_force_p(self, q, qdot, params, out=None):
        """f_int with the material constants taken from the device vector
        ``params`` = (p0, p1, p2, kv_eta, kv_lambda) (float64, 5, same GPU); the
        mesh's own constants are neither used nor changed, nothing synchronises."""
        out = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if out is None else out
        N.check(N.lib().tlfea_internal_force_p(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                               _ptr(params, n=5), _ptr(out, n=self.n_dof), _stream()),
                "tlfea_internal_force_p")
        return out

    def vjp_p(self, q, qdot, params, w, want_q=True, want_qdot=True, want_params=True):
        """vjp() at the device material vector ``params`` (see internal_force_p)."""
        dev = q.device
        gq = torch.empty(self.n_dof, dtype=torch.float64, device=dev) if want_q else None
        gqd = torch.empty(self.n_dof, dtype=torch.float64, device=dev) if want_qdot else None
        gp = torch.empty(5, dtype=torch.float64, device=dev) if want_params else None
        N.check(N.lib().tlfea_internal_force_vjp_p(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                                   _ptr(params, n=5), _ptr(w, n=self.n_dof), _ptr(gq), _ptr(gqd),
                                                   _ptr(gp), _stream()),
                "tlfea_internal_force_vjp_p")
        return gq, gqd, gp

    def build_upper_pattern(self) -> int:
        """Build the upper-triangle pattern (rows cut at the diagonal); returns nnz_upper."""
        n = ctypes.c_int64()
        N.check(N.lib().tlfea_build_upper_pattern(self._h, ctypes.byref(n)), "tlfea_build_upper_pattern")
        self.nnz_upper = n.value
        return n.value

    def csr_pattern_upper(self):
        """(row_offsets, col_indices) of the upper triangle, int32 host tensors."""
        ro = torch.empty(self.n_dof + 1, dtype=torch.int32)
        cols = torch.empty(max(self.nnz_upper, 1), dtype=torch.int32)
        N.check(N.lib().tlfea_get_csr_pattern_upper(self._h, ctypes.c_void_p(ro.data_ptr()),
                                                    ctypes.c_void_p(cols.data_ptr()), 0, None),
                "tlfea_get_csr_pattern_upper")
        return ro, cols[: self.nnz_upper]

    def assemble_upper(self, q, qdot=None, alpha: float = 1.0, beta: float = 1.0, f=None, vals=None):
        """f and the upper triangle of the (symmetric, undamped) tangent."""
        f = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if f is None else f
        vals = torch.empty(self.nnz_upper, dtype=torch.float64, device=q.device) if vals is None else vals
        N.check(N.lib().tlfea_assemble_upper(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof), float(alpha),
                                             float(beta), _ptr(f, n=self.n_dof), _ptr(vals, n=self.nnz_upper),
                                             _stream()), "tlfea_assemble_upper")
        return f, vals

    def adamw_solve(self, q_n, v_n, v, h: float, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
                    f_ext=None, max_iters=100, check_every=10, eps_in=0.0, eps_rel=0.0, q=None, work=None):
        """First-order inner solver of one time step (AdamW on the velocity); v is
        updated in place.  Returns (v, q, iterations, last ||g||, gradient)."""
        q = torch.empty_like(q_n) if q is None else q
        work = torch.empty(4 * self.n_dof, dtype=torch.float64, device=q_n.device) if work is None else work
        prm = N.AdamwParams(lr, beta1, beta2, eps, weight_decay)
        it, gn = ctypes.c_int32(), ctypes.c_double()
        N.check(N.lib().tlfea_adamw_solve(self._h, ctypes.byref(prm), float(h), _ptr(q_n, n=self.n_dof),
                                          _ptr(v_n, n=self.n_dof), _ptr(f_ext, n=self.n_dof), _ptr(v, n=self.n_dof),
                                          _ptr(q, n=self.n_dof), _ptr(work, n=4 * self.n_dof), int(max_iters),
                                          int(check_every), float(eps_in), float(eps_rel), ctypes.byref(it),
                                          ctypes.byref(gn), _stream()), "tlfea_adamw_solve")
        return v, q, it.value, gn.value, work[2 * self.n_dof: 3 * self.n_dof]

    def build_mass(self, density: float):
        """Consistent mass matrix (affine elements of any type), built once."""
        N.check(N.lib().tlfea_build_mass(self._h, float(density)), "tlfea_build_mass")

    def mass_values(self, out=None, device="cuda"):
        """M as DOF-level CSR values on the mesh pattern."""
        out = torch.empty(self.nnz, dtype=torch.float64, device=device) if out is None else out
        N.check(N.lib().tlfea_get_mass(self._h, _ptr(out, n=self.nnz), _stream()), "tlfea_get_mass")
        return out

    def assemble_newton(self, q, qdot, h: float, f=None, vals=None):
        """f_int and H = M/h + h df/dq + df/dqdot."""
        f = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if f is None else f
        vals = torch.empty(self.nnz, dtype=torch.float64, device=q.device) if vals is None else vals
        N.check(N.lib().tlfea_assemble_newton(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof), float(h),
                                              _ptr(f, n=self.n_dof), _ptr(vals, n=self.nnz), _stream()),
                "tlfea_assemble_newton")
        return f, vals

    def assemble_newton_upper(self, q, qdot, h: float, f=None, vals_upper=None):
        """f_int and the upper triangle of H = M/h + h df/dq (undamped materials)."""
        f = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if f is None else f
        n = self.nnz_upper
        vals_upper = torch.empty(n, dtype=torch.float64, device=q.device) if vals_upper is None else vals_upper
        N.check(N.lib().tlfea_assemble_newton_upper(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof),
                                                    float(h), _ptr(f, n=self.n_dof), _ptr(vals_upper, n=n),
                                                    _stream()), "tlfea_assemble_newton_upper")
        return f, vals_upper

    def newton_gradient(self, v, v_prev, f_int, f_ext, h: float, out=None):
        """g = M (v - v_prev)/h + f_int - f_ext (f_ext may be None)."""
        out = torch.empty(self.n_dof, dtype=torch.float64, device=v.device) if out is None else out
        N.check(N.lib().tlfea_newton_gradient(self._h, _ptr(v, n=self.n_dof), _ptr(v_prev, n=self.n_dof),
                                              _ptr(f_int, n=self.n_dof), _ptr(f_ext, n=self.n_dof), float(h),
                                              _ptr(out, n=self.n_dof), _stream()), "tlfea_newton_gradient")
        return out

    def set_gather_shape(self, waves: int, range_tasks: int, range_values: int):
        """Set the pass-2 launch shape (waves per workgroup, tasks and values per node range)."""
        sh = N.GatherShape(waves, range_tasks, range_values)
        N.check(N.lib().tlfea_mesh_set_gather_shape(self._h, ctypes.byref(sh)), "tlfea_mesh_set_gather_shape")

    def gather_shape(self):
        """(shape dict, number of node ranges)"""
        sh, n = N.GatherShape(), ctypes.c_int64()
        N.check(N.lib().tlfea_mesh_get_gather_shape(self._h, ctypes.byref(sh), ctypes.byref(n)),
                "tlfea_mesh_get_gather_shape")
        return sh.as_dict(), n.value

    def autotune(self, q, qdot=None, h: float = 1.0, f=None, vals=None, reps: int = 5):
        """Times the launch-shape grid on tlfea_assemble(q, qdot, h) and keeps the fastest;
        returns (shape dict, ms per call, f, vals) with f / vals holding its result."""
        f = torch.empty(self.n_dof, dtype=torch.float64, device=q.device) if f is None else f
        vals = torch.empty(self.nnz, dtype=torch.float64, device=q.device) if vals is None else vals
        sh, ms = N.GatherShape(), ctypes.c_float()
        N.check(N.lib().tlfea_mesh_autotune(self._h, _ptr(q, n=self.n_dof), _ptr(qdot, n=self.n_dof), float(h),
                                            _ptr(f, n=self.n_dof), _ptr(vals, n=self.nnz), int(reps), _stream(),
                                            ctypes.byref(sh), ctypes.byref(ms)), "tlfea_mesh_autotune")
        return sh.as_dict(), ms.value, f, vals

    def runtime_flags(self) -> int:
        """Flags raised since the last read (bit 0: det F <= 0, bit 1: non-finite stress); clears them."""
        fl = ctypes.c_uint32()
        N.check(N.lib().tlfea_get_runtime_flags(self._h, ctypes.byref(fl)), "tlfea_get_runtime_flags")
        return fl.value


class TLBatch:
    """Many bodies assembled by one launch (per-body CSR kept)."""

    def __init__(self, meshes: Sequence[TLMesh]):
        self.meshes = list(meshes)
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = ctypes.c_void_p()
        N.check(N.lib().tlfea_batch_create(arr, len(self.meshes), ctypes.byref(h)), "tlfea_batch_create")
        self._h = h
        n = len(self.meshes)
        dof = (ctypes.c_int64 * (n + 1))()
        nnz = (ctypes.c_int64 * (n + 1))()
        N.check(N.lib().tlfea_batch_offsets(self._h, dof, nnz), "tlfea_batch_offsets")
        self.dof_off = list(dof)
        self.nnz_off = list(nnz)

    def close(self):
        if getattr(self, "_h", None):
            N.lib().tlfea_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, q, qdot, h, f=None, vals=None, loop: bool = False):
        """f_int and h df/dq + df/dqdot of every body (h per body) in one graph-captured launch
        pair, or through per-body calls with loop=True."""
        nd, nz = self.dof_off[-1], self.nnz_off[-1]
        f = torch.empty(nd, dtype=torch.float64, device=q.device) if f is None else f
        vals = torch.empty(nz, dtype=torch.float64, device=q.device) if vals is None else vals
        fn = N.lib().tlfea_batch_assemble_loop if loop else N.lib().tlfea_batch_assemble
        N.check(fn(self._h, _ptr(q, n=nd), _ptr(qdot, n=nd), _ptr(h, n=len(self.meshes)), _ptr(f, n=nd),
                   _ptr(vals, n=nz), _stream()), "tlfea_batch_assemble")
        return f, vals

    def set_gather_shape(self, waves: int, range_tasks: int, range_values: int):
        sh = N.GatherShape(waves, range_tasks, range_values)
        N.check(N.lib().tlfea_batch_set_gather_shape(self._h, ctypes.byref(sh)), "tlfea_batch_set_gather_shape")

    def gather_shape(self):
        """(shape dict, number of node ranges over all bodies)"""
        sh, n = N.GatherShape(), ctypes.c_int64()
        N.check(N.lib().tlfea_batch_get_gather_shape(self._h, ctypes.byref(sh), ctypes.byref(n)),
                "tlfea_batch_get_gather_shape")
        return sh.as_dict(), n.value

    def set_schedule(self, persistent: bool, tile_elems: int = 25):
        """Persistent LPT schedule (tiles of tile_elems elements) or one workgroup per item."""
        N.check(N.lib().tlfea_batch_set_schedule(self._h, int(bool(persistent)), int(tile_elems)),
                "tlfea_batch_set_schedule")

    def schedule(self):
        """dict(persistent, tile_elems, grid_tiles, grid_ranges)"""
        v = [ctypes.c_int32() for _ in range(4)]
        N.check(N.lib().tlfea_batch_get_schedule(self._h, *[ctypes.byref(x) for x in v]), "tlfea_batch_get_schedule")
        return dict(zip(("persistent", "tile_elems", "grid_tiles", "grid_ranges"), [x.value for x in v]))

    def autotune(self, q, qdot, h, f=None, vals=None, reps: int = 5):
        """Times every schedule and launch shape on the batched launch pair and keeps the
        fastest; returns (shape dict, ms per call, f, vals) with f / vals holding its result
        (schedule() tells the schedule kept)."""
        nd, nz = self.dof_off[-1], self.nnz_off[-1]
        f = torch.empty(nd, dtype=torch.float64, device=q.device) if f is None else f
        vals = torch.empty(nz, dtype=torch.float64, device=q.device) if vals is None else vals
        sh, ms = N.GatherShape(), ctypes.c_float()
        N.check(N.lib().tlfea_batch_autotune(self._h, _ptr(q, n=nd), _ptr(qdot, n=nd), _ptr(h, n=len(self.meshes)),
                                             _ptr(f, n=nd), _ptr(vals, n=nz), int(reps), _stream(),
                                             ctypes.byref(sh), ctypes.byref(ms)), "tlfea_batch_autotune")
        return sh.as_dict(), ms.value, f, vals
