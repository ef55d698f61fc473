"""The allocation-free force entry point (tlfea_internal_force_noalloc) against
tlfea_internal_force, which it must reproduce bit for bit (same kernels, same
fixed summation order), and against the FP64 oracle at the precision's bar.

Two calls in a row through the fixed per-GPU work area, the second on a
smaller mesh (the area keeps the first call's blocks: the second must not
read them), in both precisions; a mesh whose blocks exceed the area is
rejected before any work."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd._native import TlfeaError
from tests.gpu_util import TOL, cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu

SCRATCH = 64 * 1024 * 1024


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_force_matches_allocating_call(precision):
    print(f"[gpu] noalloc force {precision}", flush=True)
    big = W.t10_beam(40, 8, 8, 3101, "t10_40x8x8", lx=0.5)            # 15,360 elements
    small = W.t10_beam(7, 3, 2, 3102, "t10_7x3x2", lx=0.35, ly=0.15)  # 252 elements
    shell = W.shell_plate(6, 3103, "ancf_6x6", thickness=0.02)
    for wl in (big, small, shell):
        m = make_mesh(wl, precision)
        q, qd = cuda(wl.q), cuda(wl.qdot)
        f_ref, _ = oracle.assemble(oracle.Mesh.of(wl.mesh), oracle.material_of(wl.material), wl.q, wl.qdot,
                                   want_K=False)
        f_alloc = m.internal_force(q, qd)
        out = torch.full((m.n_dof,), float("nan"), dtype=torch.float64, device="cuda")
        m.internal_force_noalloc(q, qd, out=out)
        torch.cuda.synchronize()
        e = rel_err(out.cpu().numpy(), f_ref)[0]
        print(f"  {wl.name}: err {e:.2e}", flush=True)
        assert torch.equal(out, f_alloc)
        assert e <= TOL[precision]
        # zero velocity through a null pointer, second call into the same area
        out0 = torch.full((m.n_dof,), float("nan"), dtype=torch.float64, device="cuda")
        m.internal_force_noalloc(q, None, out=out0)
        assert torch.equal(out0, m.internal_force(q, None))
        m.close()


def test_noalloc_rejects_meshes_beyond_the_work_area():
    print("[gpu] noalloc size limit", flush=True)
    wl = W.t10_beam(100, 20, 24, 3104, "t10_100x20x24", frac=0.0, vel_sigma=0.0)  # 288,000 elements
    assert wl.mesh.n_elem * 10 * 3 * 8 > SCRATCH >= wl.mesh.n_elem * 10 * 3 * 4
    m = make_mesh(wl, "fp64")
    q = cuda(wl.q)
    out = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(TlfeaError) as e:
        m.internal_force_noalloc(q, None, out=out)
    assert e.value.status == -7
    assert torch.count_nonzero(out).item() == 0  # nothing written
    m.set_precision("mixed")  # 4-byte blocks fit
    m.internal_force_noalloc(q, None, out=out)
    assert torch.equal(out, m.internal_force(q, None))
    m.close()


def test_noalloc_needs_the_pattern():
    from paper_2604_10357_amd.api import TLMesh
    wl = W.config1()
    m = TLMesh(wl.mesh, wl.material, "fp64")
    out = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(TlfeaError) as e:
        m.internal_force_noalloc(cuda(wl.q), None, out=out)
    assert e.value.status == -6
    m.close()
