"""GPU checks of the pass-2 launch shapes and their autotuners: every shape
gives the oracle's result, the autotuners pick a shape of the grid and leave
its result in the outputs, and a batch re-captures its graph after a change."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd._native import TlfeaError
from paper_2604_10357_amd.api import TLBatch
from tests.gpu_util import TOL, cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu

GRID = {(w, t, v) for w in (2, 4, 8) for t in (384, 768, 1536) for v in (2048, 4096, 8192)}
SHAPES = [(1, 9, 1), (2, 384, 2048), (8, 1536, 8192), (3, 100, 700), (4, 768, 4096)]


def shape_tuple(d):
    return d["waves"], d["range_tasks"], d["range_values"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", [
    ("t10_3x2x2_mr_kv", W.t10_beam(3, 2, 2, 41, "t10_3x2x2_mr_kv", lx=0.3, ly=0.2, lz=0.2)),
    ("ancf_4x3_332", W.shell_plate(4, 42, "ancf_4x3", thickness=0.02)),
], ids=["t10", "ancf"])
def test_every_shape_matches_oracle(name, wl, precision):
    print(f"[gpu] shapes {name} {precision}", flush=True)
    m = make_mesh(wl, precision)
    om = oracle.Mesh.of(wl.mesh)
    h = 1e-3
    f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, h, 1.0)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    for sh in SHAPES:
        m.set_gather_shape(*sh)
        got, n_ranges = m.gather_shape()
        assert shape_tuple(got) == sh
        if sh == (1, 9, 1):  # caps below one node: one range per pattern node
            assert n_ranges == int(wl.mesh.conn.max()) + 1
        f, vals = m.assemble(q, qd, h, 1.0)
        assert rel_err(f.cpu().numpy(), f_ref)[0] <= TOL[precision], sh
        assert rel_err(vals.cpu().numpy(), v_ref)[0] <= TOL[precision], sh
        # the force-only and tangent-only passes use the same ranges
        fo = m.internal_force(q, qd)
        assert rel_err(fo.cpu().numpy(), f_ref)[0] <= TOL[precision], sh
    m.close()


def test_shape_errors_leave_the_mesh_unchanged():
    print("[gpu] shape errors", flush=True)
    wl = W.shell_plate(4, 43, "ancf_4x3", thickness=0.02)
    m = make_mesh(wl, "mixed")
    before = m.gather_shape()
    for bad in [(0, 768, 4096), (9, 768, 4096), (4, 0, 4096), (4, 768, 0)]:
        with pytest.raises(TlfeaError) as e:
            m.set_gather_shape(*bad)
        assert e.value.status == -1
    # ANCF nodes hold 1,308 LDS values each: 64-node ranges need 654 KiB
    with pytest.raises(TlfeaError) as e:
        m.set_gather_shape(4, 1 << 20, 1 << 20)
    assert e.value.status == -2
    assert m.gather_shape() == before
    m.close()


def test_mesh_autotune_config2():
    """The T10 box of 30,720 elements, mixed: the tuned shape is one of the grid,
    the outputs hold its result, and later calls use it."""
    print("[gpu] mesh autotune config2", flush=True)
    wl = W.config2()
    m = make_mesh(wl, "mixed")
    q, qd = cuda(wl.q), cuda(wl.qdot)
    h = 1e-3
    f0, v0 = m.assemble(q, qd, h, 1.0)
    f0, v0 = f0.cpu().numpy(), v0.cpu().numpy()
    shape, ms, f, vals = m.autotune(q, qd, h, reps=3)
    print(f"  chosen {shape} {ms:.3f} ms", flush=True)
    assert shape_tuple(shape) in GRID and ms > 0
    assert m.gather_shape()[0] == shape
    torch.cuda.synchronize()
    assert rel_err(f.cpu().numpy(), f0)[0] <= 1e-13
    assert rel_err(vals.cpu().numpy(), v0)[0] <= 1e-13
    f2, v2 = m.assemble(q, qd, h, 1.0)
    assert rel_err(f2.cpu().numpy(), f0)[0] <= 1e-13
    assert rel_err(v2.cpu().numpy(), v0)[0] <= 1e-13
    f_ref, v_ref = oracle.assemble(oracle.Mesh.of(wl.mesh), oracle.material_of(wl.material), wl.q, wl.qdot, h,
                                   1.0)
    assert rel_err(f0, f_ref)[0] <= TOL["mixed"] and rel_err(v0, v_ref)[0] <= TOL["mixed"]
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_autotune_and_graph_recapture(precision):
    print(f"[gpu] batch autotune {precision}", flush=True)
    wls = W.batched_bodies(10, 51, n_lo=1, n_hi=4)
    meshes = [make_mesh(wl, precision) for wl in wls]
    b = TLBatch(meshes)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    hs = np.linspace(1e-3, 2e-3, len(wls))
    h = cuda(hs)
    f_loop, v_loop = b.assemble(q, qd, h, loop=True)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        f_pre, v_pre = torch.empty_like(f_loop), torch.empty_like(v_loop)
        b.assemble(q, qd, h, f=f_pre, vals=v_pre)                   # graph captured with the first shape
        shape, ms, f_t, v_t = b.autotune(q, qd, h, reps=2)
        b.assemble(q, qd, h, f=f_pre, vals=v_pre)                   # same pointers: captured again
        b.set_gather_shape(1, 9, 1)
        f_one, v_one = torch.empty_like(f_loop), torch.empty_like(v_loop)
        b.assemble(q, qd, h, f=f_one, vals=v_one)
        b.assemble(q, qd, h, f=f_one, vals=v_one)                   # replay
    stream.synchronize()
    print(f"  chosen {shape} {ms:.3f} ms", flush=True)
    assert shape_tuple(shape) in GRID and ms > 0
    assert b.gather_shape()[1] == sum(int(wl.mesh.conn.max()) + 1 for wl in wls)
    fl, vl = f_loop.cpu().numpy(), v_loop.cpu().numpy()
    for f, v in [(f_t, v_t), (f_pre, v_pre), (f_one, v_one)]:
        assert rel_err(f.cpu().numpy(), fl)[0] <= 1e-13
        assert rel_err(v.cpu().numpy(), vl)[0] <= 1e-13
    tol = TOL[precision]
    for k in (0, len(wls) - 1):
        wl = wls[k]
        d0, d1 = b.dof_off[k], b.dof_off[k + 1]
        z0, z1 = b.nnz_off[k], b.nnz_off[k + 1]
        f_ref, v_ref = oracle.assemble(oracle.Mesh.of(wl.mesh), oracle.material_of(wl.material), wl.q, wl.qdot,
                                       hs[k], 1.0)
        assert rel_err(fl[d0:d1], f_ref)[0] <= tol
        assert rel_err(vl[z0:z1], v_ref)[0] <= tol
    # the bodies keep their own shapes (the default of their precision)
    default = (4, 768, 2048) if precision == "mixed" else (4, 768, 4096)
    assert all(shape_tuple(mm.gather_shape()[0]) == default for mm in meshes)
    b.close()
    for mm in meshes:
        mm.close()
