"""Edge cases of the HIP path against the oracle, through the C ABI: nodes that
no element uses (empty CSR rows, zero forces, no mass), meshes without
elements, and the split / accumulating forms of the second pass, for every
element type and both precisions."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from tests.gpu_util import TOL, cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu


def bases():
    return [("t10", W.t10_beam(2, 1, 1, 61, "t10", lx=0.2, ly=0.1, lz=0.1)),
            ("shell", W.shell_plate(2, 62, "shell", thickness=0.02)),
            ("beam", W.beam_3243(3, 63, "beam"))]


def with_isolated(wl, extra=2):
    """The same body plus `extra` pattern nodes that no element references."""
    m = wl.mesh
    mc = 1 if m.elem_type == W.T10 else 4
    rng = np.random.default_rng(64)
    Xe = rng.normal(5.0, 0.1, (extra * mc, 3))
    q = np.concatenate([wl.q, Xe.ravel() + 0.01])
    qd = np.concatenate([wl.qdot, rng.normal(0, 0.05, Xe.size)])
    mesh = W.Mesh(m.elem_type, np.vstack([m.X, Xe]), m.conn, m.gl, m.thickness, getattr(m, "width", 0.0))
    return W.Workload(wl.name + "_iso", mesh, wl.material, q, qd, None)


CASES = bases()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,base", CASES, ids=[c[0] for c in CASES])
def test_isolated_nodes(name, base, precision):
    print(f"[gpu] isolated nodes {name} {precision}", flush=True)
    wl = with_isolated(base)
    m = make_mesh(wl, precision)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    ro_ref, cols_ref = oracle.csr_pattern(om)
    ro, cols = m.csr_pattern(on_device=False)
    assert np.array_equal(ro.numpy(), ro_ref) and np.array_equal(cols.numpy(), cols_ref)
    n0 = base.mesh.n_dof
    assert np.all(np.diff(ro_ref)[n0:] == 0)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f, vals = m.assemble(q, qd, 1e-3, 1.0)
    f_ref, v_ref = oracle.assemble(om, omat, wl.q, wl.qdot, 1e-3, 1.0, pattern=(ro_ref, cols_ref))
    fh = f.cpu().numpy()
    assert np.all(fh[n0:] == 0.0)
    assert rel_err(fh, f_ref)[0] <= TOL[precision]
    assert rel_err(vals.cpu().numpy(), v_ref)[0] <= TOL[precision]
    fo = m.internal_force(q, qd).cpu().numpy()
    assert np.all(fo[n0:] == 0.0) and rel_err(fo, f_ref)[0] <= TOL[precision]
    # mass and gradient: isolated nodes have no mass rows, so g = f_int - f_ext there
    m.build_mass(1000.0)
    mv = m.mass_values().cpu().numpy()
    assert rel_err(mv, oracle.mass_csr(om, 1000.0, (ro_ref, cols_ref)))[0] <= 1e-13
    g = m.newton_gradient(qd, torch.zeros_like(qd), f, None, 1e-3).cpu().numpy()
    assert np.array_equal(g[n0:], fh[n0:])
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,base", CASES, ids=[c[0] for c in CASES])
def test_mesh_without_elements(name, base, precision):
    print(f"[gpu] no elements {name} {precision}", flush=True)
    b = base.mesh
    mesh = W.Mesh(b.elem_type, b.X, b.conn[:0].copy(), b.gl, b.thickness, getattr(b, "width", 0.0))
    wl = W.Workload("empty", mesh, base.material, base.q, base.qdot, None)
    m = make_mesh(wl, precision)
    assert m.nnz == 0
    ro, _ = m.csr_pattern(on_device=False)
    assert np.all(ro.numpy() == 0)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f = torch.full((m.n_dof,), 7.0, dtype=torch.float64, device="cuda")
    m.assemble(q, qd, 1e-3, 1.0, f=f)
    assert torch.count_nonzero(f).item() == 0
    fo = m.internal_force(q, qd)
    assert torch.count_nonzero(fo).item() == 0
    m.close()


SPLIT_CASES = [("t10", W.t10_beam(3, 2, 2, 65, "t10", lx=0.3, ly=0.2, lz=0.2)),
               ("shell", W.shell_plate(3, 66, "shell", thickness=0.02)),
               ("beam", W.beam_3243(11, 67, "beam"))]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", SPLIT_CASES, ids=[c[0] for c in SPLIT_CASES])
def test_split_and_accumulate_every_path(name, wl, precision):
    """Pass 2 alone with f only, with K only and accumulating onto existing
    values, after one pass 1 with the tangent: the same results as the fused
    call on every element type and precision (element rows in mixed
    precision, point records in FP64)."""
    print(f"[gpu] split / accumulate {name} {precision}", flush=True)
    m = make_mesh(wl, precision)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f, vals = m.assemble(q, qd, 2e-3, 1.0)
    m.assemble_points(q, qd, 2e-3, 1.0, want_tangent=True)
    f1 = torch.empty_like(f)
    m.assemble_nodes(f1, None)
    v1 = torch.empty_like(vals)
    m.assemble_nodes(None, v1)
    assert rel_err(f1.cpu().numpy(), f.cpu().numpy())[0] <= 1e-14
    assert rel_err(v1.cpu().numpy(), vals.cpu().numpy())[0] <= 1e-13
    base_f = torch.linspace(-1, 1, m.n_dof, dtype=torch.float64, device="cuda")
    base_v = torch.linspace(2, 3, m.nnz, dtype=torch.float64, device="cuda")
    f2, v2 = base_f.clone(), base_v.clone()
    m.assemble_nodes(f2, v2, accumulate=True)
    assert rel_err((f2 - base_f).cpu().numpy(), f.cpu().numpy())[0] <= 1e-12
    assert rel_err((v2 - base_v).cpu().numpy(), vals.cpu().numpy())[0] <= 1e-12
    f3, v3 = base_f.clone(), base_v.clone()
    m.assemble_accumulate(q, qd, 2e-3, 1.0, f3, v3)
    assert rel_err((f3 - base_f).cpu().numpy(), f.cpu().numpy())[0] <= 1e-12
    assert rel_err((v3 - base_v).cpu().numpy(), vals.cpu().numpy())[0] <= 1e-12
    # and the fused result against the oracle
    om = oracle.Mesh.of(wl.mesh)
    f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, 2e-3, 1.0)
    assert rel_err(f.cpu().numpy(), f_ref)[0] <= TOL[precision]
    assert rel_err(vals.cpu().numpy(), v_ref)[0] <= TOL[precision]
    m.close()


@pytest.mark.parametrize("gl", [(3, 3, 2), (4, 4, 3)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shell_batch(precision, gl):
    """Shells of different sizes in one batched launch (point records for
    every precision), against the oracle body by body."""
    from paper_2604_10357_amd.api import TLBatch
    print(f"[gpu] shell batch {gl} {precision}", flush=True)
    wls = [W.shell_plate(n, 70 + n, f"s{n}", thickness=0.02, gl=gl) for n in (2, 4, 1, 3)]
    meshes = [make_mesh(wl, precision) for wl in wls]
    b = TLBatch(meshes)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    hs = np.linspace(1e-3, 2e-3, len(wls))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        f, vals = b.assemble(q, qd, cuda(hs))
    stream.synchronize()
    for k, wl in enumerate(wls):
        d0, d1 = b.dof_off[k], b.dof_off[k + 1]
        z0, z1 = b.nnz_off[k], b.nnz_off[k + 1]
        om = oracle.Mesh.of(wl.mesh)
        f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, hs[k], 1.0)
        assert rel_err(f[d0:d1].cpu().numpy(), f_ref)[0] <= TOL[precision], k
        assert rel_err(vals[z0:z1].cpu().numpy(), v_ref)[0] <= TOL[precision], k
    b.close()
    for m in meshes:
        m.close()


def test_vjp_damped_shell_443():
    """The backward product on the 4x4x3 shell with Kelvin-Voigt damping
    (cotangents for q, qdot and the material constants) against the oracle."""
    print("[gpu] vjp shell 443 kv", flush=True)
    wl = W.shell_plate(3, 75, "s443", thickness=0.02, gl=(4, 4, 3))
    wl.material = W.Material(W.SVK, (2e9, 0.3, 0.0), 5e3, 5e3)
    rng = np.random.default_rng(76)
    wl.qdot = rng.normal(0, 0.05, wl.q.shape)
    wl.w = rng.normal(0, 1.0, wl.q.shape)
    m = make_mesh(wl, "fp64")
    om = oracle.Mesh.of(wl.mesh)
    gq_ref, gqd_ref, gp_ref = oracle.vjp(om, oracle.material_of(wl.material), wl.q, wl.qdot, wl.w)
    gq, gqd, gp = m.vjp(cuda(wl.q), cuda(wl.qdot), cuda(wl.w))
    assert rel_err(gq.cpu().numpy(), gq_ref)[0] <= 1e-12
    assert np.abs(gqd_ref).max() > 0 and rel_err(gqd.cpu().numpy(), gqd_ref)[0] <= 1e-12
    gp = gp.cpu().numpy()
    for i in range(5):
        if gp_ref[i] != 0.0:
            assert abs(gp[i] - gp_ref[i]) <= 1e-11 * abs(gp_ref[i]), (i, gp[i], gp_ref[i])
    m.close()
