"""GPU checks of the VJP kernel, the autograd wrapper and the batched launch."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd.api import TLBatch, TLMesh
from paper_2604_10357_amd.autograd import internal_force, material_vector
from tests.gpu_util import cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu

VJP_CASES = [
    ("t10_mr_kv", W.t10_beam(3, 2, 2, 21, "t10_mr_kv", lx=0.3, ly=0.2, lz=0.2)),
    ("t10_svk_kv", W.t10_beam(2, 2, 1, 22, "t10_svk_kv", lx=0.2, ly=0.2, lz=0.1,
                              material=W.Material(W.SVK, (1e7, 0.3, 0.0), 2e3, 1e3))),
    ("ancf_svk", W.shell_plate(3, 23, "ancf", thickness=0.02)),
]


@pytest.mark.parametrize("name,wl", VJP_CASES, ids=[c[0] for c in VJP_CASES])
def test_vjp_against_oracle(name, wl):
    print(f"[gpu] vjp {name}", flush=True)
    m = make_mesh(wl)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    gq_ref, gqd_ref, gp_ref = oracle.vjp(om, omat, wl.q, wl.qdot, wl.w)
    gq, gqd, gp = m.vjp(cuda(wl.q), cuda(wl.qdot), cuda(wl.w))
    # fixed-order sums: a second call gives the same bits
    gq2, gqd2, gp2 = m.vjp(cuda(wl.q), cuda(wl.qdot), cuda(wl.w))
    assert torch.equal(gq, gq2) and torch.equal(gqd, gqd2) and torch.equal(gp, gp2)
    assert rel_err(gq.cpu().numpy(), gq_ref)[0] <= 1e-12
    if np.abs(gqd_ref).max() > 0:
        assert rel_err(gqd.cpu().numpy(), gqd_ref)[0] <= 1e-12
    gp = gp.cpu().numpy()
    for i in range(5):
        if gp_ref[i] != 0.0:
            assert abs(gp[i] - gp_ref[i]) <= 1e-11 * abs(gp_ref[i]), (i, gp[i], gp_ref[i])
    # transpose of the GPU tangent applied to w
    q, qd, w = cuda(wl.q), cuda(wl.qdot), cuda(wl.w)
    vals = m.tangent(q, qd, alpha=1.0, beta=0.0).cpu().numpy()
    ro, cols = m.csr_pattern(on_device=False)
    ro, cols = ro.numpy(), cols.numpy()
    KTw = np.zeros(m.n_dof)
    rows = np.repeat(np.arange(m.n_dof), np.diff(ro))
    np.add.at(KTw, cols, vals * wl.w[rows])
    assert rel_err(gq.cpu().numpy(), KTw)[0] <= 1e-12
    m.close()


def test_autograd_function_gradients():
    wl = VJP_CASES[0][1]
    m = make_mesh(wl)
    q = cuda(wl.q).requires_grad_(True)
    qd = cuda(wl.qdot).requires_grad_(True)
    p = material_vector(wl.material, "cuda").requires_grad_(True)
    w = cuda(wl.w)
    f = internal_force(m, q, qd, p)
    (f * w).sum().backward()
    om = oracle.Mesh.of(wl.mesh)
    gq_ref, gqd_ref, gp_ref = oracle.vjp(om, oracle.material_of(wl.material), wl.q, wl.qdot, wl.w)
    assert rel_err(q.grad.cpu().numpy(), gq_ref)[0] <= 1e-12
    assert rel_err(qd.grad.cpu().numpy(), gqd_ref)[0] <= 1e-12
    assert rel_err(p.grad.cpu().numpy(), gp_ref)[0] <= 1e-11
    # directional central difference on the FP64 path
    v = torch.from_numpy(np.random.default_rng(3).normal(size=wl.q.shape)).cuda()
    eps = 1e-6
    with torch.no_grad():
        fp = m.internal_force(q.detach() + eps * v, qd.detach())
        fm = m.internal_force(q.detach() - eps * v, qd.detach())
    fd = float(((fp - fm) / (2 * eps) * w).sum())
    an = float((q.grad * v).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)
    m.close()


@pytest.mark.parametrize("case", [0, 1], ids=["mr_kv", "svk_kv"])
def test_autograd_device_parameters_leave_the_mesh_material(case):
    """The autograd forward and backward read the material vector on the GPU:
    at constants other than the mesh's (x1.1 each) they match the oracle at
    those constants, the mesh's own material is unchanged afterwards, and only
    the requested gradients are formed."""
    print(f"[gpu] autograd device params {case}", flush=True)
    wl = VJP_CASES[case][1]
    m = make_mesh(wl)
    base = material_vector(wl.material, "cuda")
    p = (base * 1.1).requires_grad_(True)
    q = cuda(wl.q).requires_grad_(True)
    qd = cuda(wl.qdot)
    f = internal_force(m, q, qd, p)
    (f * cuda(wl.w)).sum().backward()
    pv = (base * 1.1).cpu().tolist()
    mat2 = W.Material(wl.material.kind, tuple(pv[:3]) if wl.material.kind == W.MOONEY_RIVLIN else (pv[0], pv[1], 0.0),
                      pv[3], pv[4])
    om = oracle.Mesh.of(wl.mesh)
    f_ref, _ = oracle.assemble(om, oracle.material_of(mat2), wl.q, wl.qdot, want_K=False)
    gq_ref, _, gp_ref = oracle.vjp(om, oracle.material_of(mat2), wl.q, wl.qdot, wl.w)
    assert rel_err(f.detach().cpu().numpy(), f_ref)[0] <= 1e-12
    assert rel_err(q.grad.cpu().numpy(), gq_ref)[0] <= 1e-12
    gp = p.grad.cpu().numpy()
    for i in range(5):
        if gp_ref[i] != 0.0:
            assert abs(gp[i] - gp_ref[i]) <= 1e-11 * abs(gp_ref[i]), (i, gp[i], gp_ref[i])
    # the mesh still computes with its own constants
    f0_ref, _ = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, want_K=False)
    assert rel_err(m.internal_force(cuda(wl.q), qd).cpu().numpy(), f0_ref)[0] <= 1e-12
    m.close()


def test_vjp_config5_fd_and_transpose():
    """Large T10 beam: VJP against a directional central difference (step 1e-6,
    FP64 path) and against the transpose of the GPU tangent."""
    print("[gpu] vjp config5", flush=True)
    wl = W.config5()
    m = make_mesh(wl, "fp64")
    q, qd, w = cuda(wl.q), cuda(wl.qdot), cuda(wl.w)
    gq, gqd, gp = m.vjp(q, qd, w)
    v = torch.from_numpy(np.random.default_rng(4).normal(size=wl.q.shape)).cuda()

    def cdiff(eps):
        return float(((m.internal_force(q + eps * v, qd) - m.internal_force(q - eps * v, qd)) / (2 * eps) * w).sum())

    # the stated step 1e-6 is 2e-4 of the 5 mm cell: its truncation error is
    # O((eps / h)^2) ~ 1e-6 relative; Richardson extrapolation with eps / 2
    # removes that term
    fd1, fd2 = cdiff(1e-6), cdiff(5e-7)
    fdr = (4.0 * fd2 - fd1) / 3.0
    an = float((gq * v).sum())
    print(f"  fd(1e-6) {fd1:.9e} richardson {fdr:.9e} vjp {an:.9e}", flush=True)
    assert abs(fd1 - an) <= 1e-5 * abs(an)
    assert abs(fdr - an) <= 1e-7 * abs(an)
    vals = m.tangent(q, qd, alpha=1.0, beta=0.0)
    ro, cols = m.csr_pattern(on_device=True)
    rows = torch.repeat_interleave(torch.arange(m.n_dof, device="cuda"), (ro[1:] - ro[:-1]).long())
    KTw = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    KTw.index_add_(0, cols.long(), vals * w[rows])
    assert rel_err(gq.cpu().numpy(), KTw.cpu().numpy())[0] <= 1e-12
    # parameter gradient of Mooney-Rivlin constants vs central differences
    base = [wl.material.params[0], wl.material.params[1], wl.material.params[2]]
    for i in range(3):
        hstep = 1e-6 * base[i]
        up, dn = list(base), list(base)
        up[i] += hstep
        dn[i] -= hstep
        m.set_material(W.Material(W.MOONEY_RIVLIN, tuple(up), wl.material.kv_eta, wl.material.kv_lambda))
        fu = m.internal_force(q, qd)
        m.set_material(W.Material(W.MOONEY_RIVLIN, tuple(dn), wl.material.kv_eta, wl.material.kv_lambda))
        fdn = m.internal_force(q, qd)
        fdp = float(((fu - fdn) * w).sum()) / (2 * hstep)
        assert abs(fdp - float(gp[i])) <= 1e-6 * abs(fdp), (i, fdp, float(gp[i]))
    m.close()


def batch_workloads(n=12, seed=31):
    return W.batched_bodies(n, seed, n_lo=1, n_hi=4)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_oracle_and_loop(precision):
    print(f"[gpu] batch {precision}", flush=True)
    wls = batch_workloads()
    meshes = [make_mesh(wl, precision) for wl in wls]
    b = TLBatch(meshes)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    hs = np.linspace(1e-3, 2e-3, len(wls))
    h = cuda(hs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = [b.assemble(q, qd, h) for _ in range(3)]   # graph captured once, replayed
        f_loop, v_loop = b.assemble(q, qd, h, loop=True)
    stream.synchronize()
    f, vals = outs[-1]
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k, wl in enumerate(wls):
        d0, d1 = b.dof_off[k], b.dof_off[k + 1]
        z0, z1 = b.nnz_off[k], b.nnz_off[k + 1]
        om = oracle.Mesh.of(wl.mesh)
        f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, hs[k], 1.0)
        assert rel_err(f[d0:d1].cpu().numpy(), f_ref)[0] <= tol, k
        assert rel_err(vals[z0:z1].cpu().numpy(), v_ref)[0] <= tol, k
    for fo, vo in outs[:-1]:
        assert torch.equal(fo, f) or rel_err(fo.cpu().numpy(), f.cpu().numpy())[0] <= 1e-14
    assert rel_err(f_loop.cpu().numpy(), f.cpu().numpy())[0] <= 1e-13
    assert rel_err(v_loop.cpu().numpy(), vals.cpu().numpy())[0] <= 1e-13
    b.close()
    for m in meshes:
        m.close()


def test_batch_refuses_members_changed_after_creation():
    """A batch copies its members' pattern arrays, materials and precision:
    after a member's material, precision or pattern changes, the graph and loop
    forms both refuse to run (instead of reading freed arrays or disagreeing)."""
    from paper_2604_10357_amd._native import TlfeaError
    print("[gpu] stale batch", flush=True)
    wls = batch_workloads(4, 37)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    h = cuda(np.full(len(wls), 1e-3))
    for change in ("material", "precision", "pattern"):
        meshes = [make_mesh(wl, "mixed") for wl in wls]
        b = TLBatch(meshes)
        b.assemble(q, qd, h)  # fine before the change
        if change == "material":
            meshes[1].set_material(W.Material(W.SVK, (2e6, 0.3, 0.0), 0.0, 0.0))
        elif change == "precision":
            meshes[2].set_precision("fp64")
        else:
            meshes[3].build_pattern()
        for loop in (False, True):
            with pytest.raises(TlfeaError) as e:
                b.assemble(q, qd, h, loop=loop)
            assert e.value.status == -1
        b.close()
        for m in meshes:
            m.close()


@pytest.mark.parametrize("tile_elems", [25, 16])
def test_batch_persistent_lpt_schedule(tile_elems):
    """The persistent LPT schedule (work counters, longest items first) against
    the oracle body by body and against the one-workgroup-per-item schedule,
    over graph replays; the counters restart on every call."""
    print(f"[gpu] batch persistent {tile_elems}", flush=True)
    wls = batch_workloads(14, 41)
    meshes = [make_mesh(wl, "mixed") for wl in wls]
    b = TLBatch(meshes)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    hs = np.linspace(1e-3, 2e-3, len(wls))
    h = cuda(hs)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        f0, v0 = b.assemble(q, qd, h)  # one workgroup per item
        b.set_schedule(True, tile_elems)
        sch = b.schedule()
        outs = [b.assemble(q, qd, h) for _ in range(3)]  # captured once, replayed
    stream.synchronize()
    assert sch["persistent"] == 1 and sch["tile_elems"] == tile_elems
    assert 1 <= sch["grid_tiles"] and 1 <= sch["grid_ranges"]
    for f, v in outs:
        assert rel_err(f.cpu().numpy(), f0.cpu().numpy())[0] <= 1e-13
        assert rel_err(v.cpu().numpy(), v0.cpu().numpy())[0] <= 1e-13
    f, vals = outs[-1]
    for k, wl in enumerate(wls):
        d0, d1 = b.dof_off[k], b.dof_off[k + 1]
        z0, z1 = b.nnz_off[k], b.nnz_off[k + 1]
        om = oracle.Mesh.of(wl.mesh)
        f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, hs[k], 1.0)
        assert rel_err(f[d0:d1].cpu().numpy(), f_ref)[0] <= 1e-5, k
        assert rel_err(vals[z0:z1].cpu().numpy(), v_ref)[0] <= 1e-5, k
    b.set_schedule(False)
    assert b.schedule()["persistent"] == 0
    b.close()
    for m in meshes:
        m.close()


def test_batch_autotune_caches_its_choice():
    """The autotuner times every schedule and shape, keeps the fastest, and a
    batch created later over bodies of the same sizes starts with that choice."""
    print("[gpu] batch autotune cache", flush=True)
    wls = batch_workloads(10, 43)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    h = cuda(np.full(len(wls), 1e-3))
    meshes = [make_mesh(wl, "mixed") for wl in wls]
    b = TLBatch(meshes)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        shape, ms, f_t, v_t = b.autotune(q, qd, h, reps=2)
        chosen = b.schedule()
        f1, v1 = b.assemble(q, qd, h)
    stream.synchronize()
    assert ms > 0
    assert rel_err(f1.cpu().numpy(), f_t.cpu().numpy())[0] <= 1e-13
    meshes2 = [make_mesh(wl, "mixed") for wl in wls]
    b2 = TLBatch(meshes2)
    assert b2.schedule()["persistent"] == chosen["persistent"]
    assert b2.schedule()["tile_elems"] == chosen["tile_elems"]
    assert b2.gather_shape()[0] == shape
    for obj in [b, b2] + meshes + meshes2:
        obj.close()
