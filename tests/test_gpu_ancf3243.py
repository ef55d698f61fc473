"""Parity of the ANCF3243 beam element (two nodes of four coefficient vectors,
Gauss-Legendre 3 x 2 x 2; Sec. 4.3) on the HIP path with the FP64 oracle,
through the C ABI: pattern and slot map bit-exact, f and K in both
precisions, the VJP, the batched launch, a long chain on sampled rows, and
the descriptor checks."""

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd.api import TLBatch, TLMesh
from paper_2604_10357_amd._native import TlfeaError
from tests.gpu_util import TOL, cuda, dense_rows, make_mesh, oracle_rows, rel_err

pytestmark = pytest.mark.gpu


def cases():
    out = [("beam3_svk", W.beam_3243(3, 41, "beam3_svk"))]
    # 37 elements: 444 points (a ragged stage tile) over several node ranges
    out.append(("beam37_mr_kv", W.beam_3243(37, 42, "beam37_mr_kv",
                                            material=W.Material(W.MOONEY_RIVLIN, (2e5, 5e4, 1e8), 1e3, 1e3))))
    out.append(("beam1_svk_kv", W.beam_3243(1, 43, "beam1_svk_kv",
                                            material=W.Material(W.SVK, (7e8, 0.33, 0.0), 2e3, 1e3))))
    return out


CASES = cases()


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_beam_pattern_and_slots_bit_exact(name, wl):
    print(f"[gpu] beam pattern {name}", flush=True)
    m = make_mesh(wl)
    om = oracle.Mesh.of(wl.mesh)
    ro_ref, cols_ref = oracle.csr_pattern(om)
    assert m.nnz == cols_ref.shape[0] == 144 * (3 * wl.mesh.n_elem + 1)
    ro, cols = m.csr_pattern(on_device=False)
    assert np.array_equal(ro.numpy(), ro_ref)
    assert np.array_equal(cols.numpy(), cols_ref)
    slots = m.slot_map(on_device=False).numpy()
    assert slots.shape[1:] == (24, 24)
    assert np.array_equal(slots, oracle.slot_map(om, (ro_ref, cols_ref)))
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_beam_force_and_tangent(name, wl, precision):
    print(f"[gpu] beam f/K {name} {precision}", flush=True)
    m = make_mesh(wl, precision)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    pat = oracle.csr_pattern(om)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    tol = TOL[precision]
    for alpha, beta in [(1e-3, 1.0), (1.0, 0.0), (0.0, 1.0)]:
        f, vals = m.assemble(q, qd, alpha, beta)
        f_ref, v_ref = oracle.assemble(om, omat, wl.q, wl.qdot, alpha, beta, pattern=pat)
        ef = rel_err(f.cpu().numpy(), f_ref)[0]
        ek = rel_err(vals.cpu().numpy(), v_ref)[0]
        print(f"  a={alpha} b={beta}  f {ef:.2e}  K {ek:.2e}", flush=True)
        assert ef <= tol and ek <= tol, (alpha, beta, ef, ek)
    f1 = m.internal_force(q, None)
    f1_ref, _ = oracle.assemble(om, omat, wl.q, None, want_K=False)
    assert rel_err(f1.cpu().numpy(), f1_ref)[0] <= tol
    m.close()


@pytest.mark.parametrize("name,wl", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_beam_vjp(name, wl):
    print(f"[gpu] beam vjp {name}", flush=True)
    m = make_mesh(wl)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    gq_ref, gqd_ref, gp_ref = oracle.vjp(om, omat, wl.q, wl.qdot, wl.w)
    gq, gqd, gp = m.vjp(cuda(wl.q), cuda(wl.qdot), cuda(wl.w))
    assert rel_err(gq.cpu().numpy(), gq_ref)[0] <= 1e-12
    if np.abs(gqd_ref).max() > 0:
        assert rel_err(gqd.cpu().numpy(), gqd_ref)[0] <= 1e-12
    gp = gp.cpu().numpy()
    for i in range(5):
        if gp_ref[i] != 0.0:
            assert abs(gp[i] - gp_ref[i]) <= 1e-11 * abs(gp_ref[i]), (i, gp[i], gp_ref[i])
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_beam_batch(precision):
    print(f"[gpu] beam batch {precision}", flush=True)
    wls = [W.beam_3243(n, 50 + n, f"b{n}") for n in (1, 4, 9, 2, 17)]
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
    tol = TOL[precision]
    for k, wl in enumerate(wls):
        d0, d1 = b.dof_off[k], b.dof_off[k + 1]
        z0, z1 = b.nnz_off[k], b.nnz_off[k + 1]
        om = oracle.Mesh.of(wl.mesh)
        f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, hs[k], 1.0)
        assert rel_err(f[d0:d1].cpu().numpy(), f_ref)[0] <= tol, k
        assert rel_err(vals[z0:z1].cpu().numpy(), v_ref)[0] <= tol, k
    b.close()
    for m in meshes:
        m.close()


def translated(wl, node):
    """The same body and state moved rigidly so that `node` sits at the origin
    (only position coefficients move; f and K are invariant).  Far along a
    long chain the oracle's reference Jacobian, formed from absolute
    coordinates, loses about eps |X| / L of its relative accuracy; on the
    translated copy it keeps full precision."""
    s = wl.mesh.X[4 * node].copy()
    X = wl.mesh.X.copy()
    X[0::4] -= s
    q = wl.q.reshape(-1, 3).copy()
    q[0::4] -= s
    mesh = W.Mesh(W.ANCF3243, X, wl.mesh.conn, wl.mesh.gl, wl.mesh.thickness, wl.mesh.width)
    return W.Workload(wl.name, mesh, wl.material, q.ravel(), wl.qdot, wl.w)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_beam_long_chain_sampled(precision):
    """A 200,000-element chain (the paper's largest-but-one beam resolution,
    40 km long) in the default launch shape: rows of sampled nodes (ends and
    interior, up to 40 km from the origin) against the oracle's element sums
    on a translated copy, and the global force balance (the forces on the
    position coefficients sum to zero)."""
    print(f"[gpu] beam chain 200000 {precision}", flush=True)
    wl = W.beam_3243(200_000, 44, "beam_chain")
    m = make_mesh(wl, precision)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f, vals = m.assemble(q, qd, 1e-3, 1.0)
    ro, cols = m.csr_pattern(on_device=False)
    ro, cols, f, vals = ro.numpy(), cols.numpy(), f.cpu().numpy(), vals.cpu().numpy()
    omat = oracle.material_of(wl.material)
    want, rows_ref, f_ref = [], {}, {}
    for node in [0, 1, 77_777, 123_456, 199_999, 200_000]:
        wn = translated(wl, node)
        fn, rn, wrows = oracle_rows(oracle.Mesh.of(wn.mesh), omat, wn, 1e-3, 1.0, [node])
        want += wrows
        rows_ref.update(rn)
        f_ref.update({r: fn[r] for r in wrows})
    got = dense_rows(ro, cols, vals, want)
    scale_k = max(abs(v) for r in want for v in rows_ref[r].values())
    scale_f = max(abs(f_ref[r]) for r in want)
    tol = TOL[precision]
    for r in want:
        assert set(got[r]) == set(rows_ref[r]), r
        assert max(abs(got[r][c] - rows_ref[r][c]) for c in got[r]) <= tol * scale_k, r
        assert abs(f[r] - f_ref[r]) <= tol * scale_f, r
    # translation invariance: the force components of the position coefficients sum to zero
    fr = f.reshape(-1, 4, 3)[:, 0, :].sum(axis=0)
    assert np.abs(fr).max() <= (1e-9 if precision == "fp64" else 1e-4) * np.abs(f).max() * np.sqrt(wl.mesh.n_elem)
    m.close()


def test_beam_descriptor_checks():
    print("[gpu] beam descriptor", flush=True)
    wl = W.beam_3243(2, 45, "desc")
    bad_w = W.Mesh(W.ANCF3243, wl.mesh.X, wl.mesh.conn, (3, 2, 2), 0.1, 0.0)
    with pytest.raises(TlfeaError) as e:
        TLMesh(bad_w, wl.material)
    assert e.value.status == -1
    bad_gl = W.Mesh(W.ANCF3243, wl.mesh.X, wl.mesh.conn, (3, 3, 2), 0.1, 0.1)
    with pytest.raises(TlfeaError) as e:
        TLMesh(bad_gl, wl.material)
    assert e.value.status == -2
    # coincident nodes: zero length gives a singular reference Jacobian
    X = wl.mesh.X.copy()
    X[4] = X[0]
    with pytest.raises(TlfeaError):
        TLMesh(W.Mesh(W.ANCF3243, X, wl.mesh.conn, (3, 2, 2), 0.1, 0.1), wl.material)
    m = TLMesh(wl.mesh, wl.material)
    info = m.info()
    assert info["n_en"] == 8 and info["n_qp"] == 12
    m.close()
