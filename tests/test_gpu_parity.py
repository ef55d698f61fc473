"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: CSR pattern and slot map bit-exact; f, K values and VJPs within
max|d| / max|ref| <= 1e-12 (FP64 path) or 1e-5 (mixed path).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from tests.gpu_util import TOL, cuda, dense_rows, make_mesh, oracle_rows, rel_err

pytestmark = pytest.mark.gpu


def small_cases():
    """(name, workload) pairs spanning elements, materials, damping and tails."""
    out = [("cfg1_svk", W.config1())]
    out.append(("t10_3x2x2_mr_kv", W.t10_beam(3, 2, 2, 11, "t10_3x2x2_mr_kv", lx=0.3, ly=0.2, lz=0.2)))
    svk = W.Material(W.SVK, (1e7, 0.3, 0.0), 2e3, 1e3)
    out.append(("t10_2x2x1_svk_kv", W.t10_beam(2, 2, 1, 12, "t10_2x2x1_svk_kv", lx=0.2, ly=0.2, lz=0.1,
                                                material=svk)))
    # a ragged tail: 23 elements (not a multiple of any tile size)
    wl = W.t10_beam(2, 2, 2, 13, "t10_ragged23", lx=0.2, ly=0.2, lz=0.2)
    wl.mesh = W.Mesh(W.T10, wl.mesh.X, wl.mesh.conn[:23].copy())
    out.append(("t10_ragged23", wl))
    out.append(("ancf_4x3_332", W.shell_plate(4, 14, "ancf_4x3", thickness=0.02)))
    sh = W.shell_plate(3, 15, "ancf_3x3_443", thickness=0.02, gl=(4, 4, 3))
    sh.material = W.Material(W.SVK, (2e9, 0.3, 0.0), 5e3, 5e3)
    sh.qdot = np.random.default_rng(16).normal(0, 0.05, sh.q.shape)
    out.append(("ancf_3x3_443_kv", sh))
    # the 3x3x2 shell with damping: the full tangent layout on the matrix cores
    sd = W.shell_plate(4, 17, "ancf_4x3_332_kv", thickness=0.02)
    sd.material = W.Material(W.SVK, (2e9, 0.3, 0.0), 5e3, 5e3)
    sd.qdot = np.random.default_rng(18).normal(0, 0.05, sd.q.shape)
    out.append(("ancf_4x3_332_kv", sd))
    return out


CASES = small_cases()


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_pattern_and_slots_bit_exact(name, wl):
    print(f"[gpu] pattern {name}", flush=True)
    m = make_mesh(wl)
    om = oracle.Mesh.of(wl.mesh)
    ro_ref, cols_ref = oracle.csr_pattern(om)
    assert m.nnz == cols_ref.shape[0]
    ro, cols = m.csr_pattern(on_device=False)
    assert np.array_equal(ro.numpy(), ro_ref)
    assert np.array_equal(cols.numpy(), cols_ref)
    slots = m.slot_map(on_device=False).numpy()
    assert np.array_equal(slots, oracle.slot_map(om, (ro_ref, cols_ref)))
    sl_dev = m.slot_map(2, 3, on_device=True).cpu().numpy()
    assert np.array_equal(sl_dev, slots[2:5])
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_force_and_tangent(name, wl, precision):
    print(f"[gpu] f/K {name} {precision}", flush=True)
    m = make_mesh(wl, precision)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    pat = oracle.csr_pattern(om)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    tol = TOL[precision]
    for alpha, beta in [(1e-3, 1.0), (1.0, 0.0), (0.0, 1.0)]:
        f, vals = m.assemble(q, qd, alpha, beta)
        f_ref, v_ref = oracle.assemble(om, omat, wl.q, wl.qdot, alpha, beta, pattern=pat)
        ef, _ = rel_err(f.cpu().numpy(), f_ref)
        ek, _ = rel_err(vals.cpu().numpy(), v_ref)
        assert ef <= tol, (alpha, beta, ef)
        assert ek <= tol, (alpha, beta, ek)
        # separate entry points give the same results
        v2 = m.tangent(q, qd, alpha=alpha, beta=beta)
        assert rel_err(v2.cpu().numpy(), v_ref)[0] <= tol
    f1 = m.internal_force(q, qd)
    assert rel_err(f1.cpu().numpy(), f_ref)[0] <= tol
    # zero velocity through a null pointer
    f0 = m.internal_force(q, None)
    f0_ref, _ = oracle.assemble(om, omat, wl.q, None, want_K=False)
    assert rel_err(f0.cpu().numpy(), f0_ref)[0] <= tol
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_force_only_path(name, wl, precision):
    """The force-only path (element force blocks, fixed-order node sums):
    against the oracle, the same result on every call (no atomics), through the
    split entry points with accumulation, and no tangent from its records."""
    print(f"[gpu] force only {name} {precision}", flush=True)
    from paper_2604_10357_amd._native import TlfeaError
    m = make_mesh(wl, precision)
    om = oracle.Mesh.of(wl.mesh)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f_ref, _ = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, want_K=False)
    f1 = m.internal_force(q, qd)
    f2 = m.internal_force(q, qd)
    assert rel_err(f1.cpu().numpy(), f_ref)[0] <= TOL[precision]
    assert torch.equal(f1, f2)
    base = torch.linspace(-1, 1, m.n_dof, dtype=torch.float64, device="cuda")
    f3 = base.clone()
    m.assemble_points(q, qd, 1.0, 0.0, want_tangent=False)
    m.assemble_nodes(f3, None, accumulate=True)
    assert rel_err((f3 - base).cpu().numpy(), f1.cpu().numpy())[0] <= 1e-14
    with pytest.raises(TlfeaError) as e:
        m.assemble_nodes(None, torch.empty(m.nnz, dtype=torch.float64, device="cuda"))
    assert e.value.status == -1
    m.close()


def test_accumulate_adds_onto_existing_values():
    wl = W.config1()
    m = make_mesh(wl)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f, vals = m.assemble(q, qd, 1e-3, 1.0)
    base_f = torch.linspace(-1, 1, m.n_dof, dtype=torch.float64, device="cuda")
    base_v = torch.linspace(2, 3, m.nnz, dtype=torch.float64, device="cuda")
    f2, v2 = base_f.clone(), base_v.clone()
    m.assemble_accumulate(q, qd, 1e-3, 1.0, f2, v2)
    assert rel_err((f2 - base_f).cpu().numpy(), f.cpu().numpy())[0] <= 1e-12
    assert rel_err((v2 - base_v).cpu().numpy(), vals.cpu().numpy())[0] <= 1e-12
    m.close()


def test_config2_full_size():
    """30,720 T10 elements, Mooney-Rivlin + Kelvin-Voigt, every value checked."""
    print("[gpu] config2 full", flush=True)
    wl = W.config2()
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    pat = oracle.csr_pattern(om)
    f_ref, v_ref = oracle.assemble(om, omat, wl.q, wl.qdot, 1e-3, 1.0, pattern=pat)
    q, qd = cuda(wl.q), cuda(wl.qdot)
    m = make_mesh(wl, "fp64")
    ro, cols = m.csr_pattern(on_device=False)
    assert np.array_equal(ro.numpy(), pat[0]) and np.array_equal(cols.numpy(), pat[1])
    for precision in ("fp64", "mixed"):
        m.set_precision(precision)
        f, vals = m.assemble(q, qd, 1e-3, 1.0)
        ef, ef2 = rel_err(f.cpu().numpy(), f_ref)
        ek, ek2 = rel_err(vals.cpu().numpy(), v_ref)
        print(f"  config2 {precision}: f {ef:.2e} ({ef2:.2e})  K {ek:.2e} ({ek2:.2e})", flush=True)
        assert ef <= TOL[precision] and ek <= TOL[precision]
    m.close()


_CONFIG5 = {}


def _config5_reference():
    """The 480,000-element beam, its oracle CSR pattern and its oracle f and K
    (h = 1e-3), computed once for both precisions."""
    if not _CONFIG5:
        wl = W.config5()
        om = oracle.Mesh.of(wl.mesh)
        pat = oracle.csr_pattern(om)
        f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, 1e-3, 1.0, pattern=pat)
        _CONFIG5.update(wl=wl, pat=pat, f=f_ref, v=v_ref)
    return _CONFIG5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config5_full(precision):
    """480,000 T10 elements at full size in the benchmark's launch: the CSR
    pattern bit-exact against the oracle's (row offsets and all 169,094,889
    columns), every value of f and K against the oracle, and the momentum
    invariant over the whole force vector (also for the force-only path)."""
    print(f"[gpu] config5 full {precision}", flush=True)
    ref = _config5_reference()
    wl = ref["wl"]
    m = make_mesh(wl, precision)
    ro, cols = m.csr_pattern(on_device=False)
    assert np.array_equal(ro.numpy(), ref["pat"][0])
    assert np.array_equal(cols.numpy(), ref["pat"][1])
    del ro, cols
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f, vals = m.assemble(q, qd, 1e-3, 1.0)
    fh = f.cpu().numpy()
    ef, ef2 = rel_err(fh, ref["f"])
    ek, ek2 = rel_err(vals.cpu().numpy(), ref["v"])
    del vals
    print(f"  config5 {precision}: f {ef:.2e} ({ef2:.2e})  K {ek:.2e} ({ek2:.2e})", flush=True)
    assert ef <= TOL[precision] and ek <= TOL[precision]
    # momentum: each element's forces sum to zero up to the rounding of its own
    # arithmetic (float32 in the mixed path), a random walk over the elements
    fv = fh.reshape(-1, 3)
    eps = 1e-9 if precision == "fp64" else 1e-6
    assert np.abs(fv.sum(axis=0)).max() <= eps * np.abs(fv).max() * np.sqrt(len(fv))
    # the force-only path on the same mesh
    fo = m.internal_force(q, qd).cpu().numpy()
    ef0 = rel_err(fo, ref["f"])[0]
    print(f"  config5 {precision}: force-only f {ef0:.2e}", flush=True)
    assert ef0 <= TOL[precision]
    fov = fo.reshape(-1, 3)
    assert np.abs(fov.sum(axis=0)).max() <= eps * np.abs(fov).max() * np.sqrt(len(fov))
    m.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config3_sampled(precision):
    """The 256 x 256 ANCF3443 plate (65,536 elements, 3x3x2 rule) at full size in
    the benchmark's launch: the CSR pattern bit-exact against the oracle's
    (85,155,984 columns), and the rows of 517 sampled nodes (all 12 coefficient
    rows, every contribution) against the oracle."""
    print(f"[gpu] config3 sampled {precision}", flush=True)
    wl = W.config3()
    m = make_mesh(wl, precision)
    ro_ref, cols_ref = oracle.csr_pattern(oracle.Mesh.of(wl.mesh))
    ro_g, cols_g = m.csr_pattern(on_device=False)
    assert np.array_equal(ro_g.numpy(), ro_ref) and np.array_equal(cols_g.numpy(), cols_ref)
    del ro_g, cols_g, ro_ref, cols_ref
    h = 1e-3
    f, vals = m.assemble(cuda(wl.q), cuda(wl.qdot), h, 1.0)
    ro, cols = m.csr_pattern(on_device=False)
    fh, vh = f.cpu().numpy(), vals.cpu().numpy()
    n_nodes = int(wl.mesh.conn.max()) + 1
    rng = np.random.default_rng(33)
    # corners, an edge node, the centre and random interior nodes
    nodes = np.concatenate([[0, 256, n_nodes - 1, 128, n_nodes // 2], rng.choice(n_nodes, 512, replace=False)])
    om = oracle.Mesh.of(wl.mesh)
    f_ref, rows_ref, rows = oracle_rows(om, oracle.material_of(wl.material), wl, h, 1.0, nodes)
    got = dense_rows(ro.numpy(), cols.numpy(), vh, rows)
    fmax = np.abs(f_ref[rows]).max()
    kmax = max(max(abs(v) for v in r.values()) for r in rows_ref.values())
    ef = np.abs(fh[rows] - f_ref[rows]).max() / fmax
    ek = 0.0
    for r in rows:
        assert set(got[r].keys()) == set(rows_ref[r].keys())
        for c, v in rows_ref[r].items():
            ek = max(ek, abs(got[r][c] - v) / kmax)
    print(f"  config3 {precision}: sampled f {ef:.2e}  K {ek:.2e}", flush=True)
    assert ef <= TOL[precision] and ek <= TOL[precision]
    m.close()


@pytest.mark.gpu
def test_config4_full_batch():
    """All 512 cubes (about 1.7 M elements, mixed precision) in one graph-captured
    launch pair: sampled bodies against the oracle, every body against the
    per-body loop."""
    from paper_2604_10357_amd.api import TLBatch
    print("[gpu] config4 full batch", flush=True)
    wls = W.config4()
    meshes = [make_mesh(wl, "mixed") for wl in wls]
    b = TLBatch(meshes)
    q = cuda(np.concatenate([wl.q for wl in wls]))
    qd = cuda(np.concatenate([wl.qdot for wl in wls]))
    hs = np.full(len(wls), 1e-3)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        f, vals = b.assemble(q, qd, cuda(hs))
        f2, vals2 = b.assemble(q, qd, cuda(hs))  # graph replay
        fl, vl = b.assemble(q, qd, cuda(hs), loop=True)
    stream.synchronize()
    fh, vh = f.cpu().numpy(), vals.cpu().numpy()
    # The per-range LDS sums take contributions from several waves in arrival
    # order, so repeated calls agree to rounding, not bit for bit.
    assert rel_err(f2.cpu().numpy(), fh)[0] <= 1e-13 and rel_err(vals2.cpu().numpy(), vh)[0] <= 1e-13
    assert np.abs(fl.cpu().numpy() - fh).max() <= 1e-13 * np.abs(fh).max()
    assert np.abs(vl.cpu().numpy() - vh).max() <= 1e-13 * np.abs(vh).max()
    rng = np.random.default_rng(44)
    for k in sorted(set([0, len(wls) - 1] + rng.choice(len(wls), 6, replace=False).tolist())):
        wl = wls[k]
        d0, d1 = b.dof_off[k], b.dof_off[k + 1]
        z0, z1 = b.nnz_off[k], b.nnz_off[k + 1]
        om = oracle.Mesh.of(wl.mesh)
        f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, hs[k], 1.0)
        ef = rel_err(fh[d0:d1], f_ref)[0]
        ek = rel_err(vh[z0:z1], v_ref)[0]
        print(f"  body {k}: {wl.mesh.n_elem} elements, f {ef:.2e} K {ek:.2e}", flush=True)
        assert ef <= TOL["mixed"] and ek <= TOL["mixed"]
    b.close()
    for m in meshes:
        m.close()


def test_runtime_flags_and_errors():
    from paper_2604_10357_amd import _native as N
    wl = W.config1()
    m = make_mesh(wl, "fp64")
    q = cuda(wl.q)
    assert m.runtime_flags() == 0
    m.internal_force(q)
    assert m.runtime_flags() == 0
    # mirror the body (x -> -x): F = diag(-1, 1, 1), det F = -1 everywhere
    qi = wl.mesh.X.copy()
    qi[:, 0] *= -1.0
    m.internal_force(cuda(qi.ravel()))
    assert m.runtime_flags() & N.TLFEA_FLAG_INVERTED
    qn = wl.q.copy()
    qn[7] = np.nan
    m.internal_force(cuda(qn))
    assert m.runtime_flags() & N.TLFEA_FLAG_NONFINITE
    assert m.runtime_flags() == 0  # reading clears
    m.close()
    # tangent before the pattern exists
    from paper_2604_10357_amd.api import TLMesh
    m2 = TLMesh(wl.mesh, wl.material)
    m2.nnz = 1
    with pytest.raises(N.TlfeaError) as e:
        m2.tangent(q, None, out=torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert e.value.status == -6
    # the VJP's per-node sums run over the pattern's node ranges as well
    with pytest.raises(N.TlfeaError) as e:
        m2.vjp(q, None, q)
    assert e.value.status == -6
    m2.close()
    # the VJP reuses the work buffer: pass 2 alone then has nothing to reduce
    m3 = make_mesh(wl, "fp64")
    m3.assemble_points(q, None, 1.0, 1.0, True)
    m3.vjp(q, None, q)
    with pytest.raises(N.TlfeaError) as e:
        m3.assemble_nodes(torch.empty(m3.n_dof, dtype=torch.float64, device="cuda"), None)
    assert e.value.status == -1
    m3.close()
    # degenerate reference element: a flat tetrahedron (coplanar corners)
    corners = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=float)
    X = np.vstack([corners, [(corners[a] + corners[b]) / 2 for a, b in W.T10_EDGES]])
    with pytest.raises(N.TlfeaError) as e:
        TLMesh(W.Mesh(W.T10, X, np.arange(10, dtype=np.int32)[None, :]), wl.material)
    assert e.value.status == -3
