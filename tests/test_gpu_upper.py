"""Upper-triangle export and symmetric assembly for undamped materials:
pattern bit-exact against the oracle's full pattern cut at the diagonal,
values against the oracle and against the full GPU assembly, and the error
paths (damped material, pattern not built)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd._native import TlfeaError
from tests.gpu_util import TOL, cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu


def undamped(wl):
    m = wl.material
    wl.material = W.Material(m.kind, m.params, 0.0, 0.0)
    return wl


CASES = [
    ("t10_3x2x2_svk", undamped(W.t10_beam(3, 2, 2, 91, "t10_svk", lx=0.3, ly=0.2, lz=0.2,
                                          material=W.Material(W.SVK, (1e7, 0.3, 0.0), 0.0, 0.0)))),
    ("t10_3x2x2_mr", undamped(W.t10_beam(3, 2, 2, 92, "t10_mr", lx=0.3, ly=0.2, lz=0.2))),
    ("ancf_4x3_332", undamped(W.shell_plate(4, 93, "ancf", thickness=0.02))),
    ("ancf_3x3_443", undamped(W.shell_plate(3, 95, "ancf443", thickness=0.02, gl=(4, 4, 3)))),
    ("beam_9", undamped(W.beam_3243(9, 96, "beam"))),
]


def upper_of(ro, cols, vals=None):
    """Rows cut at the diagonal: (row offsets, columns[, values]) of the upper triangle."""
    n = len(ro) - 1
    keep = np.concatenate([np.arange(ro[r], ro[r + 1])[cols[ro[r]:ro[r + 1]] >= r] for r in range(n)])
    lens = np.array([np.count_nonzero(cols[ro[r]:ro[r + 1]] >= r) for r in range(n)])
    ro_u = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    out = (ro_u, cols[keep])
    return out if vals is None else out + (vals[keep],)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_upper_pattern_and_values(name, wl, precision):
    print(f"[gpu] upper {name} {precision}", flush=True)
    m = make_mesh(wl, precision)
    nnz_u = m.build_upper_pattern()
    om = oracle.Mesh.of(wl.mesh)
    ro, cols = oracle.csr_pattern(om)
    ro_u_ref, cols_u_ref = upper_of(ro, cols)
    assert nnz_u == len(cols_u_ref)
    ro_u, cols_u = m.csr_pattern_upper()
    assert np.array_equal(ro_u.numpy(), ro_u_ref)
    assert np.array_equal(cols_u.numpy(), cols_u_ref)
    h = 1e-3
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f_u, v_u = m.assemble_upper(q, qd, h, 1.0)
    f_ref, v_ref = oracle.assemble(om, oracle.material_of(wl.material), wl.q, wl.qdot, h, 1.0, pattern=(ro, cols))
    _, _, vu_ref = upper_of(ro, cols, v_ref)
    assert rel_err(f_u.cpu().numpy(), f_ref)[0] <= TOL[precision]
    assert rel_err(v_u.cpu().numpy(), vu_ref)[0] <= TOL[precision]
    # the same entries as the full assembly
    f_full, v_full = m.assemble(q, qd, h, 1.0)
    _, _, vu_full = upper_of(ro, cols, v_full.cpu().numpy())
    assert rel_err(v_u.cpu().numpy(), vu_full)[0] <= 1e-13
    # and the full matrix is symmetric: its lower triangle mirrors the upper one
    n = wl.mesh.n_dof
    K = np.zeros((n, n))
    vf = v_full.cpu().numpy()
    for r in range(n):
        K[r, cols[ro[r]:ro[r + 1]]] = vf[ro[r]:ro[r + 1]]
    assert np.abs(K - K.T).max() <= TOL[precision] * np.abs(K).max()
    m.close()


def test_upper_error_paths():
    print("[gpu] upper errors", flush=True)
    wl = CASES[0][1]
    m = make_mesh(wl, "fp64")
    q = cuda(wl.q)
    m.nnz_upper = m.nnz
    with pytest.raises(TlfeaError) as e:  # pattern not built
        m.assemble_upper(q, q, 1.0, 0.0)
    assert e.value.status == -1
    m.close()
    damped = W.t10_beam(2, 2, 1, 94, "damped", lx=0.2, ly=0.2, lz=0.1)
    assert damped.material.kv_eta > 0
    d = make_mesh(damped, "mixed")
    d.build_upper_pattern()
    with pytest.raises(TlfeaError) as e:
        d.assemble_upper(cuda(damped.q), cuda(damped.qdot), 1e-3, 1.0)
    assert e.value.status == -2
    d.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_newton_matrix_upper(name, wl, precision):
    """H = M/h + h df/dq in upper-triangle storage: against the oracle's mass and
    tangent cut at the diagonal, and against the full GPU Newton matrix."""
    print(f"[gpu] newton upper {name} {precision}", flush=True)
    rho, h = 1100.0, 2e-3
    m = make_mesh(wl, precision)
    m.build_mass(rho)
    m.build_upper_pattern()
    om = oracle.Mesh.of(wl.mesh)
    ro, cols = oracle.csr_pattern(om)
    rng = np.random.default_rng(97)
    v = rng.normal(0, 0.02, wl.mesh.n_dof)
    q = wl.q + h * v
    f_u, H_u = m.assemble_newton_upper(cuda(q), cuda(v), h)
    f_ref, K_ref = oracle.assemble(om, oracle.material_of(wl.material), q, v, h, 1.0, pattern=(ro, cols))
    H_ref = oracle.mass_csr(om, rho, (ro, cols)) / h + K_ref
    _, _, Hu_ref = upper_of(ro, cols, H_ref)
    assert rel_err(f_u.cpu().numpy(), f_ref)[0] <= TOL[precision]
    assert rel_err(H_u.cpu().numpy(), Hu_ref)[0] <= TOL[precision]
    _, H_full = m.assemble_newton(cuda(q), cuda(v), h)
    _, _, Hu_full = upper_of(ro, cols, H_full.cpu().numpy())
    assert rel_err(H_u.cpu().numpy(), Hu_full)[0] <= 1e-13
    m.close()


def test_newton_matrix_upper_errors():
    print("[gpu] newton upper errors", flush=True)
    wl = CASES[0][1]
    m = make_mesh(wl, "mixed")
    q = cuda(wl.q)
    m.nnz_upper = m.nnz
    with pytest.raises(TlfeaError) as e:  # no mass
        m.assemble_newton_upper(q, q, 1e-3)
    assert e.value.status == -1
    m.build_mass(1000.0)
    with pytest.raises(TlfeaError) as e:  # no upper pattern
        m.assemble_newton_upper(q, q, 1e-3)
    assert e.value.status == -1
    m.close()
    damped = W.t10_beam(2, 2, 1, 98, "damped", lx=0.2, ly=0.2, lz=0.1)
    d = make_mesh(damped, "mixed")
    d.build_mass(1000.0)
    d.build_upper_pattern()
    with pytest.raises(TlfeaError) as e:
        d.assemble_newton_upper(cuda(damped.q), cuda(damped.qdot), 1e-3)
    assert e.value.status == -2
    d.close()
