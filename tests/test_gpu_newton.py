"""Parity of the Newton-step pieces (consistent mass, Newton matrix
H = M/h + h K_t, gradient g = M (v - v_prev)/h + f_int - f_ext) with the FP64
CPU oracle, through the C ABI, for T10, the ANCF3443 shell (both rules) and
the ANCF3243 beam."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd._native import TlfeaError
from tests.gpu_util import TOL, cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu

CASES = [
    ("t10_3x2x2_mr_kv", W.t10_beam(3, 2, 2, 81, "t10_3x2x2_mr_kv", lx=0.3, ly=0.2, lz=0.2)),
    ("t10_ragged23", None),
    ("cfg2", W.config2()),
]
_w = W.t10_beam(2, 2, 2, 82, "t10_ragged23", lx=0.2, ly=0.2, lz=0.2)
_w.mesh = W.Mesh(W.T10, _w.mesh.X, _w.mesh.conn[:23].copy())
CASES[1] = ("t10_ragged23", _w)
_sh = W.shell_plate(3, 85, "ancf_3x3_443_kv", thickness=0.02, gl=(4, 4, 3))
_sh.material = W.Material(W.SVK, (2e9, 0.3, 0.0), 5e3, 5e3)
CASES += [("ancf_4x3_332", W.shell_plate(4, 86, "ancf_4x3", thickness=0.02)),
          ("ancf_3x3_443_kv", _sh),
          ("beam37_mr_kv", W.beam_3243(37, 87, "beam37_mr_kv",
                                       material=W.Material(W.MOONEY_RIVLIN, (2e5, 5e4, 1e8), 1e3, 1e3)))]
RHO = 1100.0


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_mass_matches_oracle(name, wl):
    print(f"[gpu] mass {name}", flush=True)
    m = make_mesh(wl, "fp64")
    m.build_mass(RHO)
    got = m.mass_values().cpu().numpy()
    om = oracle.Mesh.of(wl.mesh)
    ref = oracle.mass_csr(om, RHO)
    assert rel_err(got, ref)[0] <= 1e-13
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_newton_matrix_and_gradient(name, wl, precision):
    print(f"[gpu] newton {name} {precision}", flush=True)
    m = make_mesh(wl, precision)
    m.build_mass(RHO)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    pat = oracle.csr_pattern(om)
    h = 2e-3
    rng = np.random.default_rng(83)
    n = wl.mesh.n_dof
    v_prev = rng.normal(0, 0.05, n)
    v = v_prev + rng.normal(0, 0.02, n)
    q = wl.q + h * v  # q = q_n + h v with q_n the workload's state
    f, H = m.assemble_newton(cuda(q), cuda(v), h)
    f_ref, K_ref = oracle.assemble(om, omat, q, v, h, 1.0, pattern=pat)
    M_ref = oracle.mass_csr(om, RHO, pat)
    H_ref = M_ref / h + K_ref
    ef, eH = rel_err(f.cpu().numpy(), f_ref)[0], rel_err(H.cpu().numpy(), H_ref)[0]
    print(f"  f {ef:.2e}  H {eH:.2e}", flush=True)
    assert ef <= TOL[precision] and eH <= TOL[precision]
    f_ext = rng.normal(0, 1.0, n)
    g = m.newton_gradient(cuda(v), cuda(v_prev), f, cuda(f_ext), h).cpu().numpy()
    g_ref = oracle.gradient(pat, M_ref, v, v_prev, f.cpu().numpy(), f_ext, h)
    assert rel_err(g, g_ref)[0] <= 1e-12
    g0 = m.newton_gradient(cuda(v), cuda(v_prev), f, None, h).cpu().numpy()
    assert rel_err(g0, g_ref + f_ext)[0] <= 1e-12
    # without the mass term the same call path gives the tangent alone
    _, K = m.assemble(cuda(q), cuda(v), h, 1.0)
    assert rel_err(K.cpu().numpy(), K_ref)[0] <= TOL[precision]
    m.close()


def test_newton_error_paths():
    print("[gpu] newton errors", flush=True)
    wl = CASES[0][1]
    m = make_mesh(wl, "mixed")
    q = cuda(wl.q)
    with pytest.raises(TlfeaError) as e:
        m.assemble_newton(q, q, 1e-3)
    assert e.value.status == -1
    with pytest.raises(TlfeaError) as e:
        m.newton_gradient(q, q, q, None, 1e-3)
    assert e.value.status == -1
    with pytest.raises(TlfeaError) as e:
        m.build_mass(-1.0)
    assert e.value.status == -1
    m.build_mass(RHO)
    with pytest.raises(TlfeaError) as e:
        m.assemble_newton(q, q, 0.0)
    assert e.value.status == -1
    m.close()
    # a curved beam element (a reference slope off the chord) is not supported
    bw = W.beam_3243(2, 84, "curved_beam")
    Xb = bw.mesh.X.copy()
    Xb[5] = [0.995, 0.0, 0.0998]
    cb = make_mesh(W.Workload("curved_beam", W.Mesh(W.ANCF3243, Xb, bw.mesh.conn, (3, 2, 2), 0.1, 0.1),
                              bw.material, bw.q, bw.qdot, bw.w), "mixed")
    with pytest.raises(TlfeaError) as e:
        cb.build_mass(RHO)
    assert e.value.status == -2
    cb.close()
    # a curved T10 element (an edge node off its edge) is not supported
    X = wl.mesh.X.copy()
    X[int(wl.mesh.conn[0, 4])] += 0.002
    cw = W.Workload("curved", W.Mesh(W.T10, X, wl.mesh.conn), wl.material, wl.q, wl.qdot, wl.w)
    cm = make_mesh(cw, "fp64")
    with pytest.raises(TlfeaError) as e:
        cm.build_mass(RHO)
    assert e.value.status == -2
    cm.close()
