"""The symmetric-only tangent path against the full one, in one process.

An undamped material (no Kelvin-Voigt terms) takes the symmetric record layout
and the contraction of the slots i <= k (Sec. 4.4.2, Eq. tangent_block: the
hyperelastic tangent has major symmetry); a material whose viscosities are
1e-300 takes the full layout and the full contraction, while its viscous
terms vanish (they underflow to zero in float32 and stay ~1e-300 of the
elastic ones in float64).  The two calls must then agree to the rounding of
the arithmetic they run in: much tighter than the oracle gate, so that a
misplaced transposed entry cannot hide under it.  Covers T10 (SVK and
Mooney-Rivlin), both shell rules (the matrix-core contraction) and the beam,
in both precisions, for f, K and the upper-triangle output."""
import numpy as np
import pytest
import torch

from paper_2604_10357_amd import workloads as W
from tests.gpu_util import cuda, make_mesh, rel_err

pytestmark = pytest.mark.gpu

TINY = 1e-300
# float32 contractions in a different order (six slots and transposition
# against nine slots): a few units of float32 rounding of the largest entry
GATE = {"mixed": 2e-6, "fp64": 1e-13}


def with_viscosity(wl, eta):
    m = wl.material
    return W.Workload(wl.name, wl.mesh, W.Material(m.kind, m.params, eta, eta), wl.q, wl.qdot, wl.w)


def cases():
    rng = np.random.default_rng(301)
    out = [("t10_svk", W.t10_beam(3, 2, 2, 302, "t10_svk", lx=0.3, ly=0.2, lz=0.2,
                                  material=W.Material(W.SVK, (1e7, 0.3, 0.0)))),
           ("t10_mr", W.t10_beam(3, 2, 2, 303, "t10_mr", lx=0.3, ly=0.2, lz=0.2,
                                 material=W.Material(W.MOONEY_RIVLIN, (2e5, 5e4, 1e8)))),
           ("shell_332", W.shell_plate(5, 304, "shell332", thickness=0.02)),
           ("shell_443", W.shell_plate(3, 305, "shell443", thickness=0.02, gl=(4, 4, 3))),
           ("beam", W.beam_3243(23, 306, "beam"))]
    for _, wl in out:
        wl.qdot = rng.normal(0.0, 0.05, wl.q.shape)
    return out


CASES = cases()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_symmetric_path_matches_full_path(name, wl, precision):
    print(f"[gpu] symmetric vs full {name} {precision}", flush=True)
    res = {}
    for tag, eta in (("sym", 0.0), ("full", TINY)):
        w = with_viscosity(wl, eta)
        m = make_mesh(w, precision)
        q, qd = cuda(w.q), cuda(w.qdot)
        f, vals = m.assemble(q, qd, alpha=1e-3, beta=1.0)
        vu = None
        if eta == 0.0:  # the upper-triangle output exists for undamped materials only
            m.build_upper_pattern()
            _, vu = m.assemble_upper(q, qd, alpha=1e-3, beta=1.0)
            ro, cols = m.csr_pattern(on_device=False)
            res["pattern"] = (ro.numpy(), cols.numpy())
        res[tag] = (f.cpu().numpy(), vals.cpu().numpy(), None if vu is None else vu.cpu().numpy())
        m.close()
    (fs, ks, kus), (ff, kf, _) = res["sym"], res["full"]
    ef, ek = rel_err(fs, ff)[0], rel_err(ks, kf)[0]
    assert ef <= GATE[precision] and ek <= GATE[precision], (ef, ek)
    # the upper triangle of the symmetric call is the upper part of the full K
    ro, cols = res["pattern"]
    n = len(ro) - 1
    keep = np.concatenate([np.arange(ro[r], ro[r + 1])[cols[ro[r]:ro[r + 1]] >= r] for r in range(n)])
    assert rel_err(kus, kf[keep])[0] <= GATE[precision]


@pytest.mark.parametrize("name,wl", [CASES[0], CASES[2]], ids=[CASES[0][0], CASES[2][0]])
def test_split_pass_keeps_the_layout_of_its_pass_1(name, wl):
    """Pass 2 alone reduces what pass 1 left, in the layout pass 1 wrote it: a
    material change between the two (here to a damped one, whose pass 1 would
    write the full float64 records) does not change how pass 2 reads them."""
    print(f"[gpu] split pass layout {name}", flush=True)
    m = make_mesh(wl, "fp64")
    q, qd = cuda(wl.q), cuda(wl.qdot)
    f, vals = m.assemble(q, qd, alpha=1e-3, beta=1.0)
    m.assemble_points(q, qd, 1e-3, 1.0, want_tangent=True)
    mat = wl.material
    m.set_material(W.Material(mat.kind, mat.params, 1e3, 1e3))
    f2, v2 = torch.empty_like(f), torch.empty_like(vals)
    m.assemble_nodes(f2, v2)
    assert rel_err(f2.cpu().numpy(), f.cpu().numpy())[0] <= 1e-14
    assert rel_err(v2.cpu().numpy(), vals.cpu().numpy())[0] <= 1e-14
    m.close()
