"""Pins of the oracle's CSR pattern and slot map (Sec. 4.2; Sec. 4.4.2:
coefficient adjacency from connectivity lifted to 3x3 DOF blocks, rows sorted)
against brute-force dense adjacency and closed-form counts, plus the workload
generator's closed-form mesh counts."""
import numpy as np
import pytest

from paper_2604_10357_amd import workloads as W


def brute_pattern(mesh):
    """Dense boolean DOF adjacency built straight from the definition."""
    n = mesh.n_dof
    adj = np.zeros((n, n), dtype=bool)
    for c in mesh.conn:
        if mesh.elem_type == W.T10:
            coefs = list(c)
        else:
            coefs = [4 * node + k for node in c for k in range(4)]
        dofs = [3 * cc + d for cc in coefs for d in range(3)]
        adj[np.ix_(dofs, dofs)] = True
    row_off = np.concatenate([[0], np.cumsum(adj.sum(axis=1))]).astype(np.int32)
    cols = np.concatenate([np.nonzero(adj[r])[0] for r in range(n)]).astype(np.int32)
    return row_off, cols


@pytest.mark.parametrize("mesh", [W.kuhn_t10_box(4, 1, 1, 1.0, 0.1, 0.1), W.kuhn_t10_box(2, 2, 2, 1, 1, 1),
                                  W.kuhn_t10_box(3, 1, 2, 1, 1, 1), W.ancf3443_plate(3, 2, 1.0, 1.0, 0.1)],
                         ids=["t10_4x1x1", "t10_2x2x2", "t10_3x1x2", "ancf_3x2"])
def test_csr_matches_brute_force(orc, mesh):
    m = orc.Mesh.of(mesh)
    ro, cols = orc.csr_pattern(m)
    bro, bcols = brute_pattern(mesh)
    assert np.array_equal(ro, bro)
    assert np.array_equal(cols, bcols)


def test_config1_nnz(orc):
    m = orc.Mesh.of(W.config1().mesh)
    ro, cols = orc.csr_pattern(m)
    assert cols.shape[0] == 12447


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_ancf_nnz_closed_form(orc, n):
    # each node is adjacent to (self + neighbours) of a tensor grid: sum = (3n+1)^2;
    # every adjacent node pair is a 12x12 DOF block
    m = orc.Mesh.of(W.ancf3443_plate(n, n, 1.0, 1.0, 0.01))
    _, cols = orc.csr_pattern(m)
    assert cols.shape[0] == (3 * n + 1) ** 2 * 144


def test_slot_map_consistent(orc):
    wl = W.config1()
    m = orc.Mesh.of(wl.mesh)
    mt = orc.material_of(wl.material)
    pat = orc.csr_pattern(m)
    ro, cols = pat
    slots = orc.slot_map(m, pat)
    # each slot sits in the right row and column
    for e in range(m.n_elem):
        dofs = np.array([3 * c + d for c in wl.mesh.conn[e] for d in range(3)])
        s = slots[e]
        rows = np.searchsorted(ro, s, side="right") - 1
        assert np.array_equal(rows, np.repeat(dofs[:, None], 30, axis=1))
        assert np.array_equal(cols[s], np.repeat(dofs[None, :], 30, axis=0))
    # scattering element matrices through the slot map reproduces the assembly
    _, vals = orc.assemble(m, mt, wl.q, wl.qdot, 1e-3, 1.0, pattern=pat, want_f=False)
    acc = np.zeros_like(vals)
    for e in range(m.n_elem):
        _, Ke = orc.element(m, mt, e, wl.q, wl.qdot, 1e-3, 1.0)
        np.add.at(acc, slots[e].ravel(), Ke.ravel())
    assert np.abs(acc - vals).max() <= 1e-13 * np.abs(vals).max()


def test_generator_counts():
    for (nx, ny, nz) in [(4, 1, 1), (2, 3, 1), (5, 2, 2)]:
        mesh = W.kuhn_t10_box(nx, ny, nz, 1.0, 1.0, 1.0)
        assert mesh.n_elem == 6 * nx * ny * nz
        assert mesh.n_coef == W.t10_node_count(nx, ny, nz)
        assert len(np.unique(mesh.conn)) == mesh.n_coef
        X, c = mesh.X, mesh.conn
        vol = np.einsum("ij,ij->i", np.cross(X[c[:, 1]] - X[c[:, 0]], X[c[:, 2]] - X[c[:, 0]]), X[c[:, 3]] - X[c[:, 0]])
        assert vol.min() > 0
        assert abs(vol.sum() / 6 - 1.0) < 1e-12
    p = W.ancf3443_plate(7, 5, 1.0, 1.0, 0.01)
    assert p.n_elem == 35 and p.n_coef == 4 * 8 * 6


def test_generator_is_seeded():
    a = W.config1()
    b = W.config1()
    assert np.array_equal(a.q, b.q) and np.array_equal(a.qdot, b.qdot) and np.array_equal(a.w, b.w)
    c = W.config1(seed=7)
    assert not np.array_equal(a.q, c.q)


def test_openmp_timing_form_matches_the_oracle():
    """The threaded form the benchmark times on all host cores computes the
    same sums (only the order of the scatter differs)."""
    import oracle

    wl = W.t10_beam(3, 2, 2, 61, "omp_check", lx=0.3, ly=0.2, lz=0.2)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    pat = oracle.csr_pattern(om)
    f1, v1 = oracle.assemble(om, omat, wl.q, wl.qdot, 1e-3, 1.0, pattern=pat)
    f2, v2, threads = oracle.assemble_omp(om, omat, wl.q, wl.qdot, 1e-3, 1.0, pat)
    assert threads >= 1
    assert np.abs(f2 - f1).max() <= 1e-13 * np.abs(f1).max()
    assert np.abs(v2 - v1).max() <= 1e-13 * np.abs(v1).max()
