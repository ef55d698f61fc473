"""The paper's printed mesh statistics fix the DOF conventions: three DOFs per
T10 node, 4 coefficient vectors x 3 = 12 DOFs per ANCF3443 node on a
structured n x n plate with (n+1)^2 nodes, and 12 DOFs per node of an
n-element ANCF3243 chain with n + 1 nodes (Sec. 5.1, 5.2 and 5.3 tables)."""
import math
import os

import numpy as np

from paper_2604_10357_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_mesh_statistics.txt")


def rows():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        el, res, dofs, nodes, elems = line.split()
        out.append((el, res, int(dofs), int(nodes), int(elems)))
    return out


def test_t10_three_dofs_per_node():
    t10 = [r for r in rows() if r[0] == "T10"]
    assert len(t10) == 6
    for _, _, dofs, nodes, _ in t10:
        assert dofs == 3 * nodes


def test_ancf3443_plate_counts_match_paper():
    ancf = [r for r in rows() if r[0] == "ANCF3443"]
    assert len(ancf) == 6
    for _, _, dofs, nodes, elems in ancf:
        n = math.isqrt(elems)
        assert n * n == elems
        mesh = W.ancf3443_plate(n, n, 4.0, 2.0, 0.1)
        assert mesh.n_elem == elems
        assert mesh.n_coef == 4 * nodes
        assert mesh.n_dof == dofs
        assert len(np.unique(mesh.conn)) == nodes


def test_ancf3243_chain_counts_match_paper():
    import oracle
    beam = [r for r in rows() if r[0] == "ANCF3243"]
    assert len(beam) == 6
    for _, res, dofs, nodes, elems in beam:
        mesh = W.ancf3243_chain(elems)
        assert mesh.n_elem == elems
        assert mesh.n_coef == 4 * nodes
        assert mesh.n_dof == dofs
        assert len(np.unique(mesh.conn)) == nodes
    # the oracle's pattern at RES0: an interior node couples to itself and its two
    # neighbours (3 x 144 values per node), an end node to two
    mesh = W.ancf3243_chain(beam[0][4])
    ro, cols = oracle.csr_pattern(oracle.Mesh.of(mesh))
    assert len(cols) == 144 * (3 * beam[0][4] + 1)

