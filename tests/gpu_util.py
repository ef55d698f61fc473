"""Helpers shared by the GPU parity tests (no test functions here)."""
import numpy as np
import torch

import oracle
from paper_2604_10357_amd import workloads as W
from paper_2604_10357_amd.api import TLMesh


def rel_err(got, ref):
    """max|got - ref| / max|ref| over the whole result (the gate), plus the 2-norm ratio."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    d = got - ref
    if den == 0.0:  # an exactly zero reference must be reproduced exactly
        return float(np.abs(got).max()), float(np.abs(got).max())
    return float(np.abs(d).max() / den), float(np.linalg.norm(d) / np.linalg.norm(ref))


TOL = {"fp64": 1e-12, "mixed": 1e-5}


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def dense_rows(ro, cols, vals, rows):
    out = {}
    for r in rows:
        a, b = ro[r], ro[r + 1]
        out[r] = dict(zip(cols[a:b].tolist(), vals[a:b].tolist()))
    return out


def oracle_rows(om, omat, wl, alpha, beta, nodes):
    """Exact f and K rows of the given pattern nodes from the oracle, using only
    the elements incident to them (every contribution to those rows)."""
    conn = wl.mesh.conn
    npn = conn.shape[1]
    mc = 1 if wl.mesh.elem_type == W.T10 else 4
    inc = np.nonzero(np.isin(conn, nodes).any(axis=1))[0].astype(np.int32)
    f = np.zeros(wl.mesh.n_dof)
    rows = {}
    for e in inc:
        fe, Ke = oracle.element(om, omat, int(e), wl.q, wl.qdot, alpha, beta)
        coefs = [int(c) for c in conn[e]] if mc == 1 else [4 * int(n) + k for n in conn[e] for k in range(4)]
        dofs = [3 * c + d for c in coefs for d in range(3)]
        for a, r in enumerate(dofs):
            f[r] += fe[a]
            row = rows.setdefault(r, {})
            for b, c in enumerate(dofs):
                row[c] = row.get(c, 0.0) + Ke[a, b]
    want_rows = [3 * (mc * n + k) + d for n in nodes for k in range(mc) for d in range(3)]
    return f, {r: rows[r] for r in want_rows}, want_rows


def make_mesh(wl, precision="fp64"):
    m = TLMesh(wl.mesh, wl.material, precision)
    m.build_pattern()
    return m
