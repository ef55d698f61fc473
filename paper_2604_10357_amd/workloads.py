"""Seeded synthetic workloads: meshes, states and cotangents.

This module only produces *data* (mesh topology, reference coordinates,
perturbed states, material parameter draws).  It contains none of the
finite-element arithmetic; both the CPU oracle (``oracle/``) and the HIP
library consume what it returns.

Workload shapes follow the paper's benchmarks (T10 beam sagging and the
ANCF3443 plate, Sec. 5.1 and Sec. 5.3; material tables in App. A): a box beam
meshed with quadratic tetrahedra, a flat shell plate of ANCF3443 elements,
and many independent T10 bodies of uneven size.  The paper's own meshes are
unstructured and not available, so structured meshes of the same element
families stand in for them.

Conventions
-----------
* T10 local node order: corners 0-3, then the mid-edge nodes of edges
  (0,1), (1,2), (0,2), (0,3), (1,3), (2,3).
* T10 boxes use the Kuhn (Freudenthal) split of every hexahedral cell into six
  tetrahedra sharing the cell diagonal, which is conforming across cells.
  Nodes live on the doubled grid, so a box of nx*ny*nz cells has
  (2nx+1)(2ny+1)(2nz+1) nodes; node ids run with x slowest.
* ANCF3443: each physical node carries four coefficient vectors
  (r, r_x, r_y, r_z); coefficient c = 4*node + k, DOF = 3*c + d.  The element
  connectivity lists its four physical nodes counter-clockwise starting at
  parent corner (-1,-1).
* Generalised coordinates are flat float64 arrays with DOF = 3*coef + d.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional

import numpy as np

T10 = 1
ANCF3443 = 2
ANCF3243 = 3
SVK = 1
MOONEY_RIVLIN = 2

# ordering of the six mid-edge nodes of a T10 element
T10_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


@dataclasses.dataclass
class Material:
    kind: int                 # SVK or MOONEY_RIVLIN
    params: tuple             # SVK: (E, nu, 0); MR: (mu10, mu01, kappa)
    kv_eta: float = 0.0       # Kelvin-Voigt shear-like viscosity
    kv_lambda: float = 0.0    # Kelvin-Voigt volumetric viscosity


@dataclasses.dataclass
class Mesh:
    elem_type: int
    X: np.ndarray             # (n_coef, 3) float64 reference coefficients
    conn: np.ndarray          # (n_elem, 10) T10 node ids | (n_elem, 4) ANCF physical nodes
    gl: tuple = (0, 0, 0)     # ANCF Gauss-Legendre points per parent direction
    thickness: float = 0.0    # ANCF3443 shell thickness; ANCF3243 cross-section height (z)
    width: float = 0.0        # ANCF3243 cross-section width (y)

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_coef(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_dof(self) -> int:
        return 3 * self.n_coef


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    material: Material
    q: np.ndarray             # (n_dof,) current generalised coordinates
    qdot: np.ndarray          # (n_dof,) generalised velocities
    w: Optional[np.ndarray] = None   # (n_dof,) cotangent for the VJP


# ----------------------------------------------------------------------------
# mesh topology
# ----------------------------------------------------------------------------

def kuhn_t10_box(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float) -> Mesh:
    """Quadratic-tetrahedron mesh of a box, six Kuhn tetrahedra per cell."""
    gx, gy, gz = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    ii, jj, kk = np.meshgrid(np.arange(gx), np.arange(gy), np.arange(gz), indexing="ij")
    X = np.stack([ii.ravel() * (lx / (2 * nx)),
                  jj.ravel() * (ly / (2 * ny)),
                  kk.ravel() * (lz / (2 * nz))], axis=1).astype(np.float64)

    # the six tetrahedra of the unit cell, corners in doubled-grid offsets
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        v0 = np.zeros(3, dtype=np.int64)
        v1 = v0 + unit[perm[0]]
        v2 = v1 + unit[perm[1]]
        v3 = np.ones(3, dtype=np.int64)
        corners = [v0, v1, v2, v3]
        vol = np.linalg.det(np.stack([v1 - v0, v2 - v0, v3 - v0]).astype(float))
        if vol < 0:                      # keep a positive orientation
            corners = [v0, v2, v1, v3]
        nodes = [2 * c for c in corners]
        nodes += [(nodes[a] + nodes[b]) // 2 for a, b in T10_EDGES]
        tets.append(np.stack(nodes))     # (10, 3) doubled-grid offsets
    tets = np.stack(tets)                # (6, 10, 3)

    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = 2 * np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)   # (ncell, 3)
    pts = base[:, None, None, :] + tets[None]                           # (ncell, 6, 10, 3)
    ids = (pts[..., 0] * gy + pts[..., 1]) * gz + pts[..., 2]
    conn = ids.reshape(-1, 10).astype(np.int32)
    return Mesh(T10, X, conn)


def ancf3443_plate(nx: int, ny: int, lx: float, ly: float, thickness: float,
                   gl=(3, 3, 2)) -> Mesh:
    """Flat rectangular ANCF3443 plate in the z = 0 plane, reference gradients
    r_x = e_x, r_y = e_y, r_z = e_z."""
    ix, iy = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    pos = np.stack([ix.ravel() * (lx / nx), iy.ravel() * (ly / ny),
                    np.zeros(ix.size)], axis=1)
    n_nodes = pos.shape[0]
    X = np.zeros((4 * n_nodes, 3))
    X[0::4] = pos
    X[1::4] = (1.0, 0.0, 0.0)
    X[2::4] = (0.0, 1.0, 0.0)
    X[3::4] = (0.0, 0.0, 1.0)
    ex, ey = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ex, ey = ex.ravel(), ey.ravel()
    node = lambda a, b: a * (ny + 1) + b
    conn = np.stack([node(ex, ey), node(ex + 1, ey), node(ex + 1, ey + 1),
                     node(ex, ey + 1)], axis=1).astype(np.int32)
    return Mesh(ANCF3443, X, conn, gl=tuple(gl), thickness=float(thickness))


def t10_node_count(nx, ny, nz):
    return (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1)


# ----------------------------------------------------------------------------
# the five benchmark configurations
# ----------------------------------------------------------------------------

MR_BASE = dict(mu10=2e5, mu01=5e4, kappa=1e8, eta=1e3)


def _t10_perturbed(mesh: Mesh, h, rng, frac, vel_sigma):
    """q = X + U(-frac*h_k, +frac*h_k) per axis; qdot ~ N(0, vel_sigma^2)."""
    h = np.asarray(h, dtype=np.float64)
    noise = rng.uniform(-1.0, 1.0, size=mesh.X.shape) * (frac * h)[None, :]
    q = (mesh.X + noise).ravel()
    qdot = rng.normal(0.0, vel_sigma, size=q.shape[0])
    return q, qdot


def config1(seed: int = 1001) -> Workload:
    """24 T10 elements, SVK E=1e7 nu=0.3, +-1% position noise, N(0,0.01^2) velocities."""
    rng = np.random.default_rng(seed)
    mesh = kuhn_t10_box(4, 1, 1, 1.0, 0.1, 0.1)
    mat = Material(SVK, (1e7, 0.3, 0.0))
    q, qdot = _t10_perturbed(mesh, (0.25, 0.1, 0.1), rng, 0.01, 0.01)
    w = rng.normal(0.0, 1.0, size=q.shape[0])
    return Workload("t10_box_4x1x1_svk", mesh, mat, q, qdot, w)


def t10_beam(nx, ny, nz, seed, name, lx=1.0, ly=0.1, lz=0.1, frac=0.02, vel_sigma=0.05,
             material: Optional[Material] = None) -> Workload:
    rng = np.random.default_rng(seed)
    mesh = kuhn_t10_box(nx, ny, nz, lx, ly, lz)
    if material is None:
        material = Material(MOONEY_RIVLIN, (MR_BASE["mu10"], MR_BASE["mu01"], MR_BASE["kappa"]),
                            MR_BASE["eta"], MR_BASE["eta"])
    q, qdot = _t10_perturbed(mesh, (lx / nx, ly / ny, lz / nz), rng, frac, vel_sigma)
    w = rng.normal(0.0, 1.0, size=q.shape[0])
    return Workload(name, mesh, material, q, qdot, w)


def config2(seed: int = 1002) -> Workload:
    """30,720 T10 elements (80x8x8 cells), Mooney-Rivlin + Kelvin-Voigt."""
    return t10_beam(80, 8, 8, seed, "t10_beam_80x8x8_mr_kv")


def config5(seed: int = 1005) -> Workload:
    """480,000 T10 elements (200x20x20 cells), Mooney-Rivlin + Kelvin-Voigt."""
    return t10_beam(200, 20, 20, seed, "t10_beam_200x20x20_mr_kv")


def shell_plate(n: int, seed: int, name: str, amp=0.05, noise=1e-3, E=2e9, nu=0.3,
                thickness=0.01, gl=(3, 3, 2)) -> Workload:
    """ANCF3443 plate [0,1]^2 bent into z = amp*sin(pi x) sin(pi y) plus noise."""
    rng = np.random.default_rng(seed)
    mesh = ancf3443_plate(n, n, 1.0, 1.0, thickness, gl)
    pos = mesh.X[0::4]
    x, y = pos[:, 0], pos[:, 1]
    z = amp * np.sin(np.pi * x) * np.sin(np.pi * y)
    zx = amp * np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
    zy = amp * np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
    nrm = np.sqrt(1.0 + zx * zx + zy * zy)
    cur = np.zeros_like(mesh.X)
    cur[0::4] = np.stack([x, y, z], axis=1)
    cur[1::4] = np.stack([np.ones_like(x), np.zeros_like(x), zx], axis=1)
    cur[2::4] = np.stack([np.zeros_like(x), np.ones_like(x), zy], axis=1)
    cur[3::4] = np.stack([-zx / nrm, -zy / nrm, 1.0 / nrm], axis=1)
    le = 1.0 / n
    scale = np.zeros_like(cur)
    scale[0::4] = noise * le
    scale[1::4] = noise
    scale[2::4] = noise
    scale[3::4] = noise
    cur = cur + rng.uniform(-1.0, 1.0, size=cur.shape) * scale
    q = cur.ravel()
    qdot = np.zeros_like(q)
    w = rng.normal(0.0, 1.0, size=q.shape[0])
    mat = Material(SVK, (E, nu, 0.0))
    return Workload(name, mesh, mat, q, qdot, w)


def ancf3243_chain(n_elem: int, L: float = 0.2, W: float = 0.1, H: float = 0.1) -> Mesh:
    """A straight chain of ANCF3243 beam elements along x (element e spans
    nodes e and e+1); per node the coefficients r, r_x, r_y, r_z of the
    reference configuration."""
    n = n_elem + 1
    x = L * np.arange(n)
    X = np.zeros((4 * n, 3))
    X[0::4, 0] = x
    X[1::4, 0] = 1.0
    X[2::4, 1] = 1.0
    X[3::4, 2] = 1.0
    conn = np.stack([np.arange(n_elem), np.arange(1, n)], axis=1).astype(np.int32)
    return Mesh(ANCF3243, X, conn, (3, 2, 2), H, W)


def beam_3243(n_elem: int, seed: int, name: str, amp=0.02, noise=1e-3, vel_sigma=0.05,
              material: Optional[Material] = None) -> Workload:
    """ANCF3243 chain (L = 0.2, W = H = 0.1) bent into z = amp sin(pi s) over
    its length (s = x / length), with r_x, r_z following the curve, noise on
    every coefficient and random velocities; SVK E = 7e8, nu = 0.33 by default."""
    rng = np.random.default_rng(seed)
    mesh = ancf3243_chain(n_elem)
    span = 0.2 * n_elem
    x = mesh.X[0::4, 0]
    z = amp * np.sin(np.pi * x / span)
    zx = amp * np.pi / span * np.cos(np.pi * x / span)
    nrm = np.sqrt(1.0 + zx * zx)
    cur = np.zeros_like(mesh.X)
    cur[0::4] = np.stack([x, np.zeros_like(x), z], axis=1)
    cur[1::4] = np.stack([np.ones_like(x), np.zeros_like(x), zx], axis=1)
    cur[2::4] = np.stack([np.zeros_like(x), np.ones_like(x), np.zeros_like(x)], axis=1)
    cur[3::4] = np.stack([-zx / nrm, np.zeros_like(x), 1.0 / nrm], axis=1)
    scale = np.full_like(cur, noise)
    scale[0::4] = noise * 0.2
    cur = cur + rng.uniform(-1.0, 1.0, size=cur.shape) * scale
    q = cur.ravel()
    qdot = rng.normal(0.0, vel_sigma, size=q.shape[0])
    w = rng.normal(0.0, 1.0, size=q.shape[0])
    mat = material if material is not None else Material(SVK, (7e8, 0.33, 0.0))
    return Workload(name, mesh, mat, q, qdot, w)


def beam_res32(seed: int = 1006) -> Workload:
    """The paper's largest ANCF3243 scaling resolution (Sec. 5, ANCF3243 beam
    element scaling): a 500,000-element chain, 500,001 nodes, 6,000,012 DOF,
    L = 0.2, W = H = 0.1, SVK E = 7e8, nu = 0.33."""
    return beam_3243(500_000, seed, "ancf3243_chain_500000_svk")


def config3(seed: int = 1003) -> Workload:
    """65,536 ANCF3443 shell elements (256x256), SVK E=2e9 nu=0.3, GL 3x3x2."""
    return shell_plate(256, seed, "ancf3443_plate_256x256_svk")


def svk_from_mr(mu10, mu01, kappa):
    """Small-strain equivalent (E, nu) of shear 2(mu10+mu01) and bulk kappa."""
    mu = 2.0 * (mu10 + mu01)
    K = kappa
    E = 9.0 * K * mu / (3.0 * K + mu)
    nu = (3.0 * K - 2.0 * mu) / (2.0 * (3.0 * K + mu))
    return E, nu


def batched_bodies(n_bodies: int = 512, seed: int = 1004, n_lo: int = 2, n_hi: int = 12,
                   side: float = 0.1) -> List[Workload]:
    """Independent T10 cubes of n^3 cells (n uniform in [n_lo, n_hi]); material
    alternates SVK / Mooney-Rivlin with every parameter scaled by U(0.8, 1.2)."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, n_bodies)
    mats = []
    for b in range(n_bodies):
        s = rng.uniform(0.8, 1.2, size=4)
        eta = MR_BASE["eta"] * s[3]
        if b % 2 == 0:
            # SVK: scale the shear modulus 2(mu10+mu01) and the bulk modulus kappa
            # (scaling nu itself could push it past 1/2), then convert to (E, nu)
            E, nu = svk_from_mr(MR_BASE["mu10"] * s[0], MR_BASE["mu01"] * s[0], MR_BASE["kappa"] * s[2])
            mats.append(Material(SVK, (E, nu, 0.0), eta, eta))
        else:
            mats.append(Material(MOONEY_RIVLIN, (MR_BASE["mu10"] * s[0], MR_BASE["mu01"] * s[1],
                                                 MR_BASE["kappa"] * s[2]), eta, eta))
    meshes = [kuhn_t10_box(int(n), int(n), int(n), side, side, side) for n in sizes]
    qs, qdots = [], []
    for mesh, n in zip(meshes, sizes):
        h = side / n
        noise = rng.uniform(-1.0, 1.0, size=mesh.X.shape) * (0.02 * h)
        qs.append((mesh.X + noise).ravel())
    for mesh in meshes:
        qdots.append(rng.normal(0.0, 0.05, size=mesh.n_dof))
    out = []
    for b, (mesh, mat, q, qd) in enumerate(zip(meshes, mats, qs, qdots)):
        w = rng.normal(0.0, 1.0, size=q.shape[0])
        out.append(Workload(f"body{b}_n{int(sizes[b])}", mesh, mat, q, qd, w))
    return out


def config4(seed: int = 1004) -> List[Workload]:
    """512 T10 cubes, n in U{2..12}, mixed SVK / Mooney-Rivlin, Kelvin-Voigt on."""
    return batched_bodies(512, seed)


def rotation_matrix(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def t10_rotated(nx, ny, nz, seed, name, angle=1.0, axis=(1.0, 2.0, 3.0), frac=1e-3,
                vel_sigma=0.05, lx=1.0, ly=0.1, lz=0.1,
                material: Optional[Material] = None) -> Workload:
    """A T10 box beam deformed by small noise and then turned as a rigid body.

    The reference box is [0,lx]x[0,ly]x[0,lz] with nx*ny*nz Kuhn cells; every
    node (mid-edge nodes included) is moved by U(-frac*h_k, +frac*h_k) per axis,
    which gives strains of order frac, and the perturbed body is rotated by
    ``angle`` radians about ``axis`` through the origin.  Far from the origin
    the rigid displacement is of the body's own size while the strain stays of
    order frac: the regime of a beam that bends through a large rotation.
    Velocities are N(0, vel_sigma^2) per DOF.  Draw order: position noise,
    velocity noise, cotangent."""
    rng = np.random.default_rng(seed)
    mesh = kuhn_t10_box(nx, ny, nz, lx, ly, lz)
    if material is None:
        material = Material(MOONEY_RIVLIN, (MR_BASE["mu10"], MR_BASE["mu01"], MR_BASE["kappa"]),
                            MR_BASE["eta"], MR_BASE["eta"])
    q, qdot = _t10_perturbed(mesh, (lx / nx, ly / ny, lz / nz), rng, frac, vel_sigma)
    R = rotation_matrix(axis, angle)
    q = (q.reshape(-1, 3) @ R.T).ravel()
    w = rng.normal(0.0, 1.0, size=q.shape[0])
    return Workload(name, mesh, material, q, qdot, w)
