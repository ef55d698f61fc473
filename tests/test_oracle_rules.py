"""Pins of the oracle's quadrature rules and shape functions against closed forms.

The paper names the rules (5-point Keast for T10, Gauss-Legendre products for
ANCF; Sec. 4.3, Stage 1) and the element families (Sec. 4.1) but prints no
tables, so every value here is checked against mathematics: exact monomial
integrals, interpolation (Kronecker) conditions and polynomial reproduction.
"""
import math

import numpy as np
import pytest

from paper_2604_10357_amd import workloads as W


def tet_monomial_integral(a, b, c):
    # integral over the unit tetrahedron of xi^a eta^b zeta^c
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def test_keast_exact_to_degree_3(orc):
    pts, w = orc.quadrature(orc.T10)
    assert pts.shape == (5, 3)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    assert w[0] < 0  # the Keast rule's negative centroid weight
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
                assert abs(got - tet_monomial_integral(a, b, c)) < 1e-15, (a, b, c)


def test_keast_not_exact_at_degree_4(orc):
    # a degree-3 rule must miss some quartic: guards against a wrong (higher) rule
    pts, w = orc.quadrature(orc.T10)
    got = np.sum(w * pts[:, 0] ** 4)
    assert abs(got - tet_monomial_integral(4, 0, 0)) > 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_gauss_legendre_exact(orc, n):
    x, w = orc.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14, (n, k)
    k = 2 * n  # first degree a Gauss rule misses
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > 1e-8


def test_ancf_product_rule(orc):
    pts, w = orc.quadrature(orc.ANCF3443, (3, 3, 2))
    assert pts.shape == (18, 3)
    assert abs(w.sum() - 8.0) < 1e-14
    # x^4 y^2 z^2 is integrated exactly by 3x3x2
    got = np.sum(w * pts[:, 0] ** 4 * pts[:, 1] ** 2 * pts[:, 2] ** 2)
    assert abs(got - (2 / 5) * (2 / 3) * (2 / 3)) < 1e-14
    pts, w = orc.quadrature(orc.ANCF3443, (4, 4, 3))
    assert pts.shape == (48, 3)


# ---------------------------------------------------------------- T10

T10_PARENT_NODES = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)


def t10_parent_node_coords():
    corners = T10_PARENT_NODES
    mids = [(corners[a] + corners[b]) / 2 for a, b in W.T10_EDGES]
    return np.vstack([corners, np.array(mids)])


def test_t10_kronecker_and_unity(orc):
    nodes = t10_parent_node_coords()
    for b, xb in enumerate(nodes):
        N, dN = orc.t10_shape(xb)
        expect = np.zeros(10)
        expect[b] = 1.0
        assert np.abs(N - expect).max() < 1e-15
    rng = np.random.default_rng(0)
    for _ in range(20):
        xi = rng.dirichlet(np.ones(4))[1:]
        N, dN = orc.t10_shape(xi)
        assert abs(N.sum() - 1.0) < 1e-14
        assert np.abs(dN.sum(axis=0)).max() < 1e-13


def test_t10_reproduces_quadratics_and_gradients(orc):
    nodes = t10_parent_node_coords()
    rng = np.random.default_rng(1)
    coef = rng.normal(size=10)

    def p(x):  # random full quadratic
        xi, eta, ze = x
        return (coef[0] + coef[1] * xi + coef[2] * eta + coef[3] * ze + coef[4] * xi * xi + coef[5] * eta * eta
                + coef[6] * ze * ze + coef[7] * xi * eta + coef[8] * eta * ze + coef[9] * xi * ze)

    def dp(x):
        xi, eta, ze = x
        return np.array([coef[1] + 2 * coef[4] * xi + coef[7] * eta + coef[9] * ze,
                         coef[2] + 2 * coef[5] * eta + coef[7] * xi + coef[8] * ze,
                         coef[3] + 2 * coef[6] * ze + coef[8] * eta + coef[9] * xi])

    vals = np.array([p(x) for x in nodes])
    for _ in range(20):
        xi = rng.dirichlet(np.ones(4))[1:]
        N, dN = orc.t10_shape(xi)
        assert abs(N @ vals - p(xi)) < 1e-13
        assert np.abs(vals @ dN - dp(xi)).max() < 1e-12


# ---------------------------------------------------------------- ANCF3443

def adini_closed_form(s, t, lx, ly, H, zeta):
    """Closed-form ANCF3443 shape functions, derived independently of the
    oracle: Adini-type value / slope functions per corner and the bilinear
    transverse function."""
    corners = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    S = np.zeros(16)
    for p, (sp, tp) in enumerate(corners):
        s0, t0 = sp * s, tp * t
        S[4 * p + 0] = (1 + s0) * (1 + t0) * (2 + s0 + t0 - s * s - t * t) / 8
        S[4 * p + 1] = lx / 2 * sp * (1 + s0) ** 2 * (s0 - 1) * (1 + t0) / 8
        S[4 * p + 2] = ly / 2 * tp * (1 + t0) ** 2 * (t0 - 1) * (1 + s0) / 8
        S[4 * p + 3] = H * zeta / 2 * (1 + s0) * (1 + t0) / 4
    return S


def test_ancf_matches_closed_form(orc):
    rng = np.random.default_rng(2)
    for _ in range(10):
        xi = rng.uniform(-1, 1, 3)
        lx, ly, H = rng.uniform(0.1, 2.0, 3)
        S, dS = orc.ancf3443_shape(xi, lx, ly, H)
        assert np.abs(S - adini_closed_form(xi[0], xi[1], lx, ly, H, xi[2])).max() < 1e-12
        # parent derivatives against central differences of the closed form
        for m in range(3):
            e = np.zeros(3)
            e[m] = 1e-6
            fd = (adini_closed_form(*(xi + e)[:2], lx, ly, H, (xi + e)[2])
                  - adini_closed_form(*(xi - e)[:2], lx, ly, H, (xi - e)[2])) / 2e-6
            assert np.abs(dS[:, m] - fd).max() < 1e-8


def test_ancf_interpolation_conditions(orc):
    lx, ly, H = 0.3, 0.7, 0.05
    corners = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    for p, (sp, tp) in enumerate(corners):
        S, dS = orc.ancf3443_shape(np.array([sp, tp, 0.0]), lx, ly, H)
        for r in range(4):
            # value: only r of this node; x-slope: only r_x; y-slope: only r_y
            assert abs(S[4 * r + 0] - (1.0 if r == p else 0.0)) < 1e-14
            assert abs(dS[4 * r + 1, 0] * 2 / lx - (1.0 if r == p else 0.0)) < 1e-13
            assert abs(dS[4 * r + 2, 1] * 2 / ly - (1.0 if r == p else 0.0)) < 1e-13
            assert abs(dS[4 * r + 1, 1]) < 1e-13 and abs(dS[4 * r + 2, 0]) < 1e-13
            assert abs(dS[4 * r + 0, 0]) < 1e-13 and abs(dS[4 * r + 0, 1]) < 1e-13


def test_ancf_reproduces_flat_reference(orc):
    # r = (x, y, 0), r_x = e_x, r_y = e_y, r_z = e_z on a lx x ly element: the
    # interpolated field must be exactly the parent-to-physical map
    lx, ly, H = 0.4, 0.25, 0.02
    corners = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    coefs = np.zeros((16, 3))
    for p, (sp, tp) in enumerate(corners):
        coefs[4 * p] = (sp * lx / 2, tp * ly / 2, 0)
        coefs[4 * p + 1] = (1, 0, 0)
        coefs[4 * p + 2] = (0, 1, 0)
        coefs[4 * p + 3] = (0, 0, 1)
    rng = np.random.default_rng(3)
    for _ in range(10):
        xi = rng.uniform(-1, 1, 3)
        S, dS = orc.ancf3443_shape(xi, lx, ly, H)
        r = S @ coefs
        assert np.abs(r - np.array([xi[0] * lx / 2, xi[1] * ly / 2, xi[2] * H / 2])).max() < 1e-14
        J0 = coefs.T @ dS
        assert np.abs(J0 - np.diag([lx / 2, ly / 2, H / 2])).max() < 1e-14
