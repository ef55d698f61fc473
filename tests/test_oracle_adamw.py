"""Pins of the oracle's first-order solver (Sec. 4.5, Alg. 2 without
constraints): the exact shape of its first two iterations, and convergence to
the root of the gradient found by Newton's method with the oracle's Newton
matrix (itself tied to the gradient by finite differences)."""
import numpy as np

import oracle
from paper_2604_10357_amd import workloads as W


def setup(seed=101):
    wl = W.t10_beam(2, 1, 1, seed, "adamw_pin", lx=0.2, ly=0.1, lz=0.1, frac=0.002)
    om = oracle.Mesh.of(wl.mesh)
    omat = oracle.material_of(wl.material)
    pat = oracle.csr_pattern(om)
    mv = oracle.mass_csr(om, 1000.0, pat)
    rng = np.random.default_rng(seed)
    v_n = rng.normal(0, 0.01, wl.mesh.n_dof)
    return wl, om, omat, pat, mv, v_n


def test_first_two_iterations():
    """From g = m = s = 0 the first iteration only decays v.  In the second only
    g_1 has entered the moments: m = (1 - b1) g_1, s = (1 - b2) g_1^2, so with
    the bias corrections of l = 2, m_hat = g_1 / (1 + b1) and
    s_hat = g_1^2 / (1 + b2): a step of lr sqrt(1 + b2) / (1 + b1) against the
    sign of g_1 in every component."""
    wl, om, omat, pat, mv, v_n = setup()
    h, lr, wd, eps = 1e-3, 1e-3, 0.01, 1e-30
    v0 = v_n.copy()
    v1, _, g1 = oracle.adamw_solve(om, omat, pat, mv, wl.q, v_n, None, v0, h, lr, 0.9, 0.999, eps, wd, 1)
    assert np.array_equal(v1, (1 - lr * wd) * v0)
    v2, _, _ = oracle.adamw_solve(om, omat, pat, mv, wl.q, v_n, None, v0, h, lr, 0.9, 0.999, eps, wd, 2)
    step = (1 - lr * wd) * v1 - v2
    assert np.allclose(step, lr * np.sqrt(1.999) / 1.9 * np.sign(g1), rtol=1e-12, atol=1e-18)


def test_converges_to_the_newton_root():
    wl, om, omat, pat, mv, v_n = setup()
    h = 1e-3
    ro, cols = pat
    n = wl.mesh.n_dof

    def g_of(v):
        f, _ = oracle.assemble(om, omat, wl.q + h * v, v, 1.0, 0.0, pattern=pat, want_K=False)
        return oracle.gradient(pat, mv, v, v_n, f, None, h)

    v = v_n.copy()
    for _ in range(8):  # Newton on g(v) = 0 with H = M/h + h df/dq + df/dqdot
        _, K = oracle.assemble(om, omat, wl.q + h * v, v, h, 1.0, pattern=pat)
        Hv = mv / h + K
        H = np.zeros((n, n))
        for r in range(n):
            H[r, cols[ro[r]:ro[r + 1]]] = Hv[ro[r]:ro[r + 1]]
        v = v - np.linalg.solve(H, g_of(v))
    v_star = v
    assert np.abs(g_of(v_star)).max() <= 1e-9 * np.abs(g_of(v_n)).max()
    span = np.abs(v_star - v_n).max()
    lr = 1e-2 * span
    va, _, ga = oracle.adamw_solve(om, omat, pat, mv, wl.q, v_n, None, v_n, h, lr, 0.9, 0.999, 1e-12, 0.0, 3000)
    assert np.abs(va - v_star).max() <= 1e-2 * span
    assert np.linalg.norm(ga) <= 1e-3 * np.linalg.norm(g_of(v_n))
