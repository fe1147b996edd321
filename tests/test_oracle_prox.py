"""Pins for oracle/prox.py: optimality conditions and brute-force minimisation."""

import numpy as np

import oracle as O


def test_mask_prox_optimality_and_special_cases():
    g = np.random.default_rng(0)
    v = g.standard_normal((6, 7))
    y = g.standard_normal((6, 7))
    m = (g.uniform(size=(6, 7)) < 0.6).astype(np.uint8)
    mu = 0.37
    u = O.mask_prox(v, y, m, mu)
    # gradient of 1/2 m (y - u)^2 + mu/2 (u - v)^2 vanishes
    np.testing.assert_allclose(m * (u - y) + mu * (u - v), 0.0, atol=1e-14)
    # unobserved pixels: u = v (y there is ignored), observed: eq. (15)
    np.testing.assert_allclose(u[m == 0], v[m == 0], atol=1e-15)
    np.testing.assert_allclose(u[m == 1], ((y + mu * v) / (1 + mu))[m == 1], atol=1e-15)
    # y values off the mask do not matter
    y2 = np.where(m == 1, y, 1e6)
    np.testing.assert_allclose(O.mask_prox(v, y2, m, mu), u, atol=1e-15)


def test_mask_prox_brute_force_scalar():
    t = np.linspace(-3, 3, 600001)
    for (v, y, m, mu) in [(0.3, -1.2, 1, 0.5), (1.7, 0.4, 0, 2.0), (-0.8, 0.9, 1, 1e-3)]:
        f = 0.5 * m * (y - t) ** 2 + 0.5 * mu * (t - v) ** 2
        best = t[np.argmin(f)]
        assert abs(O.mask_prox(np.array(v), np.array(y), np.array(m), mu) - best) < 2e-5


def test_vsoft_optimality():
    g = np.random.default_rng(1)
    vh, vv = g.standard_normal(500), g.standard_normal(500)
    tau = 0.8
    uh, uv = O.vsoft(vh, vv, tau)
    rho = np.hypot(vh, vv)
    nu = np.hypot(uh, uv)
    small = rho <= tau
    assert np.all(nu[small] == 0.0)
    big = ~small
    # u - v + tau u / ||u|| = 0 on the rest
    np.testing.assert_allclose(uh[big] - vh[big] + tau * uh[big] / nu[big], 0, atol=1e-13)
    np.testing.assert_allclose(uv[big] - vv[big] + tau * uv[big] / nu[big], 0, atol=1e-13)
    # 0/0 convention
    zh, zv = O.vsoft(np.zeros(3), np.zeros(3), tau)
    assert np.all(zh == 0) and np.all(zv == 0)


def test_vsoft_brute_force_grid():
    # minimise tau ||u|| + 1/2 ||u - v||^2 over a 2-D grid
    tau = 0.5
    grid = np.linspace(-2, 2, 1601)
    U, V = np.meshgrid(grid, grid, indexing="ij")
    for vh, vv in [(1.0, 0.7), (0.2, -0.3), (-1.5, 0.1)]:
        f = tau * np.hypot(U, V) + 0.5 * ((U - vh) ** 2 + (V - vv) ** 2)
        i = np.unravel_index(np.argmin(f), f.shape)
        uh, uv = O.vsoft(np.array([vh]), np.array([vv]), tau)
        assert abs(uh[0] - U[i]) < 4e-3 and abs(uv[0] - V[i]) < 4e-3


def test_soft_brute_force_and_sign_zero():
    t = np.linspace(-4, 4, 800001)
    tau = 0.7
    for v in [-2.3, -0.5, 0.0, 0.69, 1.9]:
        f = tau * np.abs(t) + 0.5 * (t - v) ** 2
        assert abs(O.soft(np.array(v), tau) - t[np.argmin(f)]) < 2e-5
    assert O.soft(np.array(0.0), tau) == 0.0
