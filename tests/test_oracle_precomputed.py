"""Pins of the oracle's precomputed sparse points (Section 3.2: a custom
interpolation scheme given as grid points and coefficients per sparse point,
behaving like a sparse function with linear weights).

* with r = 2 and the coefficients (1 - f, f) at base floor(xi) the precomputed
  functions are the linear ones, bit for bit, and so is a whole operator run;
* an r = 4 Lagrange scheme reproduces any polynomial of degree <= 3 per axis
  exactly (closed form of Lagrange interpolation);
* injection is the transpose of interpolation (dot-product identity);
* a support point outside the grid is rejected.
"""
import numpy as np
import pytest

import oracle
from paper_1807_03032_amd import workloads as W


def grid(shape, so=4, nbl=0, dt=1e-3):
    extent = tuple(10.0 * (n - 1) for n in shape)
    origin = tuple(3.0 * (a + 1) for a in range(len(shape)))
    return oracle.Grid(shape, extent, origin, so=so, dt=dt, nbl=nbl, vmax=2000.0)


def linear_support(g, coords):
    """gridpoints / coeffs that reproduce the linear weights: base floor(xi)
    clamped to n - 2, coefficients (1 - f, f)."""
    c = np.asarray(coords, dtype=np.float64).reshape(-1, g.ndim)
    gp = np.zeros(c.shape, dtype=np.int64)
    cf = np.zeros(c.shape + (2,))
    for p in range(c.shape[0]):
        for a in range(g.ndim):
            xi = (c[p, a] - g.origin[a]) / g.spacing[a]
            b = min(int(np.floor(xi)), g.shape[a] - 2)
            f = xi - b
            gp[p, a] = b
            cf[p, a] = (1.0 - f, f)
    return gp, cf


def random_coords(g, n, rng, margin=0.0):
    lo = np.array(g.origin) + margin * np.array(g.spacing)
    hi = np.array(g.origin) + (np.array(g.shape) - 1 - margin) * np.array(g.spacing)
    return lo + rng.random((n, g.ndim)) * (hi - lo)


@pytest.mark.parametrize("shape", [(23,), (19, 14), (11, 9, 8)])
def test_linear_precomputed_equals_linear(shape):
    g = grid(shape)
    rng = np.random.default_rng(11)
    coords = random_coords(g, 17, rng)
    # points on the last node and on the origin take the clamped base
    coords[0] = np.array(g.origin) + (np.array(g.shape) - 1) * np.array(g.spacing)
    coords[1] = np.array(g.origin)
    gp, cf = linear_support(g, coords)
    u = rng.standard_normal(g.array_shape)
    assert np.array_equal(oracle.interp_pre(g, gp, cf, u), oracle.interp(g, coords, u))
    q = rng.standard_normal(coords.shape[0])
    m = 1.0 + rng.random(g.array_shape)
    assert np.array_equal(oracle.inject_pre(g, gp, cf, q, u, scale=0.3, m=m),
                          oracle.inject(g, coords, q, u, scale=0.3, m=m))


@pytest.mark.parametrize("shape", [(29, 23), (15, 13, 12)])
def test_linear_precomputed_run_equals_run(shape):
    g = grid(shape, so=4, nbl=3, dt=1e-3)
    rng = np.random.default_rng(5)
    m = 1.0 / (1500.0 + 500.0 * rng.random(g.array_shape)) ** 2
    nt = 12
    sc, rc = random_coords(g, 3, rng), random_coords(g, 9, rng)
    src = rng.standard_normal((nt, 3))
    ref = oracle.iso_run(g, m, nt, src_coords=sc, src=src, rec_coords=rc)
    got = oracle.iso_run_pre(g, m, nt, linear_support(g, sc), src, linear_support(g, rc))
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(31,), (17, 15), (11, 10, 9)])
def test_lagrange_cubic_reproduces_cubics(shape):
    g = grid(shape)
    rng = np.random.default_rng(3)
    coords = random_coords(g, 25, rng)
    gp, cf = W.lagrange_support(g.shape, g.spacing, g.origin, coords, 4)
    # u = prod_a P_a(i_a), P_a a random cubic of the grid index
    P = rng.standard_normal((g.ndim, 4))
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in g.shape], indexing="ij")
    u = np.ones(g.shape)
    for a in range(g.ndim):
        u = u * np.polyval(P[a], idx[a])
    u = np.ascontiguousarray(u.T)  # numpy order: first axis fastest
    xi = (coords - np.array(g.origin)) / np.array(g.spacing)
    exact = np.prod([np.polyval(P[a], xi[:, a]) for a in range(g.ndim)], axis=0)
    got = oracle.interp_pre(g, gp, cf, u)
    assert np.max(np.abs(got - exact)) <= 1e-10 * np.max(np.abs(exact))
    # a degree-4 polynomial is not reproduced (the pin can fail)
    u4 = np.ascontiguousarray((idx[0] ** 4).T)
    assert np.max(np.abs(oracle.interp_pre(g, gp, cf, u4) - xi[:, 0] ** 4)) > 1e-3


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_inject_is_transpose_of_interp(r):
    g = grid((13, 12, 11))
    rng = np.random.default_rng(100 + r)
    coords = random_coords(g, 7, rng)
    gp, cf = W.lagrange_support(g.shape, g.spacing, g.origin, coords, r)
    u = rng.standard_normal(g.array_shape)
    q = rng.standard_normal(7)
    lhs = float(np.dot(oracle.interp_pre(g, gp, cf, u), q))
    rhs = float(np.sum(u * oracle.inject_pre(g, gp, cf, q, np.zeros(g.array_shape))))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_support_outside_grid_is_rejected():
    g = grid((10, 9))
    gp = np.array([[7, 2]], dtype=np.int64)
    cf = np.full((1, 2, 4), 0.25)  # x support 7..10 leaves the 10-point axis
    with pytest.raises(oracle.OracleError):
        oracle.interp_pre(g, gp, cf, np.zeros(g.array_shape))
    gp = np.array([[-1, 2]], dtype=np.int64)
    with pytest.raises(oracle.OracleError):
        oracle.inject_pre(g, gp, cf, [1.0], np.zeros(g.array_shape))
