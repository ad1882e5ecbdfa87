"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test targets one part of the oracle with a check that does not reuse the
oracle's own code path: exact rational closed forms, polynomial exactness,
the paper's so = 2 listings, exact discrete Fourier-mode solutions, discrete
energy conservation, symmetry / reciprocity of the discrete Green's function,
adjointness of injection and interpolation, and an independent dense
brute-force stepper on tiny grids (tests/brute.py).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------- FD weights
@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_weights_closed_form(so):
    R = so // 2
    w2 = oracle.fd_weights(so, 2)
    w1 = oracle.fd_weights(so, 1)
    e2 = [float(x) for x in brute.taylor_w2(R)]
    e1 = [float(x) for x in brute.taylor_w1(R)]
    np.testing.assert_allclose(w2, e2, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(w1, e1, rtol=1e-13, atol=1e-15)


def test_weights_quoted_values():
    # so = 4: [-5/2, 4/3, -1/12]; so = 8: [-205/72, 8/5, -1/5, 8/315, -1/560]
    np.testing.assert_allclose(oracle.fd_weights(4, 2), [-5 / 2, 4 / 3, -1 / 12], rtol=1e-14)
    np.testing.assert_allclose(oracle.fd_weights(8, 2), [-205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560], rtol=1e-14)
    np.testing.assert_allclose(oracle.fd_weights(8, 1)[1:], [4 / 5, -1 / 5, 4 / 105, -1 / 280], rtol=1e-14)


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16])
def test_weights_polynomial_exactness(so):
    """Order-so stencils differentiate x^p exactly for p <= so (+1 for the even 2nd derivative)."""
    R = so // 2
    w2 = [Fraction(x).limit_denominator(10 ** 12) for x in oracle.fd_weights(so, 2)]
    w1 = [Fraction(x).limit_denominator(10 ** 12) for x in oracle.fd_weights(so, 1)]
    x0 = Fraction(3)
    for p in range(0, so + 2):
        f = lambda x: x ** p  # noqa: E731
        d2 = w2[0] * f(x0) + sum(w2[k] * (f(x0 + k) + f(x0 - k)) for k in range(1, R + 1))
        exact2 = p * (p - 1) * x0 ** (p - 2) if p >= 2 else 0
        assert abs(float(d2 - exact2)) <= 1e-6 * max(1.0, abs(float(exact2))), (p, d2, exact2)
        if p <= so:
            d1 = sum(w1[k] * (f(x0 + k) - f(x0 - k)) for k in range(1, R + 1))
            exact1 = p * x0 ** (p - 1) if p >= 1 else 0
            assert abs(float(d1 - exact1)) <= 1e-6 * max(1.0, abs(float(exact1))), (p, d1, exact1)


def test_listing_fd1_so2_weights():
    gold = json.load(open(os.path.join(GOLDEN, "listings_so2_1d.json")))
    dx = gold["fd1_dx_weights_over_h"]
    assert oracle.fd_weights(2, 1)[1] == float(Fraction(dx["1"]))
    dt2 = gold["fd1_dt2_weights_over_dt2"]
    w2 = oracle.fd_weights(2, 2)
    assert w2[0] == float(Fraction(dt2["0"])) and w2[1] == float(Fraction(dt2["1"]))


# ---------------------------------------------------- Listings fd-3 / finject
def test_listing_fd3_and_finject_1d():
    """One step of the 1-D so = 2 operator equals Listing fd-3's update plus
    Listing finject's two increments, evaluated in exact rationals."""
    gold = json.load(open(os.path.join(GOLDEN, "listings_so2_1d.json")))["case"]
    F = Fraction
    nx, h, dt = gold["nx"], F(gold["h"]), F(gold["dt"])
    m = [F(v) for v in gold["m"]]
    up = [F(v) for v in gold["u_prev"]]
    uc = [F(v) for v in gold["u_cur"]]
    c, q = F(gold["src_coord"]), F(gold["q0"])
    at = lambda u, i: u[i] if 0 <= i < nx else F(0)  # noqa: E731  (zero halo)
    exp = [-2 * dt ** 2 * at(uc, x) / (h ** 2 * m[x]) + dt ** 2 * at(uc, x - 1) / (h ** 2 * m[x])
           + dt ** 2 * at(uc, x + 1) / (h ** 2 * m[x]) + 2 * at(uc, x) - at(up, x) for x in range(nx)]
    x1 = math.floor(c / h)
    f = c / h - x1
    exp[x1] += dt ** 2 * (1 - f) * q / m[x1]
    exp[x1 + 1] += dt ** 2 * f * q / m[x1 + 1]
    g = oracle.Grid((nx,), (float(h * (nx - 1)),), so=2, dt=float(dt))
    _, u1, _ = oracle.iso_run(g, np.array([float(v) for v in m]), 1, np.array([float(v) for v in up]),
                              np.array([float(v) for v in uc]), src_coords=[[float(c)]],
                              src=np.array([[float(q)]]))
    np.testing.assert_allclose(u1, [float(v) for v in exp], rtol=1e-13, atol=1e-13)


# --------------------------------------------------------- spatial operators
@pytest.mark.parametrize("so", [4, 8])
def test_laplacian_convergence_order(so):
    """Error of L on a smooth periodic field falls as h^so."""
    errs = []
    for n in (24, 48):
        L = 2 * math.pi
        g = oracle.Grid((n, n), (L * (n - 1) / n, L * (n - 1) / n), so=so, periodic=True)
        x = np.arange(n) * L / n
        X, Z = np.meshgrid(x, x, indexing="xy")  # numpy order (z, x)
        u = np.sin(X) * np.cos(2 * Z)
        lap = oracle.laplacian(g, u)
        errs.append(np.abs(lap + 5 * u).max())
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - so) < 0.5, (errs, rate)


@pytest.mark.parametrize("so", [4, 8])
def test_deriv1_convergence_order(so):
    errs = []
    for n in (24, 48):
        L = 2 * math.pi
        g = oracle.Grid((n, n, 4), (L * (n - 1) / n, L * (n - 1) / n, 3.0), so=so, periodic=True)
        x = np.arange(n) * L / n
        u = np.broadcast_to(np.sin(3 * x)[None, None, :], (4, n, n)).copy()
        d = oracle.deriv1(g, 0, u)
        errs.append(np.abs(d - 3 * np.cos(3 * x)[None, None, :]).max())
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - so) < 0.5, (errs, rate)


# ------------------------------------------------- exact Fourier-mode solution
@pytest.mark.parametrize("ndim,so", [(2, 4), (3, 8), (2, 12), (3, 16)])
def test_fourier_mode_exact(ndim, so):
    """On a periodic grid with eta = 0, u0 = phi, u_-1 = cos(theta) phi gives
    u_n = cos(n theta) phi exactly, cos(theta) = 1 - v^2 dt^2 lambda / 2, lambda
    the eigenvalue of -L on the mode (from the closed-form weights)."""
    shape = (12, 10, 8)[:ndim]
    h = (7.0, 9.0, 11.0)[:ndim]
    kk = (2, 3, 1)[:ndim]
    v = 1500.0
    R = so // 2
    w2 = [float(x) for x in brute.taylor_w2(R)]
    lam = 0.0
    for a in range(ndim):
        kap = 2 * math.pi * kk[a] / shape[a]
        lam += -(w2[0] + 2 * sum(w2[k] * math.cos(k * kap) for k in range(1, R + 1))) / h[a] ** 2
    lam_max = sum(-(w2[0] + 2 * sum(w2[k] * (-1) ** k for k in range(1, R + 1))) / h[a] ** 2 for a in range(ndim))
    dt = 0.5 * 2 / (v * math.sqrt(lam_max))  # stable for every mode of the grid
    cth = 1 - v * v * dt * dt * lam / 2
    th = math.acos(cth)
    idx = np.indices(tuple(reversed(shape)))[::-1]
    phi = np.ones(tuple(reversed(shape)))
    for a in range(ndim):
        phi = phi * np.cos(2 * math.pi * kk[a] * idx[a] / shape[a] + 0.3 * a)
    ext = tuple(hh * (n - 1) for hh, n in zip(h, shape))
    g = oracle.Grid(shape, ext, so=so, dt=dt, periodic=True)
    nt = 200
    m = np.full(phi.shape, 1 / v ** 2)
    up, uc, _ = oracle.iso_run(g, m, nt, u_prev=cth * phi, u_cur=phi)
    np.testing.assert_allclose(uc, math.cos(nt * th) * phi, atol=1e-10)
    np.testing.assert_allclose(up, math.cos((nt - 1) * th) * phi, atol=1e-10)


# ----------------------------------------- convergence to the wave equation
@pytest.mark.parametrize("so", [8, 16])
def test_standing_wave_converges_second_order(so):
    """The leapfrog march converges to the continuous standing wave
    u = cos(w t) sin(x) cos(2z), w = v sqrt(5), of u_tt = v^2 (u_xx + u_zz):
    with dt proportional to h (exact initial history) the error at a fixed
    time falls as dt^2 -- the time discretisation's order, the spatial error
    h^so being far smaller at these orders (at so = 4 the two are of the same
    size here and of opposite sign, which hides the order)."""
    v, T = 1.0, math.pi
    errs = []
    for n, nt in ((24, 60), (48, 120)):
        L = 2 * math.pi
        h = L / n
        dt = T / nt  # = 0.2 h
        g = oracle.Grid((n, n), (L * (n - 1) / n, L * (n - 1) / n), so=so, dt=dt, periodic=True)
        x = np.arange(n) * h
        X, Z = np.meshgrid(x, x, indexing="xy")  # numpy order (z, x)
        phi = np.sin(X) * np.cos(2 * Z)
        w = v * math.sqrt(5.0)
        m = np.full(phi.shape, 1 / v ** 2)
        _, uc, _ = oracle.iso_run(g, m, nt, u_prev=math.cos(w * dt) * phi, u_cur=phi)
        errs.append(np.abs(uc - math.cos(w * T) * phi).max())
    rate = math.log2(errs[0] / errs[1])
    assert errs[1] < 1e-2 and abs(rate - 2.0) < 0.3, (errs, rate)


# ------------------------------------------------------------- energy checks
def _energy(m, un1, un, dt, Lun):
    return float(np.sum(m * ((un1 - un) / dt) ** 2) - np.sum(un1 * Lun))


@pytest.mark.parametrize("ndim,so", [(2, 8), (3, 4)])
def test_energy_conserved_without_damping(ndim, so):
    """E = sum m((u+ - u)/dt)^2 - sum u+ . L u is constant for the leapfrog with
    symmetric L (Dirichlet zero halo), variable m, no source, no damping.
    L u is computed with the dense brute-force matrix, not the oracle."""
    shape = (9, 8, 7)[:ndim]
    h = (10.0, 12.0, 9.0)[:ndim]
    rng = np.random.default_rng(5)
    ash = tuple(reversed(shape))
    m = 1.0 / rng.uniform(1500, 3000, size=ash) ** 2
    dt = 0.3 * min(h) / (3000 * math.sqrt(ndim))
    u0 = rng.standard_normal(ash)
    um = u0 + 0.01 * rng.standard_normal(ash)
    Ld = brute.laplacian(shape, h, so // 2)
    g = oracle.Grid(shape, tuple(hh * (n - 1) for hh, n in zip(h, shape)), so=so, dt=dt)
    E = []
    up, uc = um, u0
    for _ in range(40):
        up2, uc2, _ = oracle.iso_run(g, m, 1, up, uc)
        E.append(_energy(m, uc2, uc, dt, (Ld @ uc.reshape(-1)).reshape(ash)))
        up, uc = up2, uc2
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-10 * abs(E[0]), E


def test_energy_decays_with_damping():
    shape = (16, 14)
    h = (10.0, 10.0)
    rng = np.random.default_rng(7)
    ash = tuple(reversed(shape))
    m = np.full(ash, 1 / 2000.0 ** 2)
    dt = 0.4 * 10 / (2000 * math.sqrt(2))
    g = oracle.Grid(shape, (150.0, 130.0), so=4, dt=dt, nbl=4, vmax=2000.0)
    Ld = brute.laplacian(shape, h, 2)
    up = uc = rng.standard_normal(ash)
    E = []
    for _ in range(60):
        up2, uc2, _ = oracle.iso_run(g, m, 1, up, uc)
        E.append(_energy(m, uc2, uc, dt, (Ld @ uc.reshape(-1)).reshape(ash)))
        up, uc = up2, uc2
    assert all(E[i + 1] <= E[i] * (1 + 1e-12) for i in range(len(E) - 1))
    assert E[-1] < 0.9 * E[0]


# --------------------------------------------------- symmetry and reciprocity
def test_symmetry_centre_source_2d():
    """Constant velocity, source at the centre node of a 101 x 101 grid:
    receivers mirrored about the centre record identical traces."""
    n = 101
    dt = 0.4 * 10 / (1500 * math.sqrt(2))
    g = oracle.Grid((n, n), (1000.0, 1000.0), so=4, dt=dt, nbl=20, vmax=1500.0)
    m = np.full((n, n), 1 / 1500.0 ** 2)
    nt = 120
    tt = np.arange(nt) * dt - 0.1
    q = ((1 - 2 * (math.pi * 10 * tt) ** 2) * np.exp(-(math.pi * 10 * tt) ** 2))[:, None]
    recx = np.arange(n) * 10.0
    rec = np.stack([recx, np.full(n, 660.0)], axis=1)
    _, _, tr = oracle.iso_run(g, m, nt, src_coords=[[500.0, 500.0]], src=q, rec_coords=rec)
    scale = np.abs(tr).max()
    assert scale > 0
    np.testing.assert_allclose(tr, tr[:, ::-1], atol=1e-13 * scale)


@pytest.mark.parametrize("ndim", [2, 3])
def test_reciprocity_off_grid(ndim):
    """Variable m, no damping: the trace at B from a source at A equals the trace
    at A from a source at B (injection is the adjoint of interpolation and the
    scheme is self-adjoint in the m-weighted inner product)."""
    shape = (14, 12, 10)[:ndim]
    h = (10.0,) * ndim
    ash = tuple(reversed(shape))
    rng = np.random.default_rng(11)
    m = 1 / rng.uniform(1500, 2500, size=ash) ** 2
    dt = 0.4 * 10 / (2500 * math.sqrt(ndim))
    ext = tuple(10.0 * (k - 1) for k in shape)
    g = oracle.Grid(shape, ext, so=8, dt=dt)
    A = np.array([[33.3, 47.1, 21.9][:ndim]])
    B = np.array([[91.7, 60.2, 70.4][:ndim]])
    nt = 80
    q = rng.standard_normal((nt, 1))
    _, _, tab = oracle.iso_run(g, m, nt, src_coords=A, src=q, rec_coords=B)
    _, _, tba = oracle.iso_run(g, m, nt, src_coords=B, src=q, rec_coords=A)
    assert np.abs(tab).max() > 0
    np.testing.assert_allclose(tab, tba, atol=1e-12 * np.abs(tab).max())


# ------------------------------------------------------------------ sparse
@pytest.mark.parametrize("ndim", [2, 3])
def test_inject_is_adjoint_of_interp(ndim):
    shape = (9, 7, 6)[:ndim]
    ext = tuple(5.0 * (k - 1) for k in shape)
    g = oracle.Grid(shape, ext, so=4)
    rng = np.random.default_rng(3)
    coords = rng.uniform(0, 1, size=(13, ndim)) * np.array(ext)
    coords[0] = ext  # last node on every axis (clamped base)
    coords[1] = 0.0
    u = rng.standard_normal(g.array_shape)
    d = rng.standard_normal(13)
    lhs = float(np.dot(oracle.interp(g, coords, u), d))
    rhs = float(np.sum(u * oracle.inject(g, coords, d, np.zeros(g.array_shape))))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)


@pytest.mark.parametrize("ndim", [2, 3])
def test_interp_reproduces_linear_functions(ndim):
    shape = (9, 7, 6)[:ndim]
    ext = tuple(5.0 * (k - 1) for k in shape)
    g = oracle.Grid(shape, ext, origin=(1.0, -2.0, 0.5)[:ndim], so=4)
    rng = np.random.default_rng(4)
    org = np.array(g.origin)
    coords = org + rng.uniform(0, 1, size=(20, ndim)) * np.array(ext)
    idx = np.indices(g.array_shape)[::-1]
    coef = np.array([0.7, -1.3, 2.1])[:ndim]
    f = 0.25 + sum(coef[a] * (g.origin[a] + idx[a] * g.spacing[a]) for a in range(ndim))
    exact = 0.25 + coords @ coef
    np.testing.assert_allclose(oracle.interp(g, coords, f), exact, rtol=1e-13, atol=1e-12)
    base, w = oracle.sparse_setup(g, coords)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=1e-14)
    assert (w >= 0).all()


def test_sparse_rejects_points_outside_grid():
    g = oracle.Grid((5, 5), (4.0, 4.0), so=4)
    with pytest.raises(oracle.OracleError):
        oracle.sparse_setup(g, [[4.0000001, 1.0]])
    with pytest.raises(oracle.OracleError):
        oracle.sparse_setup(g, [[-1e-9, 1.0]])
    base, w = oracle.sparse_setup(g, [[4.0, 4.0]])  # last node: base clamped to n-2, f = 1
    assert list(base[0]) == [3, 3] and w[0, 3] == 1.0


# -------------------------------------------------------------- brute force
@pytest.mark.parametrize("ndim,so,periodic", [(2, 4, False), (2, 8, True), (3, 4, False), (3, 8, False),
                                              (2, 16, False), (3, 12, True)])
def test_iso_matches_dense_brute_force(ndim, so, periodic):
    shape = (11, 9, 8)[:ndim] if so <= 8 else (19, 17, 17)[:ndim]
    h = (10.0, 11.0, 9.0)[:ndim]
    ash = tuple(reversed(shape))
    rng = np.random.default_rng(20 + so)
    m = 1 / rng.uniform(1500, 3000, size=ash) ** 2
    dt = 0.4 * min(h) / (3000 * math.sqrt(ndim))
    ext = tuple(hh * (k - 1) for hh, k in zip(h, shape))
    nbl = 0 if periodic else 3
    g = oracle.Grid(shape, ext, so=so, dt=dt, nbl=nbl, vmax=3000.0, periodic=periodic)
    src_c = rng.uniform(0, 1, size=(2, ndim)) * np.array(ext)
    rec_c = rng.uniform(0, 1, size=(5, ndim)) * np.array(ext)
    nt = 25
    q = rng.standard_normal((nt, 2))
    u0 = rng.standard_normal(ash)
    up, uc, tr = oracle.iso_run(g, m, nt, u_prev=0.5 * u0, u_cur=u0, src_coords=src_c, src=q, rec_coords=rec_c)
    bp, bc, btr = brute.iso_run(shape, h, (0.0,) * ndim, so, dt, nt, m, nbl, 3000.0, src_c, q, rec_c,
                                u_prev=0.5 * u0, u_cur=u0, periodic=periodic)
    sc = np.abs(bc).max()
    np.testing.assert_allclose(uc, bc, atol=1e-12 * sc)
    np.testing.assert_allclose(up, bp, atol=1e-12 * sc)
    np.testing.assert_allclose(tr, btr, atol=1e-12 * np.abs(btr).max())


@pytest.mark.parametrize("ndim,so,periodic", [(2, 4, False), (2, 8, True), (3, 4, False), (3, 8, True)])
def test_tti_matches_dense_brute_force(ndim, so, periodic):
    shape = (10, 9, 8)[:ndim]
    h = (10.0, 12.0, 9.0)[:ndim]
    ash = tuple(reversed(shape))
    rng = np.random.default_rng(40 + so)
    m = 1 / rng.uniform(1500, 3000, size=ash) ** 2
    eps = rng.uniform(0, 0.3, size=ash)
    delta = np.minimum(rng.uniform(0, 0.2, size=ash), eps)
    theta = rng.uniform(0, math.pi / 4, size=ash)
    phi = rng.uniform(0, math.pi / 4, size=ash) if ndim == 3 else None
    dt = 0.4 * min(h) / (3000 * math.sqrt(1.6) * math.sqrt(ndim))
    ext = tuple(hh * (k - 1) for hh, k in zip(h, shape))
    nbl = 0 if periodic else 2
    g = oracle.Grid(shape, ext, so=so, dt=dt, nbl=nbl, vmax=3000.0, periodic=periodic)
    src_c = rng.uniform(0, 1, size=(1, ndim)) * np.array(ext)
    rec_c = rng.uniform(0, 1, size=(4, ndim)) * np.array(ext)
    nt = 15
    q = rng.standard_normal((nt, 1))
    p0 = rng.standard_normal(ash)
    r0 = rng.standard_normal(ash)
    init = (0.3 * p0, p0, -0.2 * r0, r0)
    out = oracle.tti_run(g, m, eps, delta, theta, phi if ndim == 3 else None, nt, *init, src_coords=src_c, src=q,
                         rec_coords=rec_c)
    ref = brute.tti_run(shape, h, (0.0,) * ndim, so, dt, nt, m, eps, delta, theta, phi, nbl, 3000.0, src_c, q,
                        rec_c, periodic=periodic, init=init)
    for a, b in zip(out, ref):
        np.testing.assert_allclose(a, b, atol=1e-11 * max(1.0, np.abs(b).max()))


@pytest.mark.parametrize("ndim,so,periodic", [(2, 4, False), (2, 12, True), (3, 8, False), (3, 16, True)])
def test_rotated_h_matches_dense_brute_force(ndim, so, periodic):
    """H u = sum_a n_a D_a (sum_b n_b D_b u) against the dense product G G of
    explicit first-derivative matrices, with theta and phi over a full turn
    (every sign of every component of n)."""
    shape = (11, 9, 10)[:ndim]
    h = (10.0, 12.5, 8.0)[:ndim]
    ash = tuple(reversed(shape))
    rng = np.random.default_rng(70 + so + ndim)
    theta = rng.uniform(0, 2 * math.pi, size=ash)
    phi = rng.uniform(0, 2 * math.pi, size=ash) if ndim == 3 else None
    u = rng.standard_normal(ash)
    ext = tuple(hh * (k - 1) for hh, k in zip(h, shape))
    g = oracle.Grid(shape, ext, so=so, periodic=periodic)
    out = oracle.rotated_h(g, theta, phi, u)
    R = so // 2
    D = [brute.deriv1(shape, h, R, a, periodic) for a in range(ndim)]
    th = theta.reshape(-1)
    if ndim == 3:
        ph = phi.reshape(-1)
        n = [np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]
    else:
        n = [np.sin(th), np.cos(th)]
    G = sum(np.diag(n[a]) @ D[a] for a in range(ndim))
    ref = (G @ (G @ u.reshape(-1))).reshape(ash)
    np.testing.assert_allclose(out, ref, atol=1e-12 * np.abs(ref).max())
    # a transposed operand (G^T G) or a dropped normal component would differ
    assert np.abs((G.T @ (G @ u.reshape(-1))).reshape(ash) - ref).max() > 1e-3 * np.abs(ref).max()


# ------------------------------------------------------------------- TTI
@pytest.mark.parametrize("ndim", [2, 3])
def test_tti_reduces_to_iso(ndim):
    """eps = delta = 0 and p = r: A + B = L p, so p follows the isotropic operator."""
    shape = (15, 13, 12)[:ndim]
    ext = tuple(10.0 * (k - 1) for k in shape)
    ash = tuple(reversed(shape))
    rng = np.random.default_rng(8)
    m = 1 / rng.uniform(1500, 2500, size=ash) ** 2
    theta = rng.uniform(0, math.pi / 2, size=ash)
    phi = rng.uniform(0, math.pi, size=ash)
    dt = 0.4 * 10 / (2500 * math.sqrt(ndim))
    g = oracle.Grid(shape, ext, so=8, dt=dt, nbl=3, vmax=2500.0)
    nt = 30
    src_c = np.array([[55.0, 61.0, 47.0][:ndim]])
    rec_c = np.array([[20.0, 30.0, 80.0][:ndim], [101.0, 5.0, 3.0][:ndim]])
    q = rng.standard_normal((nt, 1))
    z = np.zeros(ash)
    pp, pc, rp, rc, tr = oracle.tti_run(g, m, z, z, theta, phi if ndim == 3 else None, nt, src_coords=src_c,
                                        src=q, rec_coords=rec_c)
    up, uc, tri = oracle.iso_run(g, m, nt, src_coords=src_c, src=q, rec_coords=rec_c)
    sc = np.abs(uc).max()
    np.testing.assert_allclose(pc, uc, atol=1e-12 * sc)
    np.testing.assert_allclose(rc, uc, atol=1e-12 * sc)
    np.testing.assert_allclose(tr, tri, atol=1e-12 * np.abs(tri).max())


@pytest.mark.parametrize("ndim,so", [(2, 4), (3, 8), (3, 12)])
def test_tti_plane_wave_periodic(ndim, so):
    """Constant coefficients on a periodic grid: a cosine mode stays a mode and
    its (p, r) amplitudes follow the 2x2 leapfrog recurrence with the discrete
    symbols  L -> -lambda,  n.D -> i beta  (so H -> -beta^2):
      m a'' = K a,  K = [[(1+2e)(beta^2 - lambda), -s beta^2], [s(beta^2 - lambda), -beta^2]]."""
    shape = (16, 12, 10)[:ndim]
    h = (10.0, 8.0, 12.0)[:ndim]
    kk = (3, 2, 1)[:ndim]
    R = so // 2
    v, e, dl, th, ph = 2000.0, 0.25, 0.1, 0.6, 0.4
    s = math.sqrt(1 + 2 * dl)
    nvec = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)] if ndim == 3 else \
        [math.sin(th), math.cos(th)]
    w2 = [float(x) for x in brute.taylor_w2(R)]
    w1 = [float(x) for x in brute.taylor_w1(R)]
    lam, beta = 0.0, 0.0
    for a in range(ndim):
        kap = 2 * math.pi * kk[a] / shape[a]
        lam += -(w2[0] + 2 * sum(w2[k] * math.cos(k * kap) for k in range(1, R + 1))) / h[a] ** 2
        beta += nvec[a] * 2 * sum(w1[k] * math.sin(k * kap) for k in range(1, R + 1)) / h[a]
    K = np.array([[(1 + 2 * e) * (beta ** 2 - lam), -s * beta ** 2], [s * (beta ** 2 - lam), -beta ** 2]])
    m = 1 / v ** 2
    dt = 0.3 * min(h) / (v * math.sqrt(1.6 * ndim))
    idx = np.indices(tuple(reversed(shape)))[::-1]
    ang = sum(2 * math.pi * kk[a] * idx[a] / shape[a] for a in range(ndim))
    mode = np.cos(ang)
    a_prev = np.array([0.7, -0.2])
    a_cur = np.array([1.0, 0.5])
    ext = tuple(hh * (k - 1) for hh, k in zip(h, shape))
    g = oracle.Grid(shape, ext, so=so, dt=dt, periodic=True)
    full = lambda c: np.full(mode.shape, c)  # noqa: E731
    nt = 60
    out = oracle.tti_run(g, full(m), full(e), full(dl), full(th), full(ph) if ndim == 3 else None, nt,
                         a_prev[0] * mode, a_cur[0] * mode, a_prev[1] * mode, a_cur[1] * mode)
    ap, ac = a_prev.copy(), a_cur.copy()
    for _ in range(nt):
        an = 2 * ac - ap + dt * dt / m * (K @ ac)
        ap, ac = ac, an
    sc = np.abs(ac).max()
    np.testing.assert_allclose(out[1], ac[0] * mode, atol=1e-10 * sc)
    np.testing.assert_allclose(out[3], ac[1] * mode, atol=1e-10 * sc)
    np.testing.assert_allclose(out[0], ap[0] * mode, atol=1e-10 * sc)


# ------------------------------------------------- damping, split runs
def test_damping_profile_shape():
    """Zero in the interior, symmetric, maximal at the outer faces (the paper
    names an absorbing mask but not its profile: the quadratic one is a reading)."""
    g = oracle.Grid((30, 20), (290.0, 190.0), so=4, dt=1e-3, nbl=6, vmax=2000.0)
    eta = oracle.damping(g)
    assert eta[10, 15] == 0.0
    np.testing.assert_allclose(eta, eta[::-1, ::-1], rtol=1e-14)
    emax = 3 * 2000.0 * math.log(1000.0) / (2 * 6 * 10.0)
    assert abs(eta[10, 0] - emax) <= 1e-12 * emax
    assert eta[10, 6] == 0.0 and eta[10, 5] > 0.0


def test_split_run_equals_single_run():
    prob_shape = (17, 15)
    ext = (160.0, 140.0)
    rng = np.random.default_rng(9)
    m = 1 / rng.uniform(1500, 2000, size=(15, 17)) ** 2
    dt = 0.4 * 10 / (2000 * math.sqrt(2))
    g = oracle.Grid(prob_shape, ext, so=8, dt=dt, nbl=3, vmax=2000.0)
    nt = 30
    q = rng.standard_normal((nt, 1))
    sc, rc = [[77.0, 66.0]], [[12.0, 130.0], [150.0, 3.0]]
    up, uc, tr = oracle.iso_run(g, m, nt, src_coords=sc, src=q, rec_coords=rc)
    a_up, a_uc, tra = oracle.iso_run(g, m, nt, src_coords=sc, src=q, rec_coords=rc, time_m=0, time_M=11)
    b_up, b_uc, trb = oracle.iso_run(g, m, nt, a_up, a_uc, src_coords=sc, src=q, rec_coords=rc, time_m=12,
                                     time_M=nt - 1)
    np.testing.assert_array_equal(uc, b_uc)
    np.testing.assert_array_equal(up, b_up)
    np.testing.assert_array_equal(tr[:12], tra[:12])
    np.testing.assert_array_equal(tr[12:], trb[12:])
