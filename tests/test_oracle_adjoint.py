"""Pins of the oracle's adjoint and gradient: the adjoint dot-product test
<F q, d> = <q, F^T d> in FP64, and the gradient against central finite
differences of J(m) = <d, F(m) q> along random directions."""
import math

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _setup(ndim, so, seed, nbl=3):
    shape = (16, 13, 11)[:ndim]
    h = (10.0, 12.0, 9.0)[:ndim]
    rng = np.random.default_rng(seed)
    ash = tuple(reversed(shape))
    m = 1 / rng.uniform(1500, 2500, size=ash) ** 2
    dt = 0.4 * min(h) / (2500 * math.sqrt(ndim))
    ext = tuple(hh * (k - 1) for hh, k in zip(h, shape))
    g = oracle.Grid(shape, ext, so=so, dt=dt, nbl=nbl, vmax=2500.0)
    src = rng.uniform(0, 1, size=(2, ndim)) * np.array(ext)
    rec = rng.uniform(0, 1, size=(5, ndim)) * np.array(ext)
    rec[0] = np.array(ext) * 0.02  # inside the damping layer
    return g, m, src, rec, rng


@pytest.mark.parametrize("ndim,so", [(2, 4), (2, 8), (3, 4), (3, 8)])
def test_adjoint_dot_product(ndim, so):
    g, m, src, rec, rng = _setup(ndim, so, 60 + so)
    nt = 40
    q = rng.standard_normal((nt, src.shape[0]))
    d = rng.standard_normal((nt, rec.shape[0]))
    _, _, fq = oracle.iso_run(g, m, nt, src_coords=src, src=q, rec_coords=rec)
    ftd = oracle.iso_adjoint(g, m, nt, src, rec, d)
    lhs, rhs = float(np.sum(fq * d)), float(np.sum(q * ftd))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300), (lhs, rhs)


@pytest.mark.parametrize("ndim,so", [(2, 4), (3, 8)])
def test_gradient_matches_finite_differences(ndim, so):
    g, m, src, rec, rng = _setup(ndim, so, 70 + so)
    nt = 30
    q = rng.standard_normal((nt, src.shape[0]))
    d = rng.standard_normal((nt, rec.shape[0]))
    grad = oracle.iso_gradient(g, m, nt, src, q, rec, d)

    def J(mm):
        return float(np.sum(d * oracle.iso_run(g, mm, nt, src_coords=src, src=q, rec_coords=rec)[2]))

    for k in range(3):
        dm = rng.standard_normal(m.shape) * m * 1e-6
        fd = (J(m + dm) - J(m - dm)) / 2.0
        an = float(np.sum(grad * dm))
        assert abs(fd - an) <= 1e-6 * abs(an), (k, fd, an)


def test_gradient_is_the_adjoint_state_imaging_condition():
    """With D the damping factor, C = dt^2/m and nu = C D^-1 lam, the gradient
    equals -sum_t nu(t+1) [(u(t+1) - 2u(t) + u(t-1))/dt^2 + eta (u(t+1) - u(t-1))/(2 dt)]
    (the form the GPU path evaluates); checked on the oracle's own levels."""
    g, m, src, rec, rng = _setup(2, 4, 81)
    nt = 25
    q = rng.standard_normal((nt, src.shape[0]))
    d = rng.standard_normal((nt, rec.shape[0]))
    grad = oracle.iso_gradient(g, m, nt, src, q, rec, d)
    # forward levels
    U = [np.zeros(g.array_shape), np.zeros(g.array_shape)]
    up, uc = U
    for t in range(nt):
        up, uc, _ = oracle.iso_run(g, m, nt, up, uc, src_coords=src, src=q, time_m=t, time_M=t)
        U.append(uc)
    # adjoint levels nu via the transposed recurrence, written with numpy + the oracle's Laplacian
    eta = oracle.damping(g)
    a = eta * g.dt / 2
    C = g.dt ** 2 / m
    lam1 = np.zeros(g.array_shape)
    lam2 = np.zeros(g.array_shape)
    expect = np.zeros(g.array_shape)
    for t in range(nt, 0, -1):
        lam0 = 2 * lam1 / (1 + a) + oracle.laplacian(g, C * lam1 / (1 + a)) - (1 - a) * lam2 / (1 + a)
        lam0 = oracle.inject(g, rec, d[t - 1], lam0)
        nu = C * lam0 / (1 + a)
        un, ucur, uprev = U[t + 1], U[t], U[t - 1]
        expect += -nu * ((un - 2 * ucur + uprev) / g.dt ** 2 + eta * (un - uprev) / (2 * g.dt))
        lam2, lam1 = lam1, lam0
    np.testing.assert_allclose(grad, expect, rtol=1e-9, atol=1e-12 * np.abs(expect).max())
