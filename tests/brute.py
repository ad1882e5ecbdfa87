"""Dense brute-force reference for tiny grids, written independently of the
oracle: operators are assembled as explicit matrices from the closed-form
Taylor weights (exact rationals), and stepped with numpy matrix products.

Used only to pin the oracle (arXiv 1807.03032, Section 3: eq. WE, Listings
fd-1..fd-3, eq. interp, Listing finject; Section 7.2 test-case setup).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def taylor_w2(R: int):
    """W2_k = 2(-1)^(k+1)(R!)^2 / (k^2 (R-k)!(R+k)!), W2_0 = -2 sum W2_k (exact)."""
    w = [Fraction(0)] * (R + 1)
    for k in range(1, R + 1):
        w[k] = Fraction(2 * (-1) ** (k + 1) * math.factorial(R) ** 2,
                        k * k * math.factorial(R - k) * math.factorial(R + k))
    w[0] = -2 * sum(w[1:])
    return w


def taylor_w1(R: int):
    """W1_k = (-1)^(k+1)(R!)^2 / (k (R-k)!(R+k)!) (exact), W1_0 = 0."""
    w = [Fraction(0)] * (R + 1)
    for k in range(1, R + 1):
        w[k] = Fraction((-1) ** (k + 1) * math.factorial(R) ** 2,
                        k * math.factorial(R - k) * math.factorial(R + k))
    return w


def d2_matrix(n: int, R: int, h: float, periodic=False) -> np.ndarray:
    w = [float(x) for x in taylor_w2(R)]
    M = np.zeros((n, n))
    for i in range(n):
        M[i, i] += w[0]
        for k in range(1, R + 1):
            for j in (i + k, i - k):
                if periodic:
                    M[i, j % n] += w[k]
                elif 0 <= j < n:
                    M[i, j] += w[k]
    return M / (h * h)


def d1_matrix(n: int, R: int, h: float, periodic=False) -> np.ndarray:
    w = [float(x) for x in taylor_w1(R)]
    M = np.zeros((n, n))
    for i in range(n):
        for k in range(1, R + 1):
            for j, sg in ((i + k, 1.0), (i - k, -1.0)):
                if periodic:
                    M[i, j % n] += sg * w[k]
                elif 0 <= j < n:
                    M[i, j] += sg * w[k]
    return M / h


def axis_op(shape, a: int, M1: np.ndarray) -> np.ndarray:
    """Lift a 1-D operator on axis a to the flattened grid (first axis fastest)."""
    mats = []
    for b in reversed(range(len(shape))):  # slowest axis first in the Kronecker product
        mats.append(M1 if b == a else np.eye(shape[b]))
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def laplacian(shape, h, R, periodic=False) -> np.ndarray:
    return sum(axis_op(shape, a, d2_matrix(shape[a], R, h[a], periodic)) for a in range(len(shape)))


def deriv1(shape, h, R, a, periodic=False) -> np.ndarray:
    return axis_op(shape, a, d1_matrix(shape[a], R, h[a], periodic))


def damping_profile(shape, h, nbl, vmax, rc=1e-3) -> np.ndarray:
    """The build's damping reading: sum over axes of eta_max (d/nbl)^2 inside the layer."""
    eta = np.zeros(int(np.prod(shape)))
    if nbl <= 0:
        return eta
    idx = np.indices(tuple(reversed(shape))).reshape(len(shape), -1)[::-1]  # idx[a] = index on axis a
    for a, n in enumerate(shape):
        i = idx[a]
        d = np.maximum(np.maximum(nbl - i, i - (n - 1 - nbl)), 0)
        emax = 3.0 * vmax * math.log(1.0 / rc) / (2.0 * nbl * h[a])
        eta += emax * (d / nbl) ** 2
    return eta


def interp_matrix(shape, h, origin, coords) -> np.ndarray:
    """Row p: (multi)linear weights of point p on its 2^d cell corners."""
    coords = np.asarray(coords, dtype=np.float64).reshape(-1, len(shape))
    N = int(np.prod(shape))
    P = np.zeros((coords.shape[0], N))
    strides = [int(np.prod(shape[:a])) for a in range(len(shape))]
    for p, c in enumerate(coords):
        base, frac = [], []
        for a in range(len(shape)):
            xi = (c[a] - origin[a]) / h[a]
            b = min(int(math.floor(xi)), shape[a] - 2)
            base.append(b)
            frac.append(xi - b)
        for corner in range(1 << len(shape)):
            w = 1.0
            lin = 0
            for a in range(len(shape)):
                bit = (corner >> a) & 1
                w *= frac[a] if bit else 1.0 - frac[a]
                lin += (base[a] + bit) * strides[a]
            P[p, lin] += w
    return P


def iso_run(shape, h, origin, so, dt, nt, m, nbl=0, vmax=0.0, src_coords=None, src=None, rec_coords=None,
            u_prev=None, u_cur=None, periodic=False):
    """Dense leapfrog: u+ = (2u - (1-a)u- + dt^2/m L u)/(1+a), a = eta dt/2; then
    u+ += dt^2 P_s^T q / m; rec = P_r u+."""
    N = int(np.prod(shape))
    L = laplacian(shape, h, so // 2, periodic)
    mv = np.asarray(m, dtype=np.float64).reshape(-1)
    a = damping_profile(shape, h, nbl, vmax) * dt / 2.0
    up = np.zeros(N) if u_prev is None else np.asarray(u_prev, dtype=np.float64).reshape(-1).copy()
    uc = np.zeros(N) if u_cur is None else np.asarray(u_cur, dtype=np.float64).reshape(-1).copy()
    Ps = interp_matrix(shape, h, origin, src_coords) if src_coords is not None else None
    Pr = interp_matrix(shape, h, origin, rec_coords) if rec_coords is not None else None
    rec = np.zeros((nt, Pr.shape[0])) if Pr is not None else None
    for t in range(nt):
        un = (2.0 * uc - (1.0 - a) * up + dt * dt / mv * (L @ uc)) / (1.0 + a)
        if Ps is not None:
            un = un + dt * dt * (Ps.T @ np.asarray(src[t], dtype=np.float64)) / mv
        if Pr is not None:
            rec[t] = Pr @ un
        up, uc = uc, un
    shp = tuple(reversed(shape))
    return up.reshape(shp), uc.reshape(shp), rec


def tti_run(shape, h, origin, so, dt, nt, m, eps, delta, theta, phi=None, nbl=0, vmax=0.0, src_coords=None,
            src=None, rec_coords=None, periodic=False, init=None):
    """Dense TTI: g = sum_a diag(n_a) D_a u, H = sum_a diag(n_a) D_a g (D_a zero outside
    the domain unless periodic), A = L p - H p, B = H r, coupled leapfrog updates."""
    N = int(np.prod(shape))
    R = so // 2
    nd = len(shape)
    L = laplacian(shape, h, R, periodic)
    D = [deriv1(shape, h, R, a, periodic) for a in range(nd)]
    th = np.asarray(theta, dtype=np.float64).reshape(-1)
    if nd == 3:
        ph = np.asarray(phi, dtype=np.float64).reshape(-1)
        n = [np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]
    else:
        n = [np.sin(th), np.cos(th)]
    G = sum(np.diag(n[a]) @ D[a] for a in range(nd))
    H = G @ G
    mv = np.asarray(m, dtype=np.float64).reshape(-1)
    ev = np.asarray(eps, dtype=np.float64).reshape(-1)
    s = np.sqrt(1.0 + 2.0 * np.asarray(delta, dtype=np.float64).reshape(-1))
    a = damping_profile(shape, h, nbl, vmax) * dt / 2.0
    z = np.zeros(N)
    if init is None:
        pp, pc, rp, rc = z.copy(), z.copy(), z.copy(), z.copy()
    else:
        pp, pc, rp, rc = (np.asarray(v, dtype=np.float64).reshape(-1).copy() for v in init)
    Ps = interp_matrix(shape, h, origin, src_coords) if src_coords is not None else None
    Pr = interp_matrix(shape, h, origin, rec_coords) if rec_coords is not None else None
    rec = np.zeros((nt, Pr.shape[0])) if Pr is not None else None
    for t in range(nt):
        A = L @ pc - H @ pc
        B = H @ rc
        c = dt * dt / mv
        pn = (2.0 * pc - (1.0 - a) * pp + c * ((1.0 + 2.0 * ev) * A + s * B)) / (1.0 + a)
        rn = (2.0 * rc - (1.0 - a) * rp + c * (s * A + B)) / (1.0 + a)
        if Ps is not None:
            inj = dt * dt * (Ps.T @ np.asarray(src[t], dtype=np.float64)) / mv
            pn, rn = pn + inj, rn + inj
        if Pr is not None:
            rec[t] = Pr @ pn
        pp, pc, rp, rc = pc, pn, rc, rn
    shp = tuple(reversed(shape))
    return pp.reshape(shp), pc.reshape(shp), rp.reshape(shp), rc.reshape(shp), rec
