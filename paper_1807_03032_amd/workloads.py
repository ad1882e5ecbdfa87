"""Seeded synthetic inputs for the wave-equation operators.

This module only draws and shapes INPUTS: velocity / anisotropy models,
source and receiver coordinates, and source wavelets.  It contains none of the
operators' arithmetic (no stencils, no interpolation weights, no damping), so
that the CPU oracle and the HIP path can both consume the same inputs.

Every floating-point model value and wavelet sample is rounded to float32 and
returned as float64, so both sides see bit-identical parameters; coordinates
stay float64 (both sides derive their interpolation data from them in FP64).

Arrays use the logical layout with the first axis fastest: numpy shape
(nz, ny, nx) for a 3D grid whose axes are (x, y, z), (nz, nx) for 2D (x, z).

Workload recipes follow the paper's test-case setup (arXiv 1807.03032,
Section 7.2: cubic grids, space orders 4-16, zero initial conditions,
damping layer, one seismic source wavelet, CFL-chosen time step).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

SPACE_ORDERS = (2, 4, 6, 8, 10, 12, 14, 16)


def f32(a):
    """Round to float32 and hand back float64 (identical values on both sides)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def ricker(f0: float, t0: float, dt: float, nt: int, amp: float = 1.0) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = n dt - t0.

    The paper only says 'a time-dependent seismic source wavelet' (Section 7.2);
    the Ricker wavelet is the customary choice.
    """
    tau = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * tau) ** 2
    return f32(amp * (1.0 - 2.0 * a) * np.exp(-a))


def cfl_dt(h_min: float, v_eff: float, ndim: int, factor: float = 0.4) -> float:
    """dt = factor * h_min / (v_eff sqrt(ndim)) (the configs' 'dt = 0.4 CFL')."""
    return factor * h_min / (v_eff * math.sqrt(ndim))


def smooth_field(shape_xyz, seed: int, lo: float, hi: float, sigma_pts: float = 10.0) -> np.ndarray:
    """Smooth seeded random field rescaled to [lo, hi].

    Recipe: white noise N(0,1) drawn with numpy PCG64(seed) on a coarse grid
    (one node every `step` points, step = max(1, round(sigma_pts/2))), a
    separable Gaussian filter of sigma = sigma_pts/step coarse nodes (truncated
    at 3 sigma, reflecting edges), min-max rescale to [lo, hi], then
    multilinear interpolation onto the full grid (values stay in [lo, hi]).
    """
    from scipy import ndimage

    shape = tuple(reversed([int(s) for s in shape_xyz]))  # numpy order
    step = max(1, int(round(sigma_pts / 2.0)))
    coarse = tuple(max(2, (s - 1 + step - 1) // step + 1) for s in shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(coarse)
    w = ndimage.gaussian_filter(w, sigma=sigma_pts / step, truncate=3.0, mode="reflect")
    wmin, wmax = float(w.min()), float(w.max())
    w = (w - wmin) / (wmax - wmin) if wmax > wmin else np.zeros_like(w)
    w = lo + (hi - lo) * w
    # multilinear upsampling, one axis at a time, fastest (smallest result) first
    out = w
    for ax in reversed(range(len(shape))):
        n = shape[ax]
        pos = np.arange(n, dtype=np.float64) / step
        pos = np.minimum(pos, out.shape[ax] - 1)
        i0 = np.minimum(np.floor(pos).astype(np.int64), out.shape[ax] - 2)
        fr = pos - i0
        a0 = np.take(out, i0, axis=ax)
        a1 = np.take(out, i0 + 1, axis=ax)
        bshape = [1] * out.ndim
        bshape[ax] = n
        fr = fr.reshape(bshape)
        out = a0 * (1.0 - fr) + a1 * fr
    return np.clip(out, lo, hi)


@dataclasses.dataclass
class Problem:
    """One forward-modelling shot: grid, model, sources, receivers, time axis."""

    name: str
    kind: str                      # "iso" or "tti"
    shape: tuple                   # (nx, nz) or (nx, ny, nz)
    extent: tuple
    origin: tuple
    so: int
    nbl: int
    nt: int
    dt: float
    vmax: float
    eps_max: float
    fields: Dict[str, np.ndarray]  # m (and eps, delta, theta, phi for tti), numpy order
    src_coords: np.ndarray         # [nsrc][ndim]
    src: np.ndarray                # [nt][nsrc]
    rec_coords: np.ndarray         # [nrec][ndim]
    rc: float = 1e-3               # damping reflection coefficient
    # precomputed sparse supports (gridpoints [n][ndim], coeffs [n][ndim][r]);
    # when set they replace the linear weights of src_coords / rec_coords
    src_pre: Optional[tuple] = None
    rec_pre: Optional[tuple] = None

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def spacing(self):
        return tuple(e / (n - 1) for e, n in zip(self.extent, self.shape))

    @property
    def npoints(self):
        return int(np.prod(self.shape))

    @property
    def array_shape(self):
        return tuple(reversed(self.shape))


def _physical_models(kind, shape, v, seed0, eps_range=(0.0, 0.3), delta_range=(0.0, 0.2),
                     angle_range=(0.0, math.pi / 4), sigma_pts=10.0):
    """m = 1/v^2 plus, for TTI, eps, delta (clamped to delta <= eps), theta, phi."""
    fields = {"m": f32(1.0 / (v * v))}
    eps_max = 0.0
    if kind == "tti":
        eps = f32(smooth_field(shape, seed0 + 1, *eps_range, sigma_pts=sigma_pts))
        delta = smooth_field(shape, seed0 + 2, *delta_range, sigma_pts=sigma_pts)
        # model-generation rule: delta <= eps keeps the coupled system well posed
        delta = f32(np.minimum(delta, eps))
        theta = f32(smooth_field(shape, seed0 + 3, *angle_range, sigma_pts=sigma_pts))
        fields.update(eps=eps, delta=delta, theta=theta)
        if len(shape) == 3:
            fields["phi"] = f32(smooth_field(shape, seed0 + 4, *angle_range, sigma_pts=sigma_pts))
        eps_max = float(eps.max())
    return fields, eps_max


def _receiver_plane(n_x, n_y, h, x_extent, y_extent, z0, seeds):
    """n_x*n_y receivers at jittered lattice positions, x fastest in the ordering."""
    gx = np.random.default_rng(seeds[0]).uniform(-0.5, 0.5, size=(n_y, n_x))
    gy = np.random.default_rng(seeds[1]).uniform(-0.5, 0.5, size=(n_y, n_x))
    gz = np.random.default_rng(seeds[2]).uniform(0.0, 1.0, size=(n_y, n_x))
    ix = np.arange(n_x)[None, :]
    iy = np.arange(n_y)[:, None]
    x = np.clip((ix + gx) * h, 0.0, x_extent)
    y = np.clip((iy + gy) * h, 0.0, y_extent)
    z = z0 + gz * h
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def config_2d_iso_101(nt: Optional[int] = None) -> Problem:
    """2D isotropic, 101x101, h = 10 m, v = 1500 m/s, so = 4, 500 steps, nbl = 20,
    10 Hz Ricker at the centre node, 101 receivers on a row 20 m below the layer."""
    shape, h, v, nbl = (101, 101), 10.0, 1500.0, 20
    nt = 500 if nt is None else nt
    extent = tuple(h * (n - 1) for n in shape)
    dt = cfl_dt(h, v, 2)
    vel = np.full(tuple(reversed(shape)), v)
    fields, _ = _physical_models("iso", shape, vel, 0)
    src_coords = np.array([[500.0, 500.0]])
    src = ricker(10.0, 0.1, dt, nt)[:, None]
    rec_coords = np.stack([np.arange(101) * 10.0, np.full(101, (nbl + 2) * h)], axis=1)
    return Problem("2d_iso_101x101_so4", "iso", shape, extent, (0.0, 0.0), 4, nbl, nt, dt, v, 0.0,
                   fields, src_coords, f32(src), rec_coords)


def config_3d_iso_256(nt: Optional[int] = None, n: int = 256) -> Problem:
    """3D isotropic, 256^3, h = 10 m, v = 1500 / 2500 m/s split at mid-depth,
    so = 8, nbl = 40, 1000 steps, 15 Hz Ricker near the surface,
    256x256 jittered receiver plane (trilinear interpolation)."""
    shape, h, nbl = (n, n, n), 10.0, 40
    nt = 1000 if nt is None else nt
    extent = tuple(h * (k - 1) for k in shape)
    vel = np.full(tuple(reversed(shape)), 1500.0)
    vel[n // 2:, :, :] = 2500.0  # numpy axis 0 is z (depth)
    dt = cfl_dt(h, 2500.0, 3)
    fields, _ = _physical_models("iso", shape, vel, 0)
    src_coords = np.array([[extent[0] / 2, extent[1] / 2, (nbl + 2.5) * h]])
    src = ricker(15.0, 1.0 / 15.0, dt, nt)[:, None]
    rec_coords = _receiver_plane(n, n, h, extent[0], extent[1], (nbl + 2) * h, (2, 3, 4))
    return Problem(f"3d_iso_{n}cube_so8", "iso", shape, extent, (0.0,) * 3, 8, nbl, nt, dt, 2500.0, 0.0,
                   fields, src_coords, f32(src), rec_coords)


def config_3d_tti_512(nt: Optional[int] = None, n: int = 512) -> Problem:
    """3D TTI, 512^3, h = 12.5 m, so = 12, nbl = 40, 800 steps; smooth seeded random
    v in [1500, 4500], eps in [0, 0.3], delta in [0, 0.2] (<= eps), theta, phi in
    [0, pi/4]; 10 Hz Ricker at the centre near the surface; 512x512 receivers."""
    shape, h, nbl = (n, n, n), 12.5, 40
    nt = 800 if nt is None else nt
    extent = tuple(h * (k - 1) for k in shape)
    v = smooth_field(shape, 11, 1500.0, 4500.0)
    fields, eps_max = _physical_models("tti", shape, v, 11)
    vmax = 4500.0
    dt = cfl_dt(h, vmax * math.sqrt(1.0 + 2.0 * 0.3), 3)
    src_coords = np.array([[extent[0] / 2, extent[1] / 2, (nbl + 2.5) * h]])
    src = ricker(10.0, 0.1, dt, nt)[:, None]
    rec_coords = _receiver_plane(n, n, h, extent[0], extent[1], (nbl + 2) * h, (16, 17, 18))
    return Problem(f"3d_tti_{n}cube_so12", "tti", shape, extent, (0.0,) * 3, 12, nbl, nt, dt, vmax, eps_max,
                   fields, src_coords, f32(src), rec_coords)


def small_problem(kind: str, shape, so: int, nt: int, seed: int = 0, nsrc: int = 1, nrec: int = 16,
                  nbl: int = 4, h: float = 10.0, vrange=(1500.0, 3000.0), src_at=None,
                  rec_coords=None, f0: Optional[float] = None, sigma_pts: float = 4.0,
                  angle_range=(0.0, math.pi / 4)) -> Problem:
    """A small seeded problem of any shape for parity tests: smooth random models,
    sources and receivers at random positions anywhere in the grid (edges
    included), a Ricker wavelet per source with jittered delay."""
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    extent = tuple(h * (k - 1) for k in shape)
    v = smooth_field(shape, seed + 100, vrange[0], vrange[1], sigma_pts=sigma_pts)
    fields, eps_max = _physical_models(kind, shape, v, seed + 100, sigma_pts=sigma_pts, angle_range=angle_range)
    vmax = float(vrange[1])
    v_eff = vmax * math.sqrt(1.0 + 2.0 * 0.3) if kind == "tti" else vmax
    dt = cfl_dt(h, v_eff, ndim)
    rng = np.random.default_rng(seed + 200)
    if src_at is not None:
        src_coords = np.asarray(src_at, dtype=np.float64).reshape(-1, ndim)
    else:
        src_coords = rng.uniform(0.0, 1.0, size=(nsrc, ndim)) * np.asarray(extent)
    ns = src_coords.shape[0]
    if f0 is None:
        f0 = vrange[0] / (8.0 * h)  # about 8 points per wavelength at the peak frequency
    src = (np.stack([ricker(f0, (1.0 + 0.2 * k) / f0, dt, nt) for k in range(ns)], axis=1) if ns
           else np.zeros((nt, 0)))
    if rec_coords is None:
        rec_coords = rng.uniform(0.0, 1.0, size=(nrec, ndim)) * np.asarray(extent)
    return Problem(f"small_{kind}_{'x'.join(map(str, shape))}_so{so}", kind, shape, extent, (0.0,) * ndim,
                   so, nbl, nt, dt, vmax, eps_max, fields, src_coords, f32(src).reshape(nt, ns),
                   np.asarray(rec_coords, dtype=np.float64).reshape(-1, ndim))


def config_3d_iso_adjoint_320(nt: Optional[int] = None, n: int = 320):
    """Adjoint / gradient workload: 3D isotropic, n^3 (320^3), h = 10 m, so = 8,
    nbl = 40, 1500 steps; smooth random background velocity in [1500, 3500] m/s
    (seed 21, sigma = 10 points) and a true model with a 5 % smooth seeded
    perturbation (seed 22); 10 Hz Ricker at the centre near the surface;
    320 x 320 jittered receiver plane (seeds 23-25).

    Returns (background problem, true squared slowness)."""
    shape, h, nbl = (n, n, n), 10.0, 40
    nt = 1500 if nt is None else nt
    extent = tuple(h * (k - 1) for k in shape)
    v_bg = smooth_field(shape, 21, 1500.0, 3500.0)
    pert = smooth_field(shape, 22, -1.0, 1.0)
    v_true = v_bg * (1.0 + 0.05 * pert)
    vmax = 3500.0 * 1.05
    fields, _ = _physical_models("iso", shape, v_bg, 0)
    m_true = f32(1.0 / (v_true * v_true))
    dt = cfl_dt(h, vmax, 3)
    src_coords = np.array([[extent[0] / 2, extent[1] / 2, (nbl + 2.5) * h]])
    src = ricker(10.0, 0.1, dt, nt)[:, None]
    rec_coords = _receiver_plane(n, n, h, extent[0], extent[1], (nbl + 2) * h, (23, 24, 25))
    prob = Problem(f"3d_iso_adjoint_{n}cube_so8", "iso", shape, extent, (0.0,) * 3, 8, nbl, nt, dt, vmax, 0.0,
                   fields, src_coords, f32(src), rec_coords)
    return prob, m_true


def lagrange_support(shape, spacing, origin, coords, r: int):
    """Inputs of a precomputed sparse function with an r-point Lagrange scheme
    per axis: for each point and axis, the first index of r consecutive grid
    nodes around the point (shifted to stay inside the grid) and the r Lagrange
    basis polynomials of those nodes evaluated at the point."""
    c = np.asarray(coords, dtype=np.float64).reshape(-1, len(shape))
    gp = np.zeros(c.shape, dtype=np.int64)
    cf = np.zeros(c.shape + (r,))
    for p in range(c.shape[0]):
        for a in range(len(shape)):
            xi = (c[p, a] - origin[a]) / spacing[a]
            b = min(max(int(np.floor(xi)) - (r - 1) // 2, 0), shape[a] - r)
            gp[p, a] = b
            for j in range(r):
                num, den = 1.0, 1.0
                for k in range(r):
                    if k != j:
                        num *= xi - (b + k)
                        den *= j - k
                cf[p, a, j] = num / den
    return gp, cf


# ---------------------------------------------------------------------------
# Served shot stream: Poisson arrivals of forward-modelling requests with
# grids from 2D 201^2 to 3D 400^3, space order in {4, 8, 12, 16}, 500-2000
# steps, isotropic or TTI, seeded smooth random models, a random source near
# the surface and a receiver line.
# ---------------------------------------------------------------------------
SERVE_SIZES = ((2, 201), (2, 401), (2, 801), (3, 100), (3, 200), (3, 300), (3, 400))


def serve_problem(kind: str, ndim: int, n: int, so: int, nt: int, seed: int, model_cache=None, h: float = 10.0,
                  nbl: int = 20, vrange=(1500.0, 4500.0)) -> Problem:
    """One request of the served stream: n^ndim grid, smooth random model
    (seeded by kind, ndim and n, shared through `model_cache`), 10 Hz Ricker
    source at a seeded random (x, y) position two points below the top damping
    layer, receivers every grid point along x on a line at that depth."""
    shape = (n,) * ndim
    extent = tuple(h * (k - 1) for k in shape)
    key = (kind, ndim, n)
    if model_cache is not None and key in model_cache:
        fields, eps_max = model_cache[key]
    else:
        mseed = 1000 + 10 * ndim + n + (5000 if kind == "tti" else 0)
        v = smooth_field(shape, mseed, vrange[0], vrange[1], sigma_pts=10.0)
        fields, eps_max = _physical_models(kind, shape, v, mseed)
        if model_cache is not None:
            model_cache[key] = (fields, eps_max)
    vmax = float(vrange[1])
    v_eff = vmax * math.sqrt(1.0 + 2.0 * 0.3) if kind == "tti" else vmax
    dt = cfl_dt(h, v_eff, ndim)
    rng = np.random.default_rng(seed)
    depth = (nbl + 2) * h
    pos = rng.uniform(0.25, 0.75, size=ndim - 1) * np.asarray(extent[:ndim - 1])
    src_coords = np.array([[*pos, depth]])
    src = ricker(10.0, 0.1, dt, nt)[:, None]
    xs = np.arange(n) * h
    if ndim == 3:
        rec_coords = np.stack([xs, np.full(n, pos[1]), np.full(n, depth)], axis=1)
    else:
        rec_coords = np.stack([xs, np.full(n, depth)], axis=1)
    return Problem(f"serve_{kind}_{ndim}d_{n}_so{so}_nt{nt}_s{seed}", kind, shape, extent, (0.0,) * ndim, so, nbl, nt,
                   dt, vmax, eps_max, fields, src_coords, f32(src), rec_coords)


def serve_stream(count: int = 24, seed: int = 7, rate_hz: float = 3.0, sizes=SERVE_SIZES, sos=(4, 8, 12, 16),
                 nt_range=(500, 2000), kinds=("iso", "tti"), model_cache=None):
    """[(arrival time in s, Problem)] with exponential inter-arrival times of
    mean 1/rate_hz (all seeded)."""
    rng = np.random.default_rng(seed)
    cache = {} if model_cache is None else model_cache
    out, t = [], 0.0
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        ndim, n = sizes[int(rng.integers(len(sizes)))]
        so = int(sos[int(rng.integers(len(sos)))])
        nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
        kind = kinds[int(rng.integers(len(kinds)))]
        out.append((t, serve_problem(kind, ndim, n, so, nt, seed * 1000 + i, cache)))
    return out
