"""Seeded synthetic problem generators (media, damping layers, sources).

This module only builds *inputs* of the Helmholtz problem
    -Lap U - omega^2/c^2 U + i omega R U = F          (Section 1, eq. 3)
on the unit box with Dirichlet walls: the wave speed c(x) at the nodes, the
damping R(x) at the nodes, the physical frequency omega, the grid spacing h,
the right-hand side F and the number of periods T handed to the
preconditioner.  It contains none of the method's arithmetic (no stencil, no
time step, no window), so both the CPU oracle and the GPU library consume the
same arrays without sharing any computation.

Workload recipe (the paper's own media are not available; these stand in):
  * "const2d"   64^2, h=1/65, c=1, 10 points per wavelength, 8-cell layer.
  * "smooth2d"  n^2 (1024^2 by default), Gaussian-filtered N(0,1) field,
                sigma=20 cells, mapped affinely to [1.5, 4.5]; 32-cell layer;
                point source at a seeded node away from the layer.
  * "layered3d" n^3 (256^3 by default), 8 layers along axis 0 with seeded
                interface depths and speeds in [1.5, 4.5], times (1+0.05 p)
                with p a smooth seeded field scaled to max|p| = 1; 8 ppw,
                24-cell layer, source at the centre.
  * "smooth3d"  n^3 (128^3), Gaussian sigma=8 field mapped to [1.5, 3.0].
Damping profile (the paper adds absorbing layers of a fixed width around the
model, Section 5.1): here the layer lies inside the grid, with per-axis depth
delta_a(i) = max(0, w - min(i, n_a-1-i)), delta = max_a delta_a and
R = R_max (delta/w)^2, R_max = 2 omega.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One Helmholtz problem: node arrays are row-major [n0][n1][(n2)]."""
    name: str
    n: tuple            # interior nodes per axis (axis 0 slowest)
    h: float            # grid spacing
    omega: float        # physical angular frequency
    c: np.ndarray       # wave speed at nodes, float64, shape n
    R: np.ndarray       # damping at nodes (Im H = omega * R), float64, shape n
    F: np.ndarray       # right-hand side, complex128, shape n
    periods: int        # T, periods per preconditioner application
    ppw: float          # points per minimum wavelength used to set omega
    width: int          # damping-layer width in cells
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.n)

    @property
    def N(self):
        return int(np.prod(self.n))


def omega_for_ppw(c_min: float, h: float, ppw: float) -> float:
    """Physical omega such that the shortest wavelength 2*pi*c_min/omega
    spans `ppw` grid spacings."""
    return 2.0 * math.pi * c_min / (ppw * h)


def damping_profile(n, width: int, r_max: float) -> np.ndarray:
    """Quadratic absorbing layer of `width` cells inside every wall."""
    if width <= 0:
        return np.zeros(n, dtype=np.float64)
    deltas = []
    for a, na in enumerate(n):
        i = np.arange(na)
        da = np.maximum(0, width - np.minimum(i, na - 1 - i)).astype(np.float64)
        shape = [1] * len(n)
        shape[a] = na
        deltas.append(da.reshape(shape))
    delta = deltas[0]
    for da in deltas[1:]:
        delta = np.maximum(delta, da)
    delta = np.broadcast_to(delta, n)
    return np.ascontiguousarray(r_max * (delta / width) ** 2)


def smooth_field(n, sigma: float, seed: int) -> np.ndarray:
    """N(0,1) white noise smoothed with a Gaussian of `sigma` cells."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n)
    return gaussian_filter(z, sigma=sigma, mode="reflect", truncate=4.0)


def map_range(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    xmin, xmax = float(x.min()), float(x.max())
    if xmax == xmin:
        return np.full_like(x, 0.5 * (lo + hi))
    return lo + (hi - lo) * (x - xmin) / (xmax - xmin)


def point_source(n, idx) -> np.ndarray:
    F = np.zeros(n, dtype=np.complex128)
    F[tuple(idx)] = 1.0
    return F


def periods_for(n, ppw: float) -> int:
    """T = ceil(n_max / ppw): about the size of the model in wavelengths."""
    return int(math.ceil(max(n) / ppw))


def const2d(n: int = 64, ppw: float = 10.0, width: int = 8) -> Problem:
    """Constant medium c=1 on n^2 nodes, h = 1/(n+1), source at the centre."""
    shape = (n, n)
    h = 1.0 / (n + 1)
    c = np.ones(shape)
    omega = omega_for_ppw(1.0, h, ppw)
    R = damping_profile(shape, width, 2.0 * omega)
    F = point_source(shape, (n // 2, n // 2))
    return Problem("const2d", shape, h, omega, c, R, F, periods_for(shape, ppw), ppw, width)


def smooth2d(n: int = 1024, seed: int = 0, src_seed: int = 1, sigma: float = 20.0,
             cmin: float = 1.5, cmax: float = 4.5, ppw: float = 10.0,
             width: int = 32) -> Problem:
    """Smooth random medium on n^2 nodes with a seeded point source."""
    shape = (n, n)
    h = 1.0 / (n + 1)
    c = map_range(smooth_field(shape, sigma, seed), cmin, cmax)
    omega = omega_for_ppw(float(c.min()), h, ppw)
    R = damping_profile(shape, width, 2.0 * omega)
    rng = np.random.default_rng(src_seed)
    lo, hi = width, n - 1 - width
    if hi < lo:
        lo, hi = 0, n - 1
    src = tuple(int(v) for v in rng.integers(lo, hi + 1, size=2))
    F = point_source(shape, src)
    return Problem("smooth2d", shape, h, omega, c, R, F, periods_for(shape, ppw), ppw,
                   width, {"seed": seed, "src": src})


def layered3d(n: int = 256, seed: int = 2, pert_seed: int = 3, ppw: float = 8.0,
              width: int = 24, layers: int = 8, cmin: float = 1.5, cmax: float = 4.5,
              pert: float = 0.05, sigma: float = 8.0) -> Problem:
    """Layered 3-D medium (layers stacked along axis 0) plus a 5% smooth
    perturbation; source at the centre node."""
    shape = (n, n, n)
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(seed)
    depths = np.sort(rng.integers(1, n, size=layers - 1))
    speeds = rng.uniform(cmin, cmax, size=layers)
    layer_of = np.searchsorted(depths, np.arange(n), side="right")
    c = np.broadcast_to(speeds[layer_of].reshape(n, 1, 1), shape).copy()
    p = smooth_field(shape, sigma, pert_seed)
    p /= np.abs(p).max()
    c *= 1.0 + pert * p
    omega = omega_for_ppw(float(c.min()), h, ppw)
    R = damping_profile(shape, width, 2.0 * omega)
    F = point_source(shape, (n // 2, n // 2, n // 2))
    return Problem("layered3d", shape, h, omega, c, R, F, periods_for(shape, ppw), ppw,
                   width, {"seed": seed, "depths": depths.tolist()})


def smooth3d(n: int = 128, seed: int = 7, sigma: float = 8.0, cmin: float = 1.5,
             cmax: float = 3.0, ppw: float = 8.0, width: int = 16) -> Problem:
    """Smooth random 3-D medium, source at the centre (sources for the
    inversion workload come from `sources_on_plane`)."""
    shape = (n, n, n)
    h = 1.0 / (n + 1)
    c = map_range(smooth_field(shape, sigma, seed), cmin, cmax)
    omega = omega_for_ppw(float(c.min()), h, ppw)
    R = damping_profile(shape, width, 2.0 * omega)
    F = point_source(shape, (n // 2, n // 2, n // 2))
    return Problem("smooth3d", shape, h, omega, c, R, F, periods_for(shape, ppw), ppw,
                   width, {"seed": seed})


def random_sources(n, count: int, seed: int, margin: int) -> np.ndarray:
    """`count` unit point sources at seeded nodes, as a [count, *n] stack."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count,) + tuple(n), dtype=np.complex128)
    for s in range(count):
        idx = tuple(int(rng.integers(margin, na - margin)) if na > 2 * margin
                    else int(rng.integers(0, na)) for na in n)
        out[(s,) + idx] = 1.0
    return out


def sources_on_plane(n, count: int, seed: int, plane: int) -> np.ndarray:
    """Unit point sources at seeded nodes on the plane axis0 == plane."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count,) + tuple(n), dtype=np.complex128)
    for s in range(count):
        rest = tuple(int(rng.integers(na // 4, na - na // 4)) for na in n[1:])
        out[(s, plane) + rest] = 1.0
    return out


def receiver_mask(n, plane: int, per_side: int) -> np.ndarray:
    """Regular per_side x per_side array of receivers on plane axis0 == plane
    (boolean mask over the nodes)."""
    mask = np.zeros(n, dtype=bool)
    grids = [np.linspace(na // 8, na - 1 - na // 8, per_side).round().astype(int)
             for na in n[1:]]
    idx = np.meshgrid(*grids, indexing="ij")
    mask[(np.full(idx[0].shape, plane),) + tuple(idx)] = True
    return mask


def gaussian_blob(n, seed: int, radius_frac: float = 0.15) -> np.ndarray:
    """Smooth bump of unit height at a seeded centre (used to perturb m)."""
    rng = np.random.default_rng(seed)
    ctr = [rng.uniform(0.35, 0.65) * na for na in n]
    r = radius_frac * max(n)
    grids = np.meshgrid(*[np.arange(na, dtype=np.float64) for na in n], indexing="ij")
    d2 = sum((g - c0) ** 2 for g, c0 in zip(grids, ctr))
    return np.exp(-d2 / (2 * r * r))


def uneven_problems(count: int = 32, seed: int = 6, lo: int = 128, hi: int = 768,
                    ppw: float = 10.0, width: int = 32):
    """`count` independent 2-D problems of uneven sizes, each with its own
    seeded medium (seed 100+i) and a centre source."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=(count, 2))
    out = []
    for i in range(count):
        shape = (int(sizes[i, 0]), int(sizes[i, 1]))
        h = 1.0 / (max(shape) + 1)
        c = map_range(smooth_field(shape, 20.0, 100 + i), 1.5, 4.5)
        omega = omega_for_ppw(float(c.min()), h, ppw)
        w = min(width, min(shape) // 4)
        R = damping_profile(shape, w, 2.0 * omega)
        F = point_source(shape, (shape[0] // 2, shape[1] // 2))
        out.append(Problem(f"uneven{i}", shape, h, omega, c, R, F,
                           periods_for(shape, ppw), ppw, w, {"seed": 100 + i}))
    return out


def random_medium(n, seed: int, cmin: float = 1.0, cmax: float = 2.0,
                  sigma: float = 2.0, ppw: float = 8.0, width: int = 2,
                  r_scale: float = 2.0) -> Problem:
    """Small smooth random problem for parity tests at tiny sizes."""
    shape = tuple(n)
    h = 1.0 / (max(shape) + 1)
    c = map_range(smooth_field(shape, sigma, seed), cmin, cmax)
    omega = omega_for_ppw(float(c.min()), h, ppw)
    R = damping_profile(shape, width, r_scale * omega)
    rng = np.random.default_rng(seed + 1000)
    F = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return Problem("random", shape, h, omega, c, R, F, periods_for(shape, ppw), ppw, width,
                   {"seed": seed})


def _model2d(name, model: int, width: int, ppw: float, c_of_xy, src_xy) -> Problem:
    """A model on the unit square, `model` nodes per axis at the cell centres
    (k + 1/2) h, h = 1/model, so that k = omega/c = 2 pi model/ppw for c = 1
    (Sec. 5.1 prints k = 335.1 for its 320 x 320 constant model at 6 points
    per wavelength); damping layers of `width` nodes are added outside it (as
    in Sec. 5.1), so the grid has model + 2 width nodes per axis.  c_of_xy(x, y)
    gives the speed at model coordinates (nodes in the layers take the speed of
    the nearest model node); the point source sits at the model node nearest
    to src_xy."""
    n = model + 2 * width
    shape = (n, n)
    h = 1.0 / model
    idx = np.clip(np.arange(n) - width, 0, model - 1)
    xs = (idx + 0.5) * h
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    c = np.ascontiguousarray(c_of_xy(X, Y), dtype=np.float64)
    omega = omega_for_ppw(float(c.min()), h, ppw)
    R = damping_profile(shape, width, 2.0 * omega)
    src = tuple(width + min(model - 1, max(0, int(math.floor(v / h)))) for v in src_xy)
    F = point_source(shape, src)
    return Problem(name, shape, h, omega, c, R, F, periods_for((model, model), ppw), ppw,
                   width, {"model": model, "src": src})


def open2d(model: int = 320, width: int = 32, ppw: float = 6.0) -> Problem:
    """Constant speed c = 1 on the unit square (the constant model of Sec. 5.1),
    point source at (0.5, 0.25)."""
    return _model2d("open2d", model, width, ppw, lambda X, Y: np.ones_like(X), (0.5, 0.25))


def disc2d(model: int = 320, width: int = 32, ppw: float = 6.0, c_out: float = 1.0,
           c_in: float = 0.5, radius: float = 0.2) -> Problem:
    """Piecewise constant model with a slow disc (speed c_in inside radius
    `radius` around (0.5, 0.5), c_out outside): waves are trapped in the disc, a
    resonant stand-in for Sec. 5.1's circular model.  Source at (0.5, 0.2),
    outside the disc."""
    def c_of(X, Y):
        inside = (X - 0.5) ** 2 + (Y - 0.5) ** 2 < radius ** 2
        return np.where(inside, c_in, c_out)
    return _model2d("disc2d", model, width, ppw, c_of, (0.5, 0.2))
