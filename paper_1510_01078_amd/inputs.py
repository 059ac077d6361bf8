"""Seeded synthetic inputs for planar photoacoustic reconstruction.

This module is shared by the GPU path's callers (tests, benchmark) and by the
CPU oracle's tests. It holds none of the reconstruction method's arithmetic:
only sensor layouts on the detection plane, detector-area weights, the
closed-form pressure traces of uniform balls, phantoms and noise.

Conventions (the paper's statement of the problem, Section 2):
  * sensors x_m = (x_m, y_m) lie in the open plane square (-X/2, X/2)^2, in metres;
  * h_m is the detector area assigned to sensor m, with sum_m h_m = X*Y
    (Section 2, eq. disc_rec and the constraint stated beneath it);
  * traces g[m, n] are pressure samples at t_n = n*dt, n = 0..Nt-1;
  * the sensor plane is z = 0 and sources sit at depth z > 0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

C_SOUND = 1500.0  # m/s, soft tissue / water


# ----------------------------------------------------------------------------
# Sensor layouts
# ----------------------------------------------------------------------------

def warp_1d(ns: int, half_side: float, exponent: float = 1.5) -> np.ndarray:
    """Power-law warped 1-D sensor coordinates, denser at the centre.

    u_i = -1 + (2i+1)/ns are equispaced cell midpoints of [-1, 1]; the sensor
    sits at L*sign(u)*|u|**exponent. Strictly increasing and odd-symmetric.
    """
    u = -1.0 + (2.0 * np.arange(ns) + 1.0) / ns
    return half_side * np.sign(u) * np.abs(u) ** exponent


def cell_widths_1d(x: np.ndarray, side: float) -> np.ndarray:
    """Widths of the cells bounded by midpoints between neighbouring sensors;
    the outer cells extend to the plane edges, so the widths sum to `side`."""
    mid = 0.5 * (x[1:] + x[:-1])
    edges = np.concatenate([[-0.5 * side], mid, [0.5 * side]])
    return np.diff(edges)


def clamp_to_plane(xy: np.ndarray, side_x: float, side_y: float) -> np.ndarray:
    """Clamp coordinates into the half-open square [-X/2, X/2) x [-Y/2, Y/2)."""
    out = np.array(xy, dtype=np.float64, copy=True)
    for d, side in ((0, side_x), (1, side_y)):
        lo = -0.5 * side
        hi = np.nextafter(0.5 * side, -np.inf)
        out[:, d] = np.clip(out[:, d], lo, hi)
    return out


def warped_sensors(ns: int, side: float, exponent: float = 1.5, jitter: float = 0.0,
                   rng: np.random.Generator | None = None):
    """Tensor-product warped layout of ns x ns sensors on a square plane.

    Returns (xy [M,2] float64, h [M] float64) with M = ns*ns and sensor index
    m = ix*ns + iy. h is the tensor product of the 1-D midpoint cell widths,
    so sum(h) = side**2 (up to rounding). With jitter > 0 each coordinate is
    moved by U(-jitter, jitter) times its own 1-D cell width (seeded) and
    clamped into the plane; the weights keep their un-jittered cell areas.
    """
    x1 = warp_1d(ns, 0.5 * side, exponent)
    w1 = cell_widths_1d(x1, side)
    gx, gy = np.meshgrid(x1, x1, indexing="ij")
    wx, wy = np.meshgrid(w1, w1, indexing="ij")
    xy = np.stack([gx.ravel(), gy.ravel()], axis=1)
    h = (wx * wy).ravel()
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs a seeded generator")
        cell = np.stack([wx.ravel(), wy.ravel()], axis=1)
        xy = xy + rng.uniform(-jitter, jitter, size=xy.shape) * cell
        xy = clamp_to_plane(xy, side, side)
    return xy, h


def grid_sensors(nx: int, ny: int, side_x: float, side_y: float):
    """Sensors exactly on the lattice x_a = (a - nx/2)*X/nx, y_b = (b - ny/2)*Y/ny
    (the regular grid of Section 2, eq. eval_equi), with h = dx*dy."""
    dx, dy = side_x / nx, side_y / ny
    xa = (np.arange(nx) - nx // 2) * dx
    yb = (np.arange(ny) - ny // 2) * dy
    gx, gy = np.meshgrid(xa, yb, indexing="ij")
    xy = np.stack([gx.ravel(), gy.ravel()], axis=1)
    h = np.full(nx * ny, dx * dy)
    return xy, h


def random_sensors(m: int, side_x: float, side_y: float, rng: np.random.Generator):
    """M uniform random sensors with equal weights X*Y/M."""
    xy = np.stack([rng.uniform(-0.5 * side_x, 0.5 * side_x, m),
                   rng.uniform(-0.5 * side_y, 0.5 * side_y, m)], axis=1)
    xy = clamp_to_plane(xy, side_x, side_y)
    return xy, np.full(m, side_x * side_y / m)


def equi_steradian_sensors(n_target: int, r0: float, drd: float):
    """Equi-steradian sensor placement (Appendix A) projected onto z = 0.

    The centre of interest sits at depth r0 below the plane centre; the
    detection region is the disc of diameter `drd`. The spherical cap seen
    from the centre of interest has solid angle Omega = 2*pi*(1 - cos th_max)
    with tan(th_max) = (drd/2)/r0; each sensor gets the unit solid angle
    omega = Omega/n_target. Polar slices k hold j_k points (a power of two)
    and satisfy omega*j_k = 2*pi*(cos th_{k-1} - cos th_k); j_k doubles when
    the chord between points of slice k exceeds 1.8 times the distance to the
    nearest point of slice k-1. Azimuths phi_{i,k} = 2*pi*i/j_k + pi/j_k +
    phi_r, with phi_r carried from the previous slice. Each point is placed
    at the polar angle midway between its slice's bounding angles.

    Returns (xy [M,2], r [M]) where r is the distance from the centre of
    interest to the sensor (the weighting of Section 6.2 uses h ~ r**3).
    The achieved M is near, not exactly, n_target.
    """
    th_max = math.atan2(0.5 * drd, r0)
    omega_cap = 2.0 * math.pi * (1.0 - math.cos(th_max))
    omega = omega_cap / n_target
    pts = []
    # slice 1: a single point at the pole enclosing exactly one unit solid angle
    cos_prev = 1.0 - omega / (2.0 * math.pi)
    th_prev = math.acos(max(-1.0, min(1.0, cos_prev)))
    pts.append((0.0, 0.0))
    j = 1
    phi_r = 0.0
    prev_ring = [(0.0, 0.0)]
    k = 1
    while th_prev < th_max - 1e-12:
        # tentative slice with j points; double j when chords grow too long
        jk = max(j, 1)
        while True:
            cos_next = math.cos(th_prev) - omega * jk / (2.0 * math.pi)
            if cos_next <= math.cos(th_max):
                cos_next = math.cos(th_max)
            th_next = math.acos(max(-1.0, min(1.0, cos_next)))
            th_mid = 0.5 * (th_prev + th_next)
            rho = r0 * math.tan(th_mid)
            chord = 2.0 * rho * math.sin(math.pi / jk) if jk > 1 else float("inf")
            ring = [(rho * math.cos(2 * math.pi * i / jk + math.pi / jk + phi_r),
                     rho * math.sin(2 * math.pi * i / jk + math.pi / jk + phi_r)) for i in range(jk)]
            dmin = min(math.hypot(px - qx, py - qy) for (px, py) in ring[:1] for (qx, qy) in prev_ring)
            if jk > 1 and chord > 1.8 * dmin:
                jk *= 2
                continue
            if jk == 1:
                jk = 2  # a ring needs at least two points to be a slice
                continue
            break
        pts.extend(ring)
        prev_ring = ring
        phi_r = phi_r + (k) * 2.0 * math.pi / jk
        th_prev = th_next
        j = jk
        k += 1
        if len(pts) > 8 * n_target + 64:
            break
    xy = np.array(pts, dtype=np.float64)
    r = np.sqrt(xy[:, 0] ** 2 + xy[:, 1] ** 2 + r0 ** 2)
    return xy, r


def power_weights(xy: np.ndarray, r: np.ndarray, power: float, total: float) -> np.ndarray:
    """Weights h_m proportional to r**power, normalised to sum to `total`
    (Section 6.2: h ~ r^3 in 3-D, ~ r^2 in 2-D)."""
    w = np.asarray(r, dtype=np.float64) ** power
    return w * (total / w.sum())


# ----------------------------------------------------------------------------
# Sources: uniform balls and their closed-form traces
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Balls:
    centres: np.ndarray  # [B,3] metres (x, y, z), z > 0 is depth
    radii: np.ndarray    # [B]
    p0: np.ndarray       # [B]

    def __len__(self):
        return len(self.radii)


def _ball_traces_part(xy, balls, idx, nt, dt, c):
    m = xy.shape[0]
    g = np.zeros((m, nt), dtype=np.float64)
    rows = np.arange(m)
    for b in idx:
        cx, cy, cz = balls.centres[b]
        R = float(balls.radii[b])
        a = float(balls.p0[b])
        d = np.sqrt((xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2 + cz * cz)
        n_lo = np.floor((d - R) / (c * dt)).astype(np.int64)
        width = int(math.ceil(2.0 * R / (c * dt))) + 3
        n_idx = n_lo[:, None] + np.arange(width)[None, :]
        arg = d[:, None] - c * (n_idx * dt)
        inside = (np.abs(arg) < R) & (n_idx >= 0) & (n_idx < nt)
        ii = np.broadcast_to(rows[:, None], n_idx.shape)[inside]
        nn = n_idx[inside]
        g[ii, nn] += (a * arg / (2.0 * d[:, None]))[inside]  # (m, n) pairs are distinct within one ball
    return g


def ball_traces(xy: np.ndarray, balls: Balls, nt: int, dt: float, c: float = C_SOUND,
                dtype=np.float64) -> np.ndarray:
    """Pressure traces on z = 0 from uniform balls (3-D wave equation, free space).

    For a ball of radius R, initial pressure p0, seen at distance d > R from its
    centre, the pressure is the N-shaped p0*(d - c*t)/(2*d) while |d - c*t| < R
    and 0 otherwise (strict inequality, point samples, no filter). Traces of
    several balls add. Returns g [M, nt].

    Many balls are split into a fixed number of contiguous groups summed on
    worker threads, then added in group order, so the result does not depend
    on the machine's core count.
    """
    xy = np.asarray(xy, dtype=np.float64)
    nballs = len(balls)
    groups = 1 if nballs < 64 else 8
    bounds = np.linspace(0, nballs, groups + 1).astype(int)
    parts = [range(bounds[i], bounds[i + 1]) for i in range(groups)]
    if groups == 1:
        g = _ball_traces_part(xy, balls, parts[0], nt, dt, c)
    else:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(groups) as ex:
            res = list(ex.map(lambda ix: _ball_traces_part(xy, balls, ix, nt, dt, c), parts))
        g = res[0]
        for r in res[1:]:
            g += r
    return g.astype(dtype, copy=False)


def voxelise_balls(balls: Balls, nx: int, ny: int, nz: int, X: float, Y: float, Z: float) -> np.ndarray:
    """Initial pressure sampled at the output voxels x_a = (a - nx/2)X/nx,
    y_b = (b - ny/2)Y/ny, z_e = e*Z/nz (sum of indicator functions)."""
    xa = (np.arange(nx) - nx // 2) * (X / nx)
    yb = (np.arange(ny) - ny // 2) * (Y / ny)
    ze = np.arange(nz) * (Z / nz)
    f = np.zeros((nx, ny, nz))
    for b in range(len(balls)):
        cx, cy, cz = balls.centres[b]
        R = balls.radii[b]
        r2 = ((xa[:, None, None] - cx) ** 2 + (yb[None, :, None] - cy) ** 2 + (ze[None, None, :] - cz) ** 2)
        f += balls.p0[b] * (r2 < R * R)
    return f


def random_balls(rng: np.random.Generator, count: int, r_range, p0_range, xy_half: float,
                 z_range_fn) -> Balls:
    """`count` balls with R ~ U(r_range), p0 ~ U(p0_range), centre x,y ~ U(+-xy_half)
    and z drawn by z_range_fn(R) -> (lo, hi)."""
    radii = rng.uniform(r_range[0], r_range[1], count)
    p0 = rng.uniform(p0_range[0], p0_range[1], count)
    cxy = rng.uniform(-xy_half, xy_half, (count, 2))
    cz = np.array([rng.uniform(*z_range_fn(R)) for R in radii])
    return Balls(np.column_stack([cxy, cz]), radii, p0)


def vessel_phantom(rng: np.random.Generator, n_tubes: int, side: float, depth: float) -> Balls:
    """Random-walk tubes rendered as ball sums.

    Each tube: radius ~ U(50, 200) um, start x,y ~ U(+-6 mm), z ~ U(4, 21) mm,
    length ~ U(3, 12) mm, p0 ~ U(0.5, 1). Balls of the tube's radius are
    placed every radius along a walk whose unit direction receives N(0, 0.15^2)
    perturbations per step and is renormalised. Balls that leave the
    reconstruction cube (with a one-radius margin) are dropped.
    """
    centres, radii, p0 = [], [], []
    for _ in range(n_tubes):
        r = rng.uniform(50e-6, 200e-6)
        pos = np.array([rng.uniform(-6e-3, 6e-3), rng.uniform(-6e-3, 6e-3), rng.uniform(4e-3, 21e-3)])
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        length = rng.uniform(3e-3, 12e-3)
        amp = rng.uniform(0.5, 1.0)
        nsteps = int(length / r)
        for _s in range(nsteps):
            inside = (abs(pos[0]) < 0.5 * side - r and abs(pos[1]) < 0.5 * side - r
                      and r < pos[2] < depth - r)
            if inside:
                centres.append(pos.copy())
                radii.append(r)
                p0.append(amp)
            d = d + rng.normal(0.0, 0.15, 3)
            d /= np.linalg.norm(d)
            pos = pos + r * d
    return Balls(np.array(centres).reshape(-1, 3), np.array(radii), np.array(p0))


def add_noise(g: np.ndarray, rel: float, rng: np.random.Generator) -> np.ndarray:
    """Add N(0, (rel*max|g|)^2) white noise."""
    s = rel * float(np.max(np.abs(g)))
    return g + rng.normal(0.0, s, size=g.shape)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One reconstruction problem: geometry, traces and output grid."""
    name: str
    xy: np.ndarray        # [M,2] float64, metres
    h: np.ndarray         # [M] float64, m^2
    g: np.ndarray         # [M,Nt] float64
    dt: float
    c: float
    shape: tuple          # (Nx, Ny, Nz)
    extent: tuple         # (X, Y, Z) metres
    balls: Balls | None = None

    @property
    def m(self):
        return self.xy.shape[0]

    @property
    def nt(self):
        return self.g.shape[1]


def config_problem(index: int, seed: int | None = None, with_data: bool = True) -> Problem:
    """The seeded synthetic workloads (seed defaults to 1000 + index).

    0: 16x16 warped sensors on a 10 mm plane, 128 samples at 20 MHz, one ball
       (R = 1 mm, p0 = 1) at seeded position, 32^3 output.
    1: 64x64 warped sensors on 20 mm, 1024 samples at 40 MHz, 8 balls
       (R ~ U(0.3, 1.5) mm, p0 ~ U(0.5, 1)) plus 1 % Gaussian noise, 128^3.
    2: 128x128 warped sensors with +-5 % jitter on 25 mm, 2048 samples at
       60 MHz, vessel phantom of 40 random-walk tubes, 256^3.
    4: 96x96 warped sensors on 20 mm, 1536 samples at 40 MHz, 8 balls, 192^3.
    Each output cube has side equal to the plane side (isotropic voxels).
    """
    seed = 1000 + index if seed is None else seed
    rng = np.random.default_rng(seed)
    c = C_SOUND
    if index == 0:
        ns, side, nt, dt, n = 16, 10e-3, 128, 50e-9, 32
        xy, h = warped_sensors(ns, side)
        balls = Balls(np.array([[rng.uniform(-1.5e-3, 1.5e-3), rng.uniform(-1.5e-3, 1.5e-3),
                                 rng.uniform(2.5e-3, 3.5e-3)]]), np.array([1e-3]), np.array([1.0]))
    elif index == 1:
        ns, side, nt, dt, n = 64, 20e-3, 1024, 25e-9, 128
        xy, h = warped_sensors(ns, side)
        balls = random_balls(rng, 8, (0.3e-3, 1.5e-3), (0.5, 1.0), 5e-3, lambda R: (R + 1e-3, 15e-3))
    elif index == 2:
        ns, side, nt, dt, n = 128, 25e-3, 2048, 1.0 / 60e6, 256
        xy, h = warped_sensors(ns, side, jitter=0.05, rng=rng)
        balls = vessel_phantom(rng, 40, side, side)
    elif index == 4:
        ns, side, nt, dt, n = 96, 20e-3, 1536, 25e-9, 192
        xy, h = warped_sensors(ns, side)
        balls = random_balls(rng, 8, (0.3e-3, 1.5e-3), (0.5, 1.0), 5e-3, lambda R: (R + 1e-3, 15e-3))
    else:
        raise ValueError(f"no single-problem workload {index}")
    g = None
    if with_data:
        g = ball_traces(xy, balls, nt, dt, c)
        if index == 1:
            g = add_noise(g, 0.01, rng)
    else:
        g = np.zeros((xy.shape[0], nt))
    return Problem(f"config{index}", xy, h, g, dt, c, (n, n, n), (side, side, side), balls)


def smooth235(n: int) -> int:
    """Smallest integer >= n whose only prime factors are 2, 3 and 5."""
    k = max(1, int(n))
    while True:
        r = k
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return k
        k += 1


def batched_problems(count: int = 32, seed: int = 1003) -> list[Problem]:
    """Uneven batch: Ns ~ U{24..96}, Nt ~ U{512..2048}, 20 mm plane, 40 MHz,
    4-8 balls each; output N = clamp(smooth235(2*Ns), 64, 192) per axis."""
    rng = np.random.default_rng(seed)
    out = []
    side, dt, c = 20e-3, 25e-9, C_SOUND
    for i in range(count):
        ns = int(rng.integers(24, 97))
        nt = int(rng.integers(512, 2049))
        n = min(192, max(64, smooth235(2 * ns)))
        if n % 2:
            n = smooth235(n + 1)
        xy, h = warped_sensors(ns, side)
        nb = int(rng.integers(4, 9))
        balls = random_balls(rng, nb, (0.3e-3, 1.5e-3), (0.5, 1.0), 5e-3, lambda R: (R + 1e-3, 15e-3))
        g = ball_traces(xy, balls, nt, dt, c)
        out.append(Problem(f"batch{i}", xy, h, g, dt, c, (n, n, n), (side, side, side), balls))
    return out


def random_problem(rng: np.random.Generator, m: int, nt: int, shape: Sequence[int],
                   extent: Sequence[float], dt: float, c: float = C_SOUND) -> Problem:
    """Random sensors (equal weights) and standard-normal traces: a generic
    linear-algebra test input with no physical structure."""
    xy, h = random_sensors(m, extent[0], extent[1], rng)
    g = rng.standard_normal((m, nt))
    return Problem("random", xy, h, g, dt, c, tuple(shape), tuple(extent))
