"""Seeded synthetic workloads for the CRM step.

This module builds initial particle states and rigid-body marker sets. It holds
no arithmetic of the method itself: it places soil particles on a jittered
lattice and BCE markers on simple collision shapes, and returns plain numpy
arrays that both the FP64 oracle and the HIP library take as input.

Workloads (stand-ins for the paper's scenes, which are not available):
  * ``column``  -- granular column settling, 16x16x16 soil particles in a
    marker box (settling set-up of the validation studies, Sec. 3).
  * ``wheel``   -- single-wheel soil bin, 200x120x40 soil particles at
    dx = 5 mm with a grousered cylinder wheel (MGRU3 single-wheel test, Sec. 3.3,
    scaled down).
  * ``plate``   -- 32x32x16 soil patch pressed by a rigid plate.
  * ``strip``   -- long terrain strip with active boxes around four wheels
    (scalability study, Sec. 5), at a reduced length.

Marker placement follows the BCE description of Sec. 2.5.1: markers at spacing
d0 = dx in ceil(K h / d0) layers (K = 2), the first on the collision surface and
the others inward.

Positions are generated in FP64 and rounded to FP32 once; both sides use the
rounded values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Material and SPH parameters shared by all workloads (column settling set-up):
# rho0 = 1700 kg/m^3, E = 1 MPa, nu = 0.3, friction 0.7, no cohesion,
# h = 1.2 dx, cubic spline kernel, unilateral artificial viscosity 0.02
# (Table 1, single-wheel row), mu(I) constants of the cone-penetration study.
DEFAULT_PARAMS = dict(
    dx=0.01, h=0.012, dt=2.5e-5, gravity=(0.0, 0.0, -9.81),
    rho0=1700.0, E=1.0e6, nu=0.3, mu_s=0.7, mu_2=0.7, I0=0.08,
    grain_d=1.0e-3, cohesion=0.0,
    av_gamma=0.02, av_xi_over_h=0.1, av_mode=2,
    ps_freq=1,
    domain_lo=(0.0, 0.0, 0.0), domain_hi=(1.0, 1.0, 1.0),
    active_domains=0, t_delay=0.0,
    grow_G=1.2, shrink_S=0.75, shrink_interval=50,
    bulk_coeff=1.0, pos_mode=0, kernel=0, skin=0.0,
)


@dataclass
class Body:
    """A rigid body carrying BCE markers (body frame) and an optional active box."""
    markers: np.ndarray                     # (m, 3) float32, body-frame offsets
    active_half: tuple = (0.0, 0.0, 0.0)    # OOBB half extents at the body origin
    pos: tuple = (0.0, 0.0, 0.0)            # initial world position of the origin
    quat: tuple = (1.0, 0.0, 0.0, 0.0)      # initial orientation (w, x, y, z)
    linvel: tuple = (0.0, 0.0, 0.0)
    angvel: tuple = (0.0, 0.0, 0.0)
    name: str = ""


@dataclass
class Scene:
    name: str
    params: dict
    pos: np.ndarray                 # (n, 3) float32 soil positions
    vel: np.ndarray | None = None   # (n, 3) float32 or None (zero)
    sigma: np.ndarray | None = None  # (n, 6) float32 or None (zero)
    rho: np.ndarray | None = None   # (n,) float32 or None (rho0)
    bodies: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def n_soil(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_markers(self) -> int:
        return int(sum(b.markers.shape[0] for b in self.bodies))

    @property
    def n_total(self) -> int:
        return self.n_soil + self.n_markers


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def lattice(nx, ny, nz, dx, origin=(0.0, 0.0, 0.0), jitter=0.05, seed=0, fp64=False):
    """Cell-centred cubic lattice, x fastest, with uniform jitter of +-jitter*dx per axis.

    The lattice is built relative to `origin` and rounded to FP32 there; with
    fp64 the origin is added afterwards in FP64 (positions far from the
    coordinate origin, for cell-offset positions), else the result is FP32."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    p = np.stack([ix.ravel(order="F"), iy.ravel(order="F"), iz.ravel(order="F")], axis=1)
    p = (p.astype(np.float64) + 0.5) * dx
    if jitter:
        rng = np.random.default_rng(seed)
        p = p + rng.uniform(-jitter * dx, jitter * dx, size=p.shape)
    p = _f32(p).astype(np.float64)
    if fp64:
        return np.ascontiguousarray(p + np.asarray(origin, dtype=np.float64))
    return _f32(p + np.asarray(origin, dtype=np.float64))


def box_container(nx, ny, nz_wall, dx, layers=3):
    """Floor (``layers`` deep) and side walls (``layers`` thick, ``nz_wall`` high)
    around a bed of nx x ny cells whose lower corner is the origin."""
    pts = []
    r = range(-layers, 0)
    for k in r:                                     # floor, under the bed
        for j in range(-layers, ny + layers):
            for i in range(-layers, nx + layers):
                pts.append((i, j, k))
    for k in range(0, nz_wall):                     # side ring
        for j in range(-layers, ny + layers):
            for i in range(-layers, nx + layers):
                if 0 <= i < nx and 0 <= j < ny:
                    continue
                pts.append((i, j, k))
    p = (np.asarray(pts, dtype=np.float64) + 0.5) * dx
    return _f32(p)


def cylinder_wheel(radius, width, dx, layers=3, grousers=0, grouser_h=0.0, side_depth=None):
    """Wheel markers in the body frame, axis along y, origin at the wheel centre.

    Cylindrical shells at radius r - l*dx (l < layers), side annuli at
    y = +-(width/2 - l*dx) between radius r - layers*dx and r - side_depth, and
    straight full-width grousers of height grouser_h, one marker thick."""
    if side_depth is None:
        side_depth = 0.05
    ny = int(round(width / dx)) + 1
    ys = -0.5 * width + dx * np.arange(ny)
    pts = []
    for l in range(layers):
        rl = radius - l * dx
        nt = int(round(2.0 * math.pi * rl / dx))
        th = 2.0 * math.pi * np.arange(nt) / nt
        for y in ys:
            pts.append(np.stack([rl * np.cos(th), np.full(nt, y), rl * np.sin(th)], axis=1))
    r_in = radius - side_depth
    rr = radius - layers * dx
    while rr > r_in - 1e-12:
        nt = int(round(2.0 * math.pi * rr / dx))
        th = 2.0 * math.pi * np.arange(nt) / nt
        for l in range(layers):
            for sgn in (-1.0, 1.0):
                y = sgn * (0.5 * width - l * dx)
                pts.append(np.stack([rr * np.cos(th), np.full(nt, y), rr * np.sin(th)], axis=1))
        rr -= dx
    if grousers:
        ng = int(round(grouser_h / dx))
        for g in range(grousers):
            th = 2.0 * math.pi * g / grousers
            for m in range(1, ng + 1):
                rg = radius + m * dx
                pts.append(np.stack([np.full(ny, rg * math.cos(th)), ys,
                                     np.full(ny, rg * math.sin(th))], axis=1))
    return _f32(np.concatenate(pts, axis=0))


def plate(lx, ly, dx, layers=3):
    """Plate markers in the body frame: origin at the centre of the bottom face,
    first layer on the bottom face, the others above it (inside the plate)."""
    nx = int(round(lx / dx)) + 1
    ny = int(round(ly / dx)) + 1
    xs = -0.5 * lx + dx * np.arange(nx)
    ys = -0.5 * ly + dx * np.arange(ny)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pts = [np.stack([X.ravel(), Y.ravel(), np.full(X.size, l * dx)], axis=1) for l in range(layers)]
    return _f32(np.concatenate(pts, axis=0))


def _params(**over):
    p = dict(DEFAULT_PARAMS)
    p.update(over)
    return p


def column(seed=0, n=16, jitter=0.05, ps_freq=1, dx=0.01, walls=True, origin=None, pos_mode=0):
    """Granular column: n^3 soil particles in a 3-layer marker box (column settling).

    With `origin` the whole column (soil, container and domain) is translated
    there, positions staying FP64 (far-from-origin terrain)."""
    h = 1.2 * dx
    o = np.zeros(3) if origin is None else np.asarray(origin, dtype=np.float64)
    pos = lattice(n, n, n, dx, jitter=jitter, seed=seed, origin=o, fp64=origin is not None)
    bodies = []
    if walls:
        bodies.append(Body(markers=box_container(n, n, n, dx), pos=tuple(o), name="container"))
    lo = tuple(o + np.array([-4 * dx, -4 * dx, -4 * dx]))
    hi = tuple(o + np.array([(n + 4) * dx, (n + 4) * dx, (n + 4) * dx]))
    params = _params(dx=dx, h=h, ps_freq=ps_freq, domain_lo=lo, domain_hi=hi, pos_mode=pos_mode)
    return Scene("column", params, pos, bodies=bodies,
                 meta=dict(n_lattice=(n, n, n), seed=seed))


def wheel_bin(seed=0, nx=200, ny=120, nz=40, dx=0.005, slip=0.3, omega=0.8, load=100.0,
              ps_freq=10, wheel_x=None):
    """Single-wheel soil bin: nx*ny*nz soil particles, container, grousered wheel.

    Wheel r = 0.25 m, width 0.2 m, 12 grousers 0.01 m tall; the grouser tips start
    on the soil surface. Driving: omega = 0.8 rad/s, v = (1 - s) * omega * r_g with
    r_g the radius including grousers (slip definition of the single-wheel test)."""
    h = 1.2 * dx
    pos = lattice(nx, ny, nz, dx, seed=seed)
    bed = (nx * dx, ny * dx, nz * dx)
    nz_wall = int(math.floor((bed[2] + 2 * h) / dx - 0.5)) + 1
    cont = Body(markers=box_container(nx, ny, nz_wall, dx), name="container")
    r, w, gh = 0.25, 0.2, 0.01
    r_g = r + gh
    wm = cylinder_wheel(r, w, dx, layers=3, grousers=12, grouser_h=gh)
    wx = (0.3 * bed[0]) if wheel_x is None else wheel_x
    wpos = (wx, 0.5 * bed[1], bed[2] + r_g)
    v = (1.0 - slip) * omega * r_g
    wheel = Body(markers=wm, pos=wpos, linvel=(v, 0.0, 0.0), angvel=(0.0, omega, 0.0),
                 name="wheel")
    lo = (-4 * dx, -4 * dx, -4 * dx)
    hi = (bed[0] + 4 * dx, bed[1] + 4 * dx, bed[2] + 2 * r_g + 4 * dx)
    params = _params(dx=dx, h=h, ps_freq=ps_freq, domain_lo=lo, domain_hi=hi)
    return Scene("wheel", params, pos, bodies=[cont, wheel],
                 meta=dict(slip=slip, omega=omega, load=load, r_g=r_g, mass=load / 9.81,
                           n_lattice=(nx, ny, nz), seed=seed))


def plate_patch(seed=0, nx=32, ny=32, nz=16, dx=0.01, speed=0.05, ps_freq=10):
    """Soil patch with a 0.1 x 0.1 m plate starting one dx above the surface,
    moving down at ``speed``."""
    h = 1.2 * dx
    pos = lattice(nx, ny, nz, dx, seed=seed)
    bed = (nx * dx, ny * dx, nz * dx)
    nz_wall = int(math.floor((bed[2] + 2 * h) / dx - 0.5)) + 1
    cont = Body(markers=box_container(nx, ny, nz_wall, dx), name="container")
    pm = plate(0.1, 0.1, dx)
    pl = Body(markers=pm, pos=(0.5 * bed[0], 0.5 * bed[1], bed[2] + dx),
              linvel=(0.0, 0.0, -speed), name="plate")
    lo = (-4 * dx, -4 * dx, -4 * dx)
    hi = (bed[0] + 4 * dx, bed[1] + 4 * dx, bed[2] + 8 * dx)
    params = _params(dx=dx, h=h, ps_freq=ps_freq, domain_lo=lo, domain_hi=hi)
    return Scene("plate", params, pos, bodies=[cont, pl], meta=dict(seed=seed))


def strip(seed=0, length=20.0, width=4.0, depth=0.3, dx=0.05, speed=5.0, half=2.0,
          wheelbase=2.5, track=1.6, x0=None, t_delay=0.0, ps_freq=10):
    """Long terrain strip with a 3-layer floor and four wheels carrying active boxes
    (half-width ``half`` in x and y, full depth), moving at ``speed`` along x."""
    h = 1.2 * dx
    nx, ny, nz = int(round(length / dx)), int(round(width / dx)), int(round(depth / dx))
    pos = lattice(nx, ny, nz, dx, seed=seed)
    floor = []
    for k in range(-3, 0):
        ii, jj = np.meshgrid(np.arange(-3, nx + 3), np.arange(-3, ny + 3), indexing="ij")
        floor.append(np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, k)], axis=1))
    floor = _f32((np.concatenate(floor).astype(np.float64) + 0.5) * dx)
    bodies = [Body(markers=floor, name="floor")]
    r, w = 0.4, 0.3
    wm = cylinder_wheel(r, w, dx, layers=3, side_depth=0.15)
    cx = (0.5 * length) if x0 is None else x0
    hz = 0.5 * (depth + 2.0 * r + 2 * h)
    for sx in (-0.5, 0.5):
        for sy in (-0.5, 0.5):
            bodies.append(Body(markers=wm, pos=(cx + sx * wheelbase, 0.5 * width + sy * track, depth + r),
                               active_half=(half, half, hz), linvel=(speed, 0.0, 0.0),
                               angvel=(0.0, speed / r, 0.0), name="wheel"))
    lo = (-4 * dx, -4 * dx, -4 * dx)
    hi = (length + 4 * dx, width + 4 * dx, depth + 2 * r + 4 * dx)
    params = _params(dx=dx, h=h, dt=2.5e-4, ps_freq=ps_freq, domain_lo=lo, domain_hi=hi,
                     active_domains=1, t_delay=t_delay)
    return Scene("strip", params, pos, bodies=bodies, meta=dict(seed=seed))


def cluster(seed=0, n=6, dx=0.01, vel_scale=0.1, sigma_scale=1.0e3, gravity=(0.0, 0.0, 0.0)):
    """Isolated jittered cluster with random velocities and stresses, no markers
    (momentum-conservation workloads)."""
    h = 1.2 * dx
    pos = lattice(n, n, n, dx, seed=seed)
    rng = np.random.default_rng(seed + 1)
    vel = _f32(rng.normal(0.0, vel_scale, size=(pos.shape[0], 3)))
    sig = _f32(rng.normal(0.0, sigma_scale, size=(pos.shape[0], 6)))
    lo = (-10 * dx,) * 3
    hi = ((n + 10) * dx,) * 3
    params = _params(dx=dx, h=h, gravity=gravity, domain_lo=lo, domain_hi=hi)
    return Scene("cluster", params, pos, vel=vel, sigma=sig, meta=dict(seed=seed))


def batch_bins(seed=0, n_bins=64, n_min=8.0e3, n_max=2.5e5, dx=0.005, ps_freq=10, gap_cells=24,
               only=None):
    """Many independent single-wheel soil bins side by side along x in one domain.

    Bin sizes N_b are drawn log-uniformly in [n_min, n_max] with the bed aspect
    5:3:1 of the single-wheel bin; the wheel (r, width, grouser height) scales
    with the bed length. Per bin: friction mu_s in [0.5, 0.9] (material b),
    slip in [0, 0.6], load in [50, 200] N. Bins are separated by `gap_cells`
    particle spacings, far more than the 2h support, so no neighbour crosses bins.

    `only` keeps the listed bins (same positions and domain), for comparing a
    bin run alone with the same bin inside the batch."""
    rng = np.random.default_rng(seed)
    N = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_bins))
    mu = rng.uniform(0.5, 0.9, size=n_bins)
    slip = rng.uniform(0.0, 0.6, size=n_bins)
    load = rng.uniform(50.0, 200.0, size=n_bins)
    h = 1.2 * dx
    parts, mats, bodies, bins = [], [], [], []
    x0 = 0.0
    zmax = ymax = 0.0
    for b in range(n_bins):
        nz = max(4, int(round((N[b] / 15.0) ** (1.0 / 3.0))))
        ny, nx = 3 * nz, 5 * nz
        bed = (nx * dx, ny * dx, nz * dx)
        s = bed[0] / 1.0
        r = max(0.25 * s, 6 * dx)
        w = max(0.2 * s, 6 * dx)
        gh = max(dx, round(0.01 * s / dx) * dx)
        r_g = r + gh
        keep = only is None or b in only
        if keep:
            p = lattice(nx, ny, nz, dx, seed=seed + 1 + b).astype(np.float64) + np.array([x0, 0.0, 0.0])
            parts.append(_f32(p))
            mats.append(np.full(p.shape[0], len(bins), dtype=np.uint16))
            nz_wall = int(math.floor((bed[2] + 2 * h) / dx - 0.5)) + 1
            bodies.append(Body(markers=box_container(nx, ny, nz_wall, dx), pos=(x0, 0.0, 0.0), name=f"container{b}"))
            omega = 0.8
            v = (1.0 - slip[b]) * omega * r_g
            wm = cylinder_wheel(r, w, dx, layers=3, grousers=12, grouser_h=gh, side_depth=min(0.05, 0.4 * r))
            bodies.append(Body(markers=wm, pos=(x0 + 0.3 * bed[0], 0.5 * bed[1], bed[2] + r_g),
                               linvel=(v, 0.0, 0.0), angvel=(0.0, omega, 0.0), name=f"wheel{b}"))
            bins.append(dict(bin=b, n=nx * ny * nz, mu_s=float(mu[b]), slip=float(slip[b]), load=float(load[b]),
                             mass=float(load[b]) / 9.81, r_g=r_g, omega=omega, x0=x0))
        zmax = max(zmax, bed[2] + 2 * r_g)
        ymax = max(ymax, bed[1])
        x0 += bed[0] + gap_cells * dx
    pos = np.concatenate(parts) if parts else np.zeros((0, 3), dtype=np.float32)
    lo = (-4 * dx, -4 * dx, -4 * dx)
    hi = (x0, ymax + 4 * dx, zmax + 4 * dx)
    params = _params(dx=dx, h=h, ps_freq=ps_freq, domain_lo=lo, domain_hi=hi)
    sc = Scene("batch", params, pos, bodies=bodies,
               meta=dict(bins=bins, material=np.concatenate(mats) if mats else np.zeros(0, np.uint16),
                         materials=np.array([[bb["mu_s"], bb["mu_s"], 0.0] for bb in bins]), seed=seed))
    return sc
