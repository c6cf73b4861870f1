"""Seeded synthetic scenes: geometry, initial conditions and run parameters.

This module is the one input source shared by the oracle and the HIP path.
It holds none of the method's arithmetic: it places particles on lattices,
draws seeded random states, and fixes the run parameters of each workload
(particle spacing, smoothing length h = 1.3 dx and support 2.6 dx as in the
paper's Sec. 4, sound speed, time step).  Kernel sums, wall pressure, normals,
reference number density and every other step of the method are computed by
each side on its own.

Conventions: positions are row-major ``(n, dim)`` float64 arrays, the last
axis is vertical and gravity points along -e_{dim-1}.  Particles sit on the
lattice points (i + 1/2) dx (the paper places particles "regularly on a
Cartesian grid", Secs. 4.1 and 4.3).  Tanks have ``layers`` of wall dummy
particles on the floor and the side walls and an open top (Fig. 1).
"""
from __future__ import annotations

import math
import dataclasses
from dataclasses import dataclass, field

import numpy as np

G = 9.81            # gravity used for every case (Sec. 4)
RHO_WATER = 1000.0  # reference density of water (Secs. 4.1-4.3)
H_OVER_DX = 1.3     # smoothing length over particle spacing (Sec. 4)


@dataclass
class Scene:
    name: str
    dim: int
    dx: float
    h: float
    rho0: float
    c0: float
    mu: float
    gamma_p: float
    g: np.ndarray            # (3,) body force; unused trailing entries are 0
    dt: float
    steps: int
    H: float                 # initial water depth (hydrostatic reference)
    fluid_x: np.ndarray      # (Nf, dim)
    fluid_v: np.ndarray      # (Nf, dim)
    fluid_rho: np.ndarray    # (Nf,)
    wall_x: np.ndarray       # (Nw, dim)
    lo: np.ndarray           # (dim,) lower corner of the cell grid
    hi: np.ndarray           # (dim,) upper corner of the cell grid
    penalty_all: bool = True
    probe: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    meta: dict = field(default_factory=dict)
    # two phases: fluid particles [0, n_heavy) are the heavy phase (rho0),
    # the rest the light phase with reference density rho0_light
    n_heavy: int | None = None
    rho0_light: float | None = None
    # prescribed rigid translation of every wall dummy (the tank):
    # X(t) = motion_amp sin(2 pi motion_freq t)
    motion_amp: tuple = (0.0, 0.0, 0.0)
    motion_freq: float = 0.0
    # two phases: 1 = a light particle sees a heavy neighbour as a moving wall
    # dummy (p* of Eq. (11), the light phase's EOS density and mass) with the
    # heavy particle's pressure, 2 = the same with the pressure extrapolated
    # from the heavy particle's light neighbours (Eq. (12) divided by rho_f);
    # 0 = the Riemann p* of Eq. (8) with each side's own state
    cross_phase: int = 0

    @property
    def n_fluid(self) -> int:
        return int(self.fluid_x.shape[0])

    @property
    def n_wall(self) -> int:
        return int(self.wall_x.shape[0])

    def with_params(self, **kw) -> "Scene":
        d = dict(self.__dict__)
        d.update(kw)
        return Scene(**d)


def sound_speed(H: float) -> float:
    """c0 = 10 sqrt(2 g H), the run parameter of every workload here."""
    return 10.0 * math.sqrt(2.0 * G * H)


def time_step(h: float, c0: float) -> float:
    """Fixed step from the CFL and body-force limits (Eqs. (23)-(24)) with the
    anticipated maximum velocity c0/10."""
    return min(0.25 * h / (c0 + 0.1 * c0), 0.25 * math.sqrt(h / G))


def _lattice(n, dx, shift=None):
    """Lattice points (i + 1/2) dx, i in [0, n_k) per axis, x fastest."""
    axes = [(np.arange(k, dtype=np.float64) + 0.5) * dx for k in n]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    pts = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    if shift is not None:
        pts = pts + np.asarray(shift, dtype=np.float64)
    return pts


def tank_walls(dim, n_in, n_top, dx, layers=3):
    """Wall dummies of an open tank whose interior holds n_in[k] lattice
    columns per horizontal axis and n_top lattice rows in height.  The walls
    are ``layers`` lattice rows thick on the floor and the sides."""
    lo = [-layers] * dim
    hi = [n + layers for n in n_in] + [n_top]
    idx = [np.arange(lo[k], hi[k]) for k in range(dim)]
    grids = np.meshgrid(*idx[::-1], indexing="ij")
    ijk = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    inside = np.ones(len(ijk), dtype=bool)
    for k in range(dim - 1):
        inside &= (ijk[:, k] >= 0) & (ijk[:, k] < n_in[k])
    inside &= ijk[:, dim - 1] >= 0
    ijk = ijk[~inside]
    return (ijk.astype(np.float64) + 0.5) * dx


def closed_tank_walls(dim, n_in, n_top, dx, layers=3):
    """Wall dummies of a closed tank (floor, sides and lid, ``layers`` rows
    thick) around an interior of n_in[k] lattice columns per horizontal axis
    and n_top rows in height."""
    lo = [-layers] * dim
    hi = [n + layers for n in n_in] + [n_top + layers]
    idx = [np.arange(lo[k], hi[k]) for k in range(dim)]
    grids = np.meshgrid(*idx[::-1], indexing="ij")
    ijk = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    inside = np.ones(len(ijk), dtype=bool)
    for k in range(dim - 1):
        inside &= (ijk[:, k] >= 0) & (ijk[:, k] < n_in[k])
    inside &= (ijk[:, dim - 1] >= 0) & (ijk[:, dim - 1] < n_top)
    ijk = ijk[~inside]
    return (ijk.astype(np.float64) + 0.5) * dx


def _two_phase_rho(z, H, top, rho_w, rho_a, c0, heavy):
    """Initial densities whose linear-EOS pressures are the two-layer
    hydrostatic profile: rho_a g (top - z) in the air, rho_a g (top - H) +
    rho_w g (H - z) in the water."""
    p = np.where(heavy, rho_a * G * (top - H) + rho_w * G * (H - z), rho_a * G * (top - z))
    return np.where(heavy, rho_w, rho_a) + p / (c0 * c0)


def _hydrostatic_rho(z, H, rho0, c0):
    """Initial density whose linear-EOS pressure is rho0 g (H - z)."""
    return rho0 + rho0 * G * (H - z) / (c0 * c0)


def _box(lo, hi):
    return np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)


def hydrostatic_tank_2d(dx=0.025, H=1.0, L=1.0, top=1.1, mu=1e-3, steps=200):
    """2-D tank at rest: L x H water on a square lattice, 3 wall layers on the
    floor and the sides up to ``top``."""
    nx = int(round(L / dx))
    nz = int(round(H / dx))
    fx = _lattice([nx, nz], dx)
    wx = tank_walls(2, [nx], int(round(top / dx)), dx)
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    rho = _hydrostatic_rho(fx[:, 1], H, RHO_WATER, c0)
    lo, hi = _box([-3.5 * dx, -3.5 * dx], [L + 3.5 * dx, top + 6 * h])
    return Scene("hydrostatic_tank_2d", 2, dx, h, RHO_WATER, c0, mu, 1.0,
                 np.array([0.0, -G, 0.0]), time_step(h, c0), steps, H, fx, np.zeros_like(fx),
                 rho, wx, lo, hi, meta=dict(L=L, top=top))


def _obstacles(dx, seed, count, tank):
    """Wall dummies of ``count`` seeded spheres/cubes resting on the floor:
    lattice points inside the union that lie less than 3 dx below its
    surface.  Shape type 50/50, radius (or cube half-size) ~ U[0.03, 0.08],
    centre x ~ U[0.7, 1.5], y ~ U[r, W - r], z = r."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        kind = int(rng.integers(0, 2))
        r = float(rng.uniform(0.03, 0.08))
        cx = float(rng.uniform(0.7, 1.5))
        cy = float(rng.uniform(r, tank[1] - r))
        shapes.append((kind, r, np.array([cx, cy, r])))
    nx, ny, nz = (int(round(t / dx)) for t in tank)
    pts = []
    for kind, r, c in shapes:
        lo = np.maximum(np.floor((c - r) / dx - 1).astype(int), 0)
        hi = np.minimum(np.ceil((c + r) / dx + 1).astype(int), [nx, ny, nz])
        axes = [np.arange(lo[k], hi[k]) for k in range(3)]
        g = np.meshgrid(*axes[::-1], indexing="ij")
        ijk = np.stack([a.ravel() for a in g[::-1]], axis=1)
        pts.append(ijk)
    ijk = np.unique(np.concatenate(pts), axis=0)
    # keep x-fastest generation order
    order = np.lexsort((ijk[:, 0], ijk[:, 1], ijk[:, 2]))
    ijk = ijk[order]
    p = (ijk.astype(np.float64) + 0.5) * dx
    depth = np.full(len(p), -np.inf)
    for kind, r, c in shapes:
        if kind == 0:
            d = r - np.linalg.norm(p - c, axis=1)
        else:
            d = np.min(r - np.abs(p - c), axis=1)
        depth = np.maximum(depth, d)
    keep = (depth >= 0.0) & (depth < 3.0 * dx)
    return p[keep], shapes


def dam_break_3d(dx=0.004, obstacles=0, seed=0, mu=1e-3, steps=2000, headroom=0.3):
    """3-D dam break: a 0.6 (x) x 0.6 (y) x 0.3 (z) m water column in the
    corner of a 1.6 x 0.6 x 0.6 m tank, 3 wall layers, optional seeded
    obstacles on the floor."""
    tank = (1.6, 0.6, 0.6)
    H = 0.3
    ntank = [int(round(tank[0] / dx)), int(round(tank[1] / dx))]
    ncol = [int(round(0.6 / dx)), int(round(0.6 / dx)), int(round(H / dx))]
    fx = _lattice(ncol, dx)
    wx = tank_walls(3, ntank, int(round(tank[2] / dx)), dx)
    meta = dict(tank=tank, column=(0.6, 0.6, H))
    if obstacles:
        ox, shapes = _obstacles(dx, seed, obstacles, tank)
        wx = np.concatenate([wx, ox])
        meta["obstacles"] = [(k, r, c.tolist()) for k, r, c in shapes]
        meta["n_obstacle"] = int(len(ox))
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    rho = _hydrostatic_rho(fx[:, 2], H, RHO_WATER, c0)
    lo, hi = _box([-3.5 * dx] * 3, [tank[0] + 3.5 * dx, tank[1] + 3.5 * dx, tank[2] + headroom])
    name = "dam_break_3d" + ("_obstacles" if obstacles else "")
    return Scene(name, 3, dx, h, RHO_WATER, c0, mu, 1.0, np.array([0.0, 0.0, -G]),
                 time_step(h, c0), steps, H, fx, np.zeros_like(fx), rho, wx, lo, hi, meta=meta)


def dam_break_2d(dx=0.005, mu=1e-3, steps=1000, probe_height=0.1, column_height=2.0, c0=None,
                 gamma_p=1.0, width=1.0, tank=(4.0, 3.0)):
    """2-D dam break: a width x column_height column in a 4 x 3 m tank.  The
    probe is the innermost layer of the left wall for 0 < z < probe_height.

    The column height is a vertical stretch of the nominal 2 m lattice
    (z = s z_ref, s = column_height / 2; masses unchanged) with the
    hydrostatic density of that height.  Sound speed and time step default
    to the nominal column (c0 = 10 sqrt(2 g 2)) and do not follow a stretch
    or a given c0: dt is held fixed."""
    W, Ht = tank
    H_ref = 2.0
    ncol = [int(round(width / dx)), int(round(H_ref / dx))]
    fx = _lattice(ncol, dx)
    s = column_height / H_ref
    fx[:, 1] *= s
    wx = tank_walls(2, [int(round(W / dx))], int(round(Ht / dx)), dx)
    h = H_OVER_DX * dx
    c_nom = sound_speed(H_ref)
    c = c_nom if c0 is None else float(c0)
    rho = _hydrostatic_rho(fx[:, 1], column_height, RHO_WATER, c)
    probe = np.nonzero((np.abs(wx[:, 0] + 0.5 * dx) < 1e-9 * dx + 1e-12) &
                       (wx[:, 1] > 0.0) & (wx[:, 1] < probe_height))[0]
    lo, hi = _box([-3.5 * dx, -3.5 * dx], [W + 3.5 * dx, Ht + 0.5])
    return Scene("dam_break_2d", 2, dx, h, RHO_WATER, c, mu, gamma_p, np.array([0.0, -G, 0.0]),
                 time_step(h, c_nom), steps, column_height, fx, np.zeros_like(fx), rho, wx, lo, hi,
                 probe=probe.astype(np.int64), meta=dict(stretch=s, width=width, tank=tank))


def wall_jet_2d(dx=0.01, speed=6.0, steps=120, mu=1e-3, gamma_p=1.0, probe_height=0.2, c0=None):
    """2-D block of water (0.2 x 0.2 m) launched at `speed` towards the left
    wall of a 1 x 1 m tank, starting 1.5 dx from it: the impact drives
    particles within dx/2 of the wall dummies, where the penalty of
    Eqs. (13)-(15) acts.  Probe: innermost left-wall layer, z < probe_height."""
    H = 0.2
    n = int(round(0.2 / dx))
    fx = _lattice([n, n], dx, shift=(1.0 * dx, 0.0))
    fv = np.zeros_like(fx)
    fv[:, 0] = -speed
    wx = tank_walls(2, [int(round(1.0 / dx))], int(round(1.0 / dx)), dx)
    h = H_OVER_DX * dx
    c_nom = sound_speed(0.3)
    c = c_nom if c0 is None else float(c0)
    rho = _hydrostatic_rho(fx[:, 1], H, RHO_WATER, c)
    probe = np.nonzero((np.abs(wx[:, 0] + 0.5 * dx) < 1e-9 * dx + 1e-12) &
                       (wx[:, 1] > 0.0) & (wx[:, 1] < probe_height))[0]
    lo, hi = _box([-3.5 * dx, -3.5 * dx], [1.0 + 3.5 * dx, 1.5])
    return Scene("wall_jet_2d", 2, dx, h, RHO_WATER, c, mu, gamma_p, np.array([0.0, -G, 0.0]),
                 time_step(h, c_nom), steps, H, fx, fv, rho, wx, lo, hi, probe=probe.astype(np.int64))


def random_box(dim=3, n=1500, seed=0, dx=0.01, box_cells=None, walls=True, H=0.3, mu=1e-3,
               vel_scale=0.1, rho_noise=0.005):
    """Seeded random cloud for stage parity: n fluid particles uniform in a
    box above a 3-layer floor (or no walls), v ~ N(0, vel_scale sqrt(2gH)),
    rho = rho0 (1 + N(0, rho_noise))."""
    rng = np.random.default_rng(seed)
    side = (n / (1.0 if dim == 3 else 1.0)) ** (1.0 / dim) * dx if box_cells is None else box_cells * dx
    fx = rng.uniform(0.0, side, size=(n, dim))
    fv = rng.normal(0.0, vel_scale * math.sqrt(2 * G * H), size=(n, dim))
    rho = RHO_WATER * (1.0 + rng.normal(0.0, rho_noise, size=n))
    if walls:
        nside = int(math.ceil(side / dx))
        wx = tank_walls(dim, [nside] * (dim - 1), 0, dx)
        wx = wx[wx[:, dim - 1] < 0.0]
    else:
        wx = np.zeros((0, dim))
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    g = np.zeros(3)
    g[dim - 1] = -G
    lo = np.full(dim, -3.5 * dx)
    hi = np.full(dim, side + 3.5 * dx)
    return Scene(f"random_box_{dim}d_s{seed}", dim, dx, h, RHO_WATER, c0, mu, 1.0, g,
                 time_step(h, c0), 1, H, fx, fv, rho, wx, lo, hi)


RHO_AIR = 1.0  # reference density of air (Sec. 4.1)


def two_phase_tank_2d(dx=0.01, L=1.0, H=0.5, top=1.0, mu=0.0, steps=200, rho_air=RHO_AIR):
    """2-D two-phase hydrostatic tank (Sec. 4.1): an L x top closed tank,
    water below z = H, air above, both at rest on one square lattice; water
    particles come first.  Inviscid as in the paper; the penalty acts on the
    light phase only; one sound speed c0 = 10 sqrt(2 g H) for both phases."""
    nx = int(round(L / dx))
    nzw = int(round(H / dx))
    nz = int(round(top / dx))
    pts = _lattice([nx, nz], dx)
    heavy = pts[:, 1] < H
    fx = np.concatenate([pts[heavy], pts[~heavy]])
    is_heavy = np.arange(len(fx)) < int(heavy.sum())
    wx = closed_tank_walls(2, [nx], nz, dx)
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    rho = _two_phase_rho(fx[:, 1], H, top, RHO_WATER, rho_air, c0, is_heavy)
    lo, hi = _box([-3.5 * dx, -3.5 * dx], [L + 3.5 * dx, top + 3.5 * dx])
    return Scene("two_phase_tank_2d", 2, dx, h, RHO_WATER, c0, mu, 1.0, np.array([0.0, -G, 0.0]),
                 time_step(h, c0), steps, H, fx, np.zeros_like(fx), rho, wx, lo, hi, penalty_all=False,
                 meta=dict(L=L, top=top, nzw=nzw), n_heavy=int(heavy.sum()), rho0_light=rho_air)


def dam_break_3d_two_phase(dx=0.005, mu=0.0, steps=1000, rho_air=RHO_AIR):
    """3-D two-phase dam break: the water column of the 3-D dam break (0.6 x
    0.6 x 0.3 m in a 1.6 x 0.6 x 0.6 m tank) with air on every other lattice
    site of the tank, which is closed by a lid; water particles come first."""
    tank = (1.6, 0.6, 0.6)
    H = 0.3
    n = [int(round(t / dx)) for t in tank]
    pts = _lattice(n, dx)
    heavy = (pts[:, 0] < 0.6) & (pts[:, 2] < H)
    fx = np.concatenate([pts[heavy], pts[~heavy]])
    is_heavy = np.arange(len(fx)) < int(heavy.sum())
    wx = closed_tank_walls(3, n[:2], n[2], dx)
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    top = tank[2]
    rho = np.where(is_heavy, _hydrostatic_rho(fx[:, 2], H, RHO_WATER, c0),
                   rho_air + rho_air * G * (top - fx[:, 2]) / (c0 * c0))
    lo, hi = _box([-3.5 * dx] * 3, [tank[0] + 3.5 * dx, tank[1] + 3.5 * dx, tank[2] + 3.5 * dx])
    return Scene("dam_break_3d_two_phase", 3, dx, h, RHO_WATER, c0, mu, 1.0, np.array([0.0, 0.0, -G]),
                 time_step(h, c0), steps, H, fx, np.zeros_like(fx), rho, wx, lo, hi, penalty_all=False,
                 meta=dict(tank=tank), n_heavy=int(heavy.sum()), rho0_light=rho_air)


SLOSH_TANK = (1.3, 0.1, 0.9)  # length x depth x height of the sloshing tank (Sec. 4.4)
SLOSH_H = 0.18                # water depth, 20 % of the height
SLOSH_A0 = 0.1                # excitation amplitude (m)
SLOSH_F0 = 0.496              # excitation frequency (1/s)


def sloshing_tank(dim=3, dx=0.01, two_phase=True, amp=SLOSH_A0, freq=SLOSH_F0, layers=4,
                  steps=1000, mu=0.0, rho_air=RHO_AIR):
    """Sloshing tank of Sec. 4.4: a closed 1.3 (x) x 0.1 (y, 3-D only) x
    0.9 (z) m tank, water to 0.18 m, air above (two_phase) or nothing,
    ``layers`` rows of wall dummies all round (4 reproduces the paper's
    particle counts: 243,432 at dx = 0.01 and 1,410,752 at dx = 0.005), the
    whole tank translated along x by X(t) = amp sin(2 pi freq t).  The fluid
    starts in hydrostatic equilibrium at rest relative to the tank (moving
    with X'(0)); water particles come first.  Inviscid; the penalty acts on
    the light phase in a two-phase run and on every particle otherwise."""
    L, W, D = SLOSH_TANK
    H = SLOSH_H
    n_in = [int(round(L / dx))] + ([int(round(W / dx))] if dim == 3 else [])
    nz = int(round(D / dx))
    pts = _lattice(n_in + [nz], dx)
    z = pts[:, dim - 1]
    heavy = z < H
    if two_phase:
        fx = np.concatenate([pts[heavy], pts[~heavy]])
    else:
        fx = pts[heavy]
    is_heavy = np.arange(len(fx)) < int(heavy.sum())
    wx = closed_tank_walls(dim, n_in, nz, dx, layers=layers)
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    rho = _two_phase_rho(fx[:, dim - 1], H, D if two_phase else H, RHO_WATER, rho_air, c0, is_heavy)
    amp_v = np.zeros(3)
    amp_v[0] = amp
    fv = np.zeros_like(fx)
    fv[:, 0] = amp * 2.0 * math.pi * freq  # X'(0): at rest in the tank
    pad = (layers + 0.5) * dx
    top = [L + pad] + ([W + pad] if dim == 3 else []) + [D + pad]
    lo, hi = _box([-pad] * dim, top)
    g = np.zeros(3)
    g[dim - 1] = -G
    extra = dict(n_heavy=int(heavy.sum()), rho0_light=rho_air) if two_phase else {}
    return Scene(f"sloshing_{dim}d" + ("_two_phase" if two_phase else ""), dim, dx, h, RHO_WATER,
                 c0, mu, 1.0, g, time_step(h, c0), steps, H, fx, fv, rho, wx, lo, hi,
                 penalty_all=not two_phase, meta=dict(tank=SLOSH_TANK[:dim - 1] + (D,),
                                                      layers=layers),
                 motion_amp=tuple(amp_v), motion_freq=float(freq), **extra)


def shaken(sc, amp=0.05, freq=5.0, axis=0):
    """``sc`` in a tank translated along ``axis`` by X(t) = amp sin(2 pi
    freq t) (walls, probe and all), the fluid at rest relative to the tank
    at t = 0 (moving with X'(0))."""
    a = [0.0, 0.0, 0.0]
    a[axis] = float(amp)
    fv = np.array(sc.fluid_v, dtype=np.float64, copy=True)
    fv[:, axis] += amp * 2.0 * math.pi * freq
    return dataclasses.replace(sc, name=sc.name + "_shaken", fluid_v=fv, motion_amp=tuple(a),
                               motion_freq=float(freq))


WEDGE_H = 5.5  # wedge height h_w (Sec. 4.5)


def wedge_walls(dx, n_in, x_apex, h_w, angle=math.pi / 3, layers=4):
    """Wall dummies of a wedge on the floor: a prism across the tank width
    (axis y in 3-D) whose cross-section is the isosceles triangle with apex
    (x_apex, h_w) of opening ``angle`` and base on the floor z = 0.  The
    dummies are the lattice points (i + 1/2) dx inside it within ``layers``
    dx of a sloped face (the base sits on the tank floor)."""
    dim = len(n_in) + 1
    half = 0.5 * angle
    b2 = h_w * math.tan(half)  # half base width
    nzw = int(math.ceil(h_w / dx))
    ix = np.arange(int(math.floor((x_apex - b2) / dx)) - 1, int(math.ceil((x_apex + b2) / dx)) + 1)
    iz = np.arange(0, nzw)
    axes = [ix] + ([np.arange(n_in[1])] if dim == 3 else []) + [iz]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    ijk = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    p = (ijk.astype(np.float64) + 0.5) * dx
    x, z = p[:, 0], p[:, dim - 1]
    c, s = math.cos(half), math.sin(half)
    # distances inside the two sloped faces (outward normals (-c, s), (c, s))
    dl = c * (x - (x_apex - b2)) - s * z
    dr = c * ((x_apex + b2) - x) - s * z
    depth = np.minimum(dl, dr)
    keep = (depth >= 0.0) & (depth < layers * dx)
    return p[keep]


def dam_break_wedge(res=40, h_w=WEDGE_H, tank=(16.0, 5.5, 3.0), column=(6.0, 2.0), layers=4,
                    mu=0.0, steps=1000, penalty_all=True, dim=3):
    """Dam break with a wedge (Sec. 4.5): dx = h_w / res, a pi/3 wedge of
    height h_w across the whole width on the middle of the downstream bed.
    Tank length x width x side height and the water column's length x height
    are in units of h_w (the paper's tank was in a figure; these sizes give
    about its 5,734,250 particles at res = 40).  ``layers`` rows of wall
    dummies on the floor and the sides, open top.  dim = 2 drops the width."""
    dx = h_w / res
    n = lambda v: int(round(v * h_w / dx))
    nx, ny, nz = n(tank[0]), n(tank[1]), n(tank[2])
    ncx, ncz = n(column[0]), n(column[1])
    H = ncz * dx
    horiz = [nx, ny] if dim == 3 else [nx]
    fx = _lattice([ncx] + horiz[1:] + [ncz], dx)
    x_apex = (ncx + (nx - ncx) // 2) * dx  # a lattice face: the wedge is mirror-symmetric on the lattice
    wt = tank_walls(dim, horiz, nz, dx, layers=layers)
    ww = wedge_walls(dx, horiz, x_apex, h_w, layers=layers)
    wx = np.concatenate([wt, ww])
    h = H_OVER_DX * dx
    c0 = sound_speed(H)
    rho = _hydrostatic_rho(fx[:, dim - 1], H, RHO_WATER, c0)
    pad = (layers + 0.5) * dx
    top = [nx * dx + pad] + ([ny * dx + pad] if dim == 3 else []) + [nz * dx + 0.5 * H]
    lo, hi = _box([-pad] * dim, top)
    g = np.zeros(3)
    g[dim - 1] = -G
    return Scene(f"dam_break_wedge_{dim}d", dim, dx, h, RHO_WATER, c0, mu, 1.0, g,
                 time_step(h, c0), steps, H, fx, np.zeros_like(fx), rho, wx, lo, hi,
                 penalty_all=penalty_all,
                 meta=dict(h_w=h_w, x_apex=x_apex, angle=math.pi / 3, n_tank_wall=int(len(wt)),
                           n_wedge_wall=int(len(ww)), layers=layers, tank_l=nx * dx,
                           tank_w=(ny * dx if dim == 3 else None)))


def inside_wedge(sc, x):
    """True for points strictly inside the wedge solid of a wedge scene."""
    x = np.asarray(x, dtype=np.float64)
    half = 0.5 * sc.meta["angle"]
    xa, hw = sc.meta["x_apex"], sc.meta["h_w"]
    b2 = hw * math.tan(half)
    c, s_ = math.cos(half), math.sin(half)
    z = x[:, sc.dim - 1]
    dl = c * (x[:, 0] - (xa - b2)) - s_ * z
    dr = c * ((xa + b2) - x[:, 0]) - s_ * z
    return (dl > 0) & (dr > 0) & (z > 0)


def by_name(name: str, **kw) -> Scene:
    table = {
        "hydrostatic_tank_2d": hydrostatic_tank_2d,
        "dam_break_3d": dam_break_3d,
        "dam_break_3d_obstacles": lambda **k: dam_break_3d(obstacles=8, **k),
        "dam_break_2d": dam_break_2d,
        "wall_jet_2d": wall_jet_2d,
        "random_box": random_box,
        "two_phase_tank_2d": two_phase_tank_2d,
        "dam_break_3d_two_phase": dam_break_3d_two_phase,
        "sloshing_tank": sloshing_tank,
        "dam_break_wedge": dam_break_wedge,
    }
    return table[name](**kw)
