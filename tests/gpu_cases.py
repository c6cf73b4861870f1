"""Shared inputs and comparison helpers of the GPU parity tests.

Scales of the scaled errors: rho -> rho0, p -> rho0 g H, v -> sqrt(2 g H),
dv/dt -> g (or the largest oracle value when that is larger: random
clouds have close pairs), positions -> dx.
"""
import math

import numpy as np

from paper_2110_02621_amd import scenes

G = 9.81
TOL32 = 1e-4   # FP32 path against the FP64 oracle (scaled max error)
TOL64 = 1e-9   # FP64 path against the FP64 oracle: summation order and FMA only


def tol(prec):
    return TOL32 if prec == "f32" else TOL64


def scales(sc):
    return dict(rho=sc.rho0, p=sc.rho0 * G * sc.H, v=math.sqrt(2 * G * sc.H), a=G, x=sc.dx)


def scaled(a, b, scale):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / scale)


def near_cutoff_scene(dim, n_pairs=1500, seed=0):
    """Particle pairs whose distance is within a few ulps of the support
    radius 2h, scattered over a box (stress case of the pair decision)."""
    base = scenes.random_box(dim=dim, n=2 * n_pairs, seed=seed, walls=True)
    rng = np.random.default_rng(seed + 100)
    side = base.fluid_x.max()
    a = rng.uniform(0.1 * side, 0.9 * side, size=(n_pairs, dim))
    u = rng.normal(size=(n_pairs, dim))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    k = rng.integers(-4, 5, size=(n_pairs, 1))
    r = 2.0 * base.h * (1.0 + k * 6e-8)
    b = a + u * r
    x = np.concatenate([a, b])
    x = np.clip(x, 0.0, side)
    return base.with_params(fluid_x=x, fluid_v=base.fluid_v[: len(x)], fluid_rho=base.fluid_rho[: len(x)],
                            name=f"near_cutoff_{dim}d")


def small_scenes():
    return {
        "box2d": lambda: scenes.random_box(dim=2, n=1500, seed=0),
        "box3d": lambda: scenes.random_box(dim=3, n=3000, seed=1),
        "dam3d": lambda: scenes.dam_break_3d(dx=0.03, steps=100),
        "dam2d": lambda: scenes.dam_break_2d(dx=0.04, steps=100),
        # the wedge of Sec. 4.5 (sharp corners: Eq. (16) normals, penalty)
        "wedge3d": lambda: scenes.dam_break_wedge(res=6, dim=3, tank=(16.0, 1.0, 3.0)),
        "wedge2d": lambda: scenes.dam_break_wedge(res=10, dim=2),
    }


def pair_set_from_lists(count, offset, lst):
    q = np.repeat(np.arange(len(count)), count)
    return set(zip(q.tolist(), lst.tolist()))
