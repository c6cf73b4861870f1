"""Dam break with a wedge (Sec. 4.5) on the HIP path (needs an MI355X).

Stage and trajectory parity of the small wedge scenes run with the other
scenes (test_gpu_parity.py).  Here: the 2-D wedge run in FP64 against the
oracle through the impact, and a 3-D run at dx = h_w/16 beyond what the
oracle reaches in test time, held to the oracle's own pins on the wedge:
no fluid particle past the first layer of dummies (depth dx below the
analytic face), and the total energy
(kinetic + potential + internal energy of the linear equation of state)
never growing.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2110_02621_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2110_02621_amd import solver
    return solver


def depth_in_wedge(sc, x):
    half = 0.5 * sc.meta["angle"]
    xa, hw = sc.meta["x_apex"], sc.meta["h_w"]
    b2 = hw * math.tan(half)
    c, s = math.cos(half), math.sin(half)
    z = x[:, sc.dim - 1]
    dl = c * (x[:, 0] - (xa - b2)) - s * z
    dr = c * ((xa + b2) - x[:, 0]) - s * z
    return np.where(z > 0.0, np.minimum(dl, dr), -1.0)


def total_energy(sc, d, rho):
    m = sc.rho0 * sc.dx ** sc.dim
    e_int = m * sc.c0 ** 2 * (np.log(rho / sc.rho0) + sc.rho0 / rho - 1.0)
    return d["Ek"] + d["Ep"] + e_int.sum()


def test_wedge_2d_fp64_matches_oracle_through_the_impact(solver_mod):
    sc = scenes.dam_break_wedge(res=10, dim=2)
    S = solver_mod.Solver(sc, "f64")
    st = O.State(O.params_from_scene(sc), sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x)
    n = int(round(4.0 / sc.dt))
    for k in range(8):
        S.step(n // 8)
        st.step(n // 8)
        d, od = S.diag(), st.diag()
        print(f"  t={S.diag()['steps'] * sc.dt:.2f} E={d['Ek'] + d['Ep']:.6e} oracle {od['Ek'] + od['Ep']:.6e}",
              flush=True)
        assert d["Ek"] + d["Ep"] == pytest.approx(od["Ek"] + od["Ep"], rel=1e-9), k
    e = S.export()
    assert np.abs(e["pos"] - st.x).max() < 1e-6 * sc.dx
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)


def test_wedge_3d_fp32_no_penetration_and_dissipation(solver_mod):
    sc = scenes.dam_break_wedge(res=16, dim=3)
    print(f"[wedge] 3-D res 16: {sc.n_fluid} fluid + {sc.n_wall} wall ({sc.meta['n_wedge_wall']} wedge)",
          flush=True)
    S = solver_mod.Solver(sc, "f32")
    E0 = total_energy(sc, S.diag(), S.export()["rho"])
    E_prev = E0
    n = int(round(4.0 / sc.dt))
    worst = -np.inf
    for k in range(20):
        S.step(n // 20)
        e = S.export()
        worst = max(worst, depth_in_wedge(sc, e["pos"]).max() / sc.dx)
        E = total_energy(sc, S.diag(), e["rho"])
        assert E <= E_prev + 1e-6 * abs(E0), (k, E, E_prev)
        E_prev = E
    print(f"  deepest fluid particle inside the wedge: {worst:.3f} dx; E/E0 = {E_prev / E0:.4f}", flush=True)
    xa, hw = sc.meta["x_apex"], sc.meta["h_w"]
    assert e["pos"][:, 0].max() > xa + hw * math.tan(sc.meta["angle"] / 2)  # water passed the wedge
    assert worst < 1.0
    assert E_prev < 0.99 * E0
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)
