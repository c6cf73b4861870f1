"""How well the probe objective's derivatives are defined at all, on the
oracle alone (no GPU).

J = sum_n dt mean(p_w over the probe) of the 2-D dam break (dx = 0.02,
100 steps).  Its derivative with respect to the viscosity acts only through
the viscous term, a second difference of the velocity field: a perturbation
of the state the size of FP32 rounding moves dJ/dmu by a relative amount
above 1e-3, while dJ/dc0 moves by far less.  Any evaluation whose state
carries FP32 rounding (the FP32 forward of the adjoint rounds it at every
step, not once) inherits that spread in dJ/dmu, so the 1e-3 target for mu
is met with the FP64 forward, and the FP32-forward mu component is held to
a bar above this measured spread.
"""
import numpy as np
import pytest

from paper_2110_02621_amd import scenes

pytestmark = pytest.mark.slow


def _fp32(sc, x, v, rho):
    L = 2.0 * sc.h
    lo = sc.wall_x.min(axis=0) - sc.dx
    c = np.floor((x - lo) / L)
    off = ((x - lo) - c * L).astype(np.float32).astype(np.float64)
    return (lo + c * L + off, v.astype(np.float32).astype(np.float64),
            sc.rho0 + (rho - sc.rho0).astype(np.float32).astype(np.float64))


def _dJ(orc, name, rel, steps, rounded):
    base = scenes.dam_break_2d(dx=0.02, steps=steps)
    th = dict(mu=base.mu, gamma_p=base.gamma_p, c0=base.c0)
    h = rel * th[name]
    J = []
    for s in (+1, -1):
        kw = dict(th)
        kw[name] += s * h
        sc = scenes.dam_break_2d(dx=0.02, steps=steps, **kw)
        x, v, r = sc.fluid_x, sc.fluid_v, sc.fluid_rho
        if rounded:
            x, v, r = _fp32(sc, x, v, r)
        st = orc.State(orc.params_from_scene(sc), x, v, r, sc.wall_x, probe=sc.probe)
        st.step(steps)
        J.append(st.J)
    return (J[0] - J[1]) / (2 * h)


def test_dJ_dmu_spread_under_fp32_rounding_of_the_state(orc):
    out = {}
    for name, rel in (("mu", 0.1), ("c0", 1e-4)):
        a = _dJ(orc, name, rel, 100, False)
        b = _dJ(orc, name, rel, 100, True)
        out[name] = abs(b / a - 1.0)
        print(f"dJ/d{name}: exact start {a:.9e}, FP32-rounded start {b:.9e}, relative spread {out[name]:.2e}")
    assert out["mu"] > 1e-3
    assert out["c0"] < 1e-4
