"""Moving tank (prescribed translation X(t) = A0 sin(2 pi f0 t), Sec. 4.4)
on the HIP path against the FP64 oracle (needs an MI355X).

The HIP path holds the state in the tank's frame (walls at rest, the tank's
velocity taken out of the fluid's at each kick, g - X''(t) in Eq. (12));
the oracle moves the walls in the fixed frame.  The two are the same
discrete step (an exact change of frame), so they are compared in the fixed
frame with the bars of the fixed-wall runs: TOL32/TOL64, and for the light
phase of a two-phase run the 5e-4 of its number-density pressure.

Trajectories in FP32 are compared while they are predictable.  The shaken
two-phase tanks amplify a perturbation fast: the oracle itself, started
1e-6 dx away, is 1.7e-3 dx away after 300 steps (3-D, with or without the
motion), and in the strongly shaken 2-D two-phase tank its water
acceleration moves by 3e-4 of scale within 10 steps.  So FP32 trajectories
stop at the horizon of each case, and the FP32 arithmetic of later steps is
checked by one-step parity: the oracle resumes from the state the GPU
exports at steps 100 and 300 and both take one step.
"""
import math

import numpy as np
import pytest

import oracle as O
from gpu_cases import G, TOL32, TOL64
from paper_2110_02621_amd import scenes

pytestmark = pytest.mark.gpu

TOL32_LIGHT = 2e-4        # light phase, one step (measured <= 1.4e-4)
TOL32_LIGHT_TRAJ = 5e-4   # light phase, 10 or more steps (measured <= 3.3e-4)


@pytest.fixture(scope="module")
def solver_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2110_02621_amd import solver
    return solver


# last step of the FP32 trajectory comparison (see the module docstring)
HORIZON32 = {"slosh2d": 100, "slosh2d_2p": 10, "slosh3d_2p": 100}

CASES = {
    # strong shake (|X''| up to 7.9 m/s^2) so that 300 steps see the
    # acceleration term and the velocity kicks change
    "slosh2d": lambda: scenes.sloshing_tank(dim=2, dx=0.02, two_phase=False, amp=0.05, freq=2.0),
    "slosh2d_2p": lambda: scenes.sloshing_tank(dim=2, dx=0.02, two_phase=True, amp=0.05, freq=2.0),
    # the paper's excitation (A0 = 0.1 m, f0 = 0.496 Hz) on the 3-D tank
    "slosh3d_2p": lambda: scenes.sloshing_tank(dim=3, dx=0.03, two_phase=True),
}


def motion(sc, step):
    w = 2 * math.pi * sc.motion_freq
    t = step * sc.dt
    a = np.asarray(sc.motion_amp[: sc.dim])
    return a * math.sin(w * t), a * w * math.cos(w * t)


def errors(sc, e, st, pw_gpu):
    n_heavy = sc.n_heavy if sc.n_heavy is not None else sc.n_fluid
    heavy = np.arange(sc.n_fluid) < n_heavy
    r0 = np.where(heavy, sc.rho0, sc.rho0_light if sc.rho0_light else sc.rho0)
    dp = np.abs(sc.c0 ** 2 * (e["rho"] - st.rho)) / (r0 * G * sc.H)
    errs = dict(x=np.abs(e["pos"] - st.x).max() / sc.dx,
                v=np.abs(e["vel"] - st.v).max() / math.sqrt(2 * G * sc.H),
                p_heavy=dp[heavy].max(),
                pw=np.abs(pw_gpu - st.pw).max() / (sc.rho0 * G * sc.H))
    if (~heavy).any():
        errs["p_light"] = dp[~heavy].max()
    for name, sel in (("a_heavy", heavy), ("a_light", ~heavy)):
        if sel.any():
            errs[name] = np.abs(e["acc"][sel] - st.a[sel]).max() / max(G, np.abs(st.a[sel]).max())
    return errs


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_moving_tank_trajectory(solver_mod, name, prec):
    sc = CASES[name]()
    print(f"[moving] {name} {prec} nf={sc.n_fluid} nw={sc.n_wall} A0={sc.motion_amp[0]} "
          f"f0={sc.motion_freq}", flush=True)
    S = solver_mod.Solver(sc, prec)
    st = O.State(O.params_from_scene(sc), sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x)

    def tol(key, n):
        if prec == "f64":
            return TOL64
        if key.endswith("light"):
            return TOL32_LIGHT if n == 1 else TOL32_LIGHT_TRAJ
        return TOL32

    e0 = S.export()
    assert np.abs(e0["vel"] - st.v).max() < 1e-6  # input velocities in the fixed frame
    done = 0
    for n in (1, 10, 100, 300):
        if prec == "f32" and n > HORIZON32[name]:
            break
        S.step(n - done)
        st.step(n - done)
        done = n
        e = S.export()
        errs = errors(sc, e, st, S.export_walls()["pw"])
        print(f"  step {n}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        bad = {k: v for k, v in errs.items() if not v <= tol(k, n)}
        assert not bad, (n, bad)
    X, V = motion(sc, done)
    assert np.abs(S.export_walls()["pos"] - (sc.wall_x + X)).max() < 1e-6 * sc.dx
    d, od = S.diag(), st.diag()
    assert d["M"] == pytest.approx(od["M"], rel=1e-12)
    assert d["Ek"] == pytest.approx(od["Ek"], rel=1e-4 if prec == "f32" else 1e-9)
    assert d["Ep"] == pytest.approx(od["Ep"], rel=1e-6 if prec == "f32" else 1e-11)
    dP = np.abs(d["P"][: sc.dim] - od["P"][: sc.dim]).max()
    assert dP <= (1e-4 if prec == "f32" else 1e-9) * np.linalg.norm(od["P"]), dP
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_moving_tank_one_step_from_evolved_states(solver_mod, name, prec):
    sc = CASES[name]()
    print(f"[moving-1step] {name} {prec}", flush=True)
    P = O.params_from_scene(sc)
    S = solver_mod.Solver(sc, prec)
    done = 0
    for n in (100, 300):
        S.step(n - done)
        done = n
        e = S.export()
        st = O.State.resume(P, e["pos"], e["vel"], e["rho"], e["acc"], sc.wall_x, n)
        S.step(1)
        st.step(1)
        done += 1
        errs = errors(sc, S.export(), st, S.export_walls()["pw"])
        print(f"  from step {n}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        t = (lambda k: TOL64) if prec == "f64" else (lambda k: TOL32_LIGHT if k.endswith("light") else TOL32)
        bad = {k: v for k, v in errs.items() if not v <= t(k)}
        assert not bad, (n, bad)
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_moving_tank_masks_and_walk_agree_bitwise(solver_mod, prec):
    sc = CASES["slosh3d_2p"]()
    a = solver_mod.Solver(sc, prec, lists=True)
    b = solver_mod.Solver(sc, prec, lists=False)
    a.step(20)
    b.step(20)
    ea, eb = a.export(), b.export()
    for k in ("pos", "vel", "rho", "acc"):
        assert np.array_equal(ea[k], eb[k]), k
    assert np.array_equal(a.export_walls()["pw"], b.export_walls()["pw"])


def test_sloshing_long_run_fp64_matches_oracle(solver_mod):
    # 1 s of the 2-D Sec. 4.4 tank shaken at the paper's A0 and f0 (water
    # only, dx = 0.02, 3180 steps): the FP64 HIP path follows the oracle's
    # energy and momentum history.
    sc = scenes.sloshing_tank(dim=2, dx=0.02, two_phase=False)
    S = solver_mod.Solver(sc, "f64")
    st = O.State(O.params_from_scene(sc), sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x)
    n = int(round(1.0 / sc.dt))
    for k in range(6):
        S.step(n // 6)
        st.step(n // 6)
        d, od = S.diag(), st.diag()
        assert d["Ek"] + d["Ep"] == pytest.approx(od["Ek"] + od["Ep"], rel=1e-9), k
        assert d["P"][0] == pytest.approx(od["P"][0], rel=1e-7, abs=1e-9 * od["M"]), k
    e = S.export()
    assert np.abs(e["pos"] - st.x).max() < 1e-6 * sc.dx


def test_full_size_sloshing_sampled_parity(solver_mod):
    # The shaken two-phase tank at the paper's dx = 0.005 (1,410,752
    # particles) in the launch configuration the bench times (FP32), 20 steps
    # in; then one step stage by stage, compared in the fixed frame on
    # sampled particles that the oracle evaluates one by one (walls at
    # x_w(0) + X(t), moving with the step's displacement rate, a_w = X'').
    sc = scenes.sloshing_tank(dim=3, dx=0.005)
    print(f"[full-slosh] nf={sc.n_fluid} (water {sc.n_heavy}) nw={sc.n_wall}", flush=True)
    S = solver_mod.Solver(sc, "f32")
    n = 20
    S.step(n)
    P = O.params_from_scene(sc)
    dt = sc.dt
    X0, V0 = motion(sc, n)
    X1, V1 = motion(sc, n + 1)
    Vh = (X1 - X0) / dt
    w = 2 * math.pi * sc.motion_freq
    A1 = -np.asarray(sc.motion_amp[:3]) * w * w * math.sin(w * (n + 1) * dt)
    rng = np.random.default_rng(7)
    e0, w0 = S.export(), S.export_walls()
    wn = w0["nrm"]
    heavy = np.arange(sc.n_fluid) < sc.n_heavy
    near_wall = np.nonzero((e0["pos"][:, 0] - X0[0] < 3 * sc.dx) | (e0["pos"][:, 2] < 3 * sc.dx))[0]
    qf = np.unique(np.concatenate([rng.choice(sc.n_heavy, 1500, replace=False),
                                   rng.choice(np.nonzero(~heavy)[0], 1500, replace=False),
                                   rng.choice(near_wall, 1000, replace=False)]))
    qw = rng.choice(sc.n_wall, 2000, replace=False)
    assert np.abs(w0["pos"] - (sc.wall_x + X0)).max() < 1e-6 * sc.dx
    r0 = np.where(heavy, sc.rho0, sc.rho0_light)
    p_scale = r0 * G * sc.H
    errs = {}

    def perr(key, got, ref, sel):
        for ph, m in (("heavy", heavy[sel]), ("light", ~heavy[sel])):
            if m.any():
                errs[f"{key}_{ph}"] = float(np.abs(sc.c0 ** 2 * (got[m] - ref[m]) / p_scale[sel][m]).max())

    # density stage at r^n (walls at X(t_n))
    S.density()
    e_mid = S.export()  # velocity is the tank-frame half step plus X'(t_{n+1}): take that back out
    sig_o = O.sigma(P, e0["pos"], w0["pos"], query=qf)
    hq = heavy[qf]
    rt_o = np.where(hq, O.reinit(O.params_copy(P, n_heavy=sc.n_fluid), sig_o, e0["rho"][qf]),
                    O.reinit(O.params_copy(P, n_heavy=0), sig_o, e0["rho"][qf]))  # Eq. (17) / Eq. (18)
    perr("p_reinit", e_mid["rho"][qf], rt_o, qf)
    vh_gpu = e_mid["vel"][qf] - V1 + Vh
    errs["v_half"] = float(np.abs(vh_gpu - (e0["vel"][qf] + 0.5 * dt * e0["acc"][qf])).max()
                           / math.sqrt(2 * G * sc.H))
    S.build_cells()
    e1 = S.export()
    vh = e1["vel"] - V1 + Vh            # fixed-frame half-step velocity of every particle
    wx1 = sc.wall_x + X1
    errs["x1"] = float(np.abs(e1["pos"][qf] - (e0["pos"][qf] + dt * vh[qf])).max() / sc.dx)
    Q = O.params_copy(P, wall_v=Vh, a_wall=A1)
    S.wall_bc()
    pw1 = S.export_walls()["pw"]
    errs["pw"] = float(np.abs(pw1[qw] - O.wall_pressure(Q, wx1, e1["pos"], e1["rho"], query=qw)).max()
                       / (sc.rho0 * G * sc.H))
    S.continuity()
    e2 = S.export()
    D_o = O.continuity(Q, e1["pos"], vh, e1["rho"], wx1, pw1, query=qf)
    # heavy: Eq. (21); light: rho0_light sigma / sigma0 at r^{n+1}
    sig1 = O.sigma(P, e1["pos"], wx1, query=qf)
    perr("p_new", e2["rho"][qf], np.where(hq, e1["rho"][qf] + dt * D_o, sc.rho0_light * sig1 / P.sigma0), qf)
    S.momentum()
    e3 = S.export()
    A_o = O.momentum(Q, e1["pos"], vh, e2["rho"], wx1, pw1, wn, query=qf)
    for ph, m in (("heavy", heavy[qf]), ("light", ~heavy[qf])):
        errs[f"acc_{ph}"] = float(np.abs(e3["acc"][qf][m] - A_o[m]).max() / max(G, np.abs(A_o[m]).max()))
    errs["v_new"] = float(np.abs(e3["vel"][qf] - (vh[qf] + 0.5 * dt * A_o)).max() / math.sqrt(2 * G * sc.H))
    print("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), S.status(), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= (TOL32_LIGHT if k.endswith("light") else TOL32)}
    assert not bad, bad
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)
