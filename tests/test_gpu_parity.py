"""HIP path against the FP64 oracle, through the C ABI (needs an MI355X).

Integer results (cell keys, sorted order, cell tables, neighbour pair sets)
must match bit for bit; fields must match within the scaled tolerances of
gpu_cases (1e-4 for the FP32 path, 1e-9 for the FP64 path).  Stage tests
feed the oracle exactly the state the GPU held before the stage.
"""
import math

import numpy as np
import pytest

import oracle as O
from gpu_cases import (G, TOL32, near_cutoff_scene, pair_set_from_lists, scaled, scales,
                       small_scenes, tol)
from paper_2110_02621_amd import scenes

pytestmark = pytest.mark.gpu

SMALL = small_scenes()


@pytest.fixture(scope="module")
def solver_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2110_02621_amd import solver
    return solver


def by_pid(raw_pid, values):
    out = np.empty_like(values)
    out[raw_pid] = values
    return out


# ---------------------------------------------------------------- sort + pairs
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", ["box2d", "box3d", "dam3d", "wedge3d", "near2d", "near3d"])
def test_pair_sets_and_sort_bitexact(solver_mod, name, prec):
    sc = near_cutoff_scene(int(name[-2])) if name.startswith("near") else SMALL[name]()
    print(f"[pairs] {name} {prec} nf={sc.n_fluid} nw={sc.n_wall}", flush=True)
    S = solver_mod.Solver(sc, prec)
    raw = S.raw()
    dim, nf = sc.dim, sc.n_fluid
    key = raw["key"][0]
    # sorted by key, cell table consistent with the keys
    assert np.all(np.diff(key) >= 0)
    cnt = np.bincount(key, minlength=int(S.desc.n_cells))
    assert np.array_equal(raw["fstart"], np.concatenate([[0], np.cumsum(cnt)]))
    wcnt = np.bincount(raw["wkey"], minlength=int(S.desc.n_cells))
    assert np.array_equal(raw["wstart"], np.concatenate([[0], np.cumsum(wcnt)]))
    # fluid order: by cell key, inside a cell by x offset (as stored, in the
    # kernel precision), ties by prior index (the input order: ids ascending)
    pid = raw["pid"][0]
    key_id = np.empty_like(key)
    key_id[pid] = key
    x_id = np.empty(nf, dtype=raw["off"][0].dtype)
    x_id[pid] = raw["off"][0][0]
    assert np.array_equal(pid, np.lexsort((np.arange(nf), x_id, key_id)))
    # walls: by cell key, ties by source index (a stable counting sort)
    assert np.array_equal(raw["wpid"], O.counting_sort(raw["wkey"][np.argsort(raw["wpid"])],
                                                       int(S.desc.n_cells))[1])
    # pair sets in the kernel's precision
    single = prec == "f32"
    L = float(S.desc.cell)
    rc2 = float(np.float32(4.0 * sc.h * sc.h)) if single else 4.0 * sc.h * sc.h
    cf, of = S.cell_coords(key), raw["off"][0].T
    cw, ow = S.cell_coords(raw["wkey"]), raw["woff"].T
    pid, wpid = raw["pid"][0], raw["wpid"]
    hff = O.pairs_bruteforce(dim, single, cf, of, cf, of, L, rc2)
    a, b = np.nonzero(hff)
    ref = set(zip(pid[a].tolist(), pid[b].tolist()))
    if sc.n_wall:
        hfw = O.pairs_bruteforce(dim, single, cf, of, cw, ow, L, rc2)
        a, b = np.nonzero(hfw)
        ref |= set(zip(pid[a].tolist(), (nf + wpid[b]).tolist()))
    same_pairs(pair_set_from_lists(*S.neighbours(0)), ref)
    if sc.n_wall:
        hwf = O.pairs_bruteforce(dim, single, cw, ow, cf, of, L, rc2)
        a, b = np.nonzero(hwf)
        ref_w = set(zip(wpid[a].tolist(), pid[b].tolist()))
        same_pairs(pair_set_from_lists(*S.neighbours(1)), ref_w)


def same_pairs(got, ref):
    """Equal pair sets; on a mismatch the counts and a few examples (a
    plain set comparison would have pytest diff sets of 1e5 pairs)."""
    missing, extra = ref - got, got - ref
    assert not missing and not extra, (len(missing), len(extra), sorted(missing)[:5], sorted(extra)[:5])


# ---------------------------------------------------------------- one step, stage by stage
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", ["box2d", "box3d", "dam3d", "dam2d", "wedge3d", "wedge2d"])
def test_stage_parity(solver_mod, name, prec):
    sc = SMALL[name]()
    print(f"[stage] {name} {prec} nf={sc.n_fluid} nw={sc.n_wall}", flush=True)
    sc_ = scales(sc)
    t = tol(prec)
    S = solver_mod.Solver(sc, prec, keep_sigma=True)
    P = O.params_from_scene(sc)
    e0, w0 = S.export(), S.export_walls()
    x0, v0, r0, a0 = e0["pos"], e0["vel"], e0["rho"], e0["acc"]
    wx, wn, pw0 = w0["pos"], w0["nrm"], w0["pw"]
    errs = {}
    # init: positions converted to cell + offset
    errs["x0"] = scaled(x0, sc.fluid_x, sc_["x"])
    errs["wx"] = scaled(wx, sc.wall_x, sc_["x"])
    # init: normals (Eq. 16) where they are clearly defined, initial p_w and dv/dt
    if sc.n_wall:
        n_o, psi = O.normals(P, wx, with_psi=True)
        big = np.linalg.norm(psi, axis=1) * sc.h > 1e-3
        small = np.linalg.norm(psi, axis=1) * sc.h < 1e-6
        errs["nrm"] = scaled(wn[big], n_o[big], 1.0)
        assert np.all(wn[small] == 0.0)
        errs["pw0"] = scaled(pw0, O.wall_pressure(P, wx, x0, r0), sc_["p"])
    A0 = O.momentum(P, x0, v0, r0, wx, pw0, wn)
    errs["a0"] = scaled(a0, A0, max(G, np.abs(A0).max()))
    # density stage: sigma, Eq. (17), half kick, drift
    S.density()
    raw = S.raw()
    pid = raw["pid"][0]
    sig = by_pid(pid, raw["sigma"])
    sig_o = O.sigma(P, x0, wx)
    errs["sigma"] = scaled(sig, sig_o, P.sigma0)
    rt_o = O.reinit(P, sig_o, r0)
    rt = by_pid(pid, raw["rho"][raw["sel_rho"]].astype(np.float64)) + sc.rho0
    errs["rho_reinit"] = scaled(rt, rt_o, sc_["rho"])
    errs["p_reinit"] = scaled(sc.c0 ** 2 * (rt - sc.rho0), sc.c0 ** 2 * (rt_o - sc.rho0), sc_["p"])
    vh_o = v0 + 0.5 * sc.dt * a0
    vh = by_pid(pid, raw["vel"][raw["sel_vel"]].T.astype(np.float64))
    errs["v_half"] = scaled(vh, vh_o, sc_["v"])
    x1 = by_pid(raw["pid"][1], S.absolute(raw["key"][1], raw["off"][1]))
    errs["x1"] = scaled(x1, x0 + sc.dt * vh, sc_["x"])
    # cell build: the drifted keys sorted, inside each cell by x offset, ties
    # by prior order
    S.build_cells()
    raw2 = S.raw()
    n1 = len(raw["key"][1])
    order = np.lexsort((np.arange(n1), raw["off"][1][0], raw["key"][1]))
    assert np.array_equal(raw2["pid"][0], raw["pid"][1][order])
    assert np.array_equal(raw2["key"][0], raw["key"][1][order])
    e1 = S.export()
    errs["x1_sorted"] = scaled(e1["pos"], x1, sc_["x"])
    assert np.array_equal(e1["vel"], vh) and np.array_equal(e1["rho"], rt)
    # wall pressure, Eq. (12)
    S.wall_bc()
    pw1 = S.export_walls()["pw"]
    if sc.n_wall:
        errs["pw"] = scaled(pw1, O.wall_pressure(P, wx, e1["pos"], e1["rho"]), sc_["p"])
    # continuity, Eqs. (9), (21)
    rb = S.raw()
    S.continuity()
    e2 = S.export()
    D_o = O.continuity(P, e1["pos"], e1["vel"], e1["rho"], wx, pw1)
    errs["rho_new"] = scaled(e2["rho"], e1["rho"] + sc.dt * D_o, sc_["rho"])
    errs["p_new"] = scaled(sc.c0 ** 2 * (e2["rho"] - sc.rho0),
                           sc.c0 ** 2 * (e1["rho"] + sc.dt * D_o - sc.rho0), sc_["p"])
    if prec == "f64":
        # drho/dt itself, from the device's stored deviations rho - rho0
        # before and after the update (the exported full densities would
        # cancel ~13 of their 16 digits in the difference)
        ra = S.raw()
        dev_b = by_pid(rb["pid"][0], rb["rho"][rb["sel_rho"]].astype(np.float64))
        dev_a = by_pid(ra["pid"][0], ra["rho"][ra["sel_rho"]].astype(np.float64))
        errs["drho_dt"] = scaled((dev_a - dev_b) / sc.dt, D_o, np.abs(D_o).max() + 1e-30)
    # momentum, Eqs. (10)-(11), (13)-(15), (22)
    S.momentum()
    e3 = S.export()
    A_o = O.momentum(P, e1["pos"], e1["vel"], e2["rho"], wx, pw1, wn)
    errs["acc"] = scaled(e3["acc"], A_o, max(G, np.abs(A_o).max()))
    errs["v_new"] = scaled(e3["vel"], e1["vel"] + 0.5 * sc.dt * A_o, sc_["v"])
    st = S.status()
    print("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), st, flush=True)
    assert st["out_of_grid"] == 0 and st["fast"] == 0
    bad = {k: v for k, v in errs.items() if not v <= t}
    assert not bad, bad


# ---------------------------------------------------------------- trajectories
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", ["dam3d", "dam2d", "wedge3d", "wedge2d"])
def test_trajectory_steps_1_10_100(solver_mod, name, prec):
    sc = SMALL[name]()
    print(f"[traj] {name} {prec} nf={sc.n_fluid} nw={sc.n_wall}", flush=True)
    s = scales(sc)
    S = solver_mod.Solver(sc, prec)
    P = O.params_from_scene(sc)
    st = O.State(P, sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x)
    done = 0
    for n in (1, 10, 100):
        S.step(n - done)
        st.step(n - done)
        done = n
        e = S.export()
        errs = dict(x=scaled(e["pos"], st.x, s["x"]), v=scaled(e["vel"], st.v, s["v"]),
                    p=scaled(sc.c0 ** 2 * (e["rho"] - sc.rho0), sc.c0 ** 2 * (st.rho - sc.rho0), s["p"]),
                    a=scaled(e["acc"], st.a, max(G, np.abs(st.a).max())),
                    pw=scaled(S.export_walls()["pw"], st.pw, s["p"]))
        print(f"  step {n}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        bad = {k: v for k, v in errs.items() if not v <= tol(prec)}
        assert not bad, (n, bad)
    d = S.diag()
    od = st.diag()
    assert d["M"] == pytest.approx(od["M"], rel=1e-12)
    assert d["steps"] == 100
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)


def test_hydrostatic_tank_fp64(solver_mod):
    # 2-D tank at rest (dx = 0.025, H = 1), pre-relaxed by the oracle; 200
    # FP64 GPU steps match 200 oracle steps and keep p within 5 % of
    # rho0 g (H - z).
    sc = scenes.hydrostatic_tank_2d()
    P = O.params_from_scene(sc)
    st = O.State(P, sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x)
    st.step(3000, damp=0.03)
    relaxed = sc.with_params(fluid_x=st.x.copy(), fluid_v=np.zeros_like(st.v), fluid_rho=st.rho.copy())
    ref = O.State(P, relaxed.fluid_x, relaxed.fluid_v, relaxed.fluid_rho, relaxed.wall_x).step(200)
    S = solver_mod.Solver(relaxed, "f64")
    S.step(200)
    e = S.export()
    s = scales(sc)
    assert scaled(e["pos"], ref.x, s["x"]) < 1e-9
    assert scaled(sc.c0 ** 2 * (e["rho"] - sc.rho0), sc.c0 ** 2 * (ref.rho - sc.rho0), s["p"]) < 1e-9
    p = sc.c0 ** 2 * (e["rho"] - sc.rho0)
    pa = sc.rho0 * G * (sc.H - e["pos"][:, 1])
    ep = np.linalg.norm(p - pa) / np.linalg.norm(pa)
    print(f"  e_p = {ep:.4f}", flush=True)
    assert ep < 5e-2


def test_determinism_bitwise(solver_mod):
    sc = SMALL["dam3d"]()
    outs = []
    for _ in range(2):
        S = solver_mod.Solver(sc, "f32")
        S.step(20)
        outs.append((S.export(), S.export_walls(), S.raw()))
    for k in ("pos", "vel", "rho", "acc"):
        assert np.array_equal(outs[0][0][k], outs[1][0][k]), k
    assert np.array_equal(outs[0][1]["pw"], outs[1][1]["pw"])
    assert np.array_equal(outs[0][2]["pid"], outs[1][2]["pid"])


def test_diag_and_probe(solver_mod):
    sc = scenes.dam_break_2d(dx=0.02, steps=50)
    assert len(sc.probe) == 5
    S = solver_mod.Solver(sc, "f64")
    P = O.params_from_scene(sc)
    st = O.State(P, sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x, probe=sc.probe)
    S.step(50)
    st.step(50)
    d, od = S.diag(), st.diag()
    e = S.export()
    od2 = O.diag(P, e["pos"], e["vel"])
    assert d["M"] == pytest.approx(od2["M"], rel=1e-12)
    assert d["Ek"] == pytest.approx(od2["Ek"], rel=1e-12)
    assert d["Ep"] == pytest.approx(od2["Ep"], rel=1e-12)
    assert d["vmax"] == pytest.approx(od2["vmax"], rel=1e-14)
    assert np.allclose(d["P"][:2], od2["P"][:2], rtol=1e-10, atol=1e-12 * od2["M"])
    assert d["J"] == pytest.approx(st.J, rel=1e-9)
    assert st.J > 0


# ---------------------------------------------------------------- edge cases
def test_edge_no_fluid(solver_mod):
    sc = SMALL["dam2d"]()
    sc = sc.with_params(fluid_x=np.zeros((0, 2)), fluid_v=np.zeros((0, 2)), fluid_rho=np.zeros(0))
    S = solver_mod.Solver(sc, "f32")
    S.step(3)
    w = S.export_walls()
    assert np.all(w["pw"] == 0.0)
    assert S.diag()["M"] == 0.0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_edge_free_fall_no_walls(solver_mod, prec):
    # isolated particle: kick-drift-kick integrates g exactly (Sec. 2.6)
    sc = scenes.random_box(dim=3, n=1, seed=3, walls=False)
    x0 = np.array([[0.05, 0.05, 0.6]])
    v0 = np.array([[0.1, -0.2, 0.3]])
    sc = sc.with_params(fluid_x=x0, fluid_v=v0, fluid_rho=np.array([1000.0]), hi=np.array([0.2, 0.2, 0.7]),
                        lo=np.array([-0.1, -0.1, -0.1]))
    S = solver_mod.Solver(sc, prec)
    S.step(100)
    t = 100 * sc.dt
    e = S.export()
    ref = x0 + v0 * t + 0.5 * np.array([0, 0, -G]) * t * t
    tol_x = 1e-12 if prec == "f64" else 2e-6
    assert np.abs(e["pos"] - ref).max() < tol_x
    assert e["rho"][0] == pytest.approx(1000.0, rel=1e-6)


def test_edge_leaving_grid_is_counted(solver_mod):
    sc = scenes.random_box(dim=3, n=1, seed=3, walls=False)
    sc = sc.with_params(fluid_x=np.array([[0.05, 0.05, 0.1]]), fluid_v=np.array([[0.0, 0.0, 5.0]]),
                        fluid_rho=np.array([1000.0]), hi=np.array([0.2, 0.2, 0.12]),
                        lo=np.array([-0.1, -0.1, -0.1]))
    S = solver_mod.Solver(sc, "f32")
    S.step(60)
    st = S.status()
    assert st["out_of_grid"] > 0
    e = S.export()
    assert np.all(e["pos"][:, 2] <= -0.1 + float(S.desc.grid[2]) * float(S.desc.cell))


def test_edge_time_step_above_cfl_rejected(solver_mod):
    from paper_2110_02621_amd.abi import SPHError
    sc = SMALL["box3d"]()
    with pytest.raises(SPHError):
        solver_mod.Solver(sc.with_params(dt=1.02 * sc.dt), "f32")


def test_edge_coincident_particles(solver_mod):
    # two particles at the same point: r = 0 pairs add W(0) to sigma and
    # nothing to the gradient sums (no NaN)
    sc = SMALL["box3d"]()
    x = sc.fluid_x.copy()
    x[1] = x[0]
    sc = sc.with_params(fluid_x=x)
    S = solver_mod.Solver(sc, "f32")
    S.step(2)
    e = S.export()
    assert np.all(np.isfinite(e["acc"])) and np.all(np.isfinite(e["rho"]))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_edge_mask_overflow_walks_the_cells(solver_mod, prec):
    # A clump of 125 particles 0.3 dx apart inside one cell, on the floor of
    # the box: every stencil row through that cell holds more than 128
    # candidates (fluid queries, and the top wall layer's queries over the
    # fluid), so those queries get count -1, are counted in the status and
    # walk the cells in every sweep.  The run must equal, bit for bit, one that
    # walks the cells throughout.
    sc = SMALL["box3d"]()
    g = np.arange(5) * 0.003
    clump = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + np.array([0.0755, 0.0755, 0.002])
    x = np.concatenate([sc.fluid_x, clump])
    v = np.concatenate([sc.fluid_v, np.zeros_like(clump)])
    rho = np.concatenate([sc.fluid_rho, np.full(len(clump), sc.rho0)])
    sc = sc.with_params(fluid_x=x, fluid_v=v, fluid_rho=rho)
    a = solver_mod.Solver(sc, prec, lists=True)
    b = solver_mod.Solver(sc, prec, lists=False)
    # the clump sits inside one cell of the grid
    L, lo = float(a.desc.cell), np.array(list(a.desc.lo))
    cells = np.floor((clump - lo) / L).astype(int)
    assert (cells == cells[0]).all()
    a.step(3)
    b.step(3)
    raw = a.raw()
    assert (raw["cnt_ff"] == -1).any() and (raw["cnt_wf"] == -1).any()
    ea, eb = a.export(), b.export()
    for k in ("pos", "vel", "rho", "acc"):
        assert np.array_equal(ea[k], eb[k]), k
    assert np.array_equal(a.export_walls()["pw"], b.export_walls()["pw"])
    sa, sb = a.status(), b.status()
    assert sa["list_overflow"] > 0 and sb["list_overflow"] == 0
    assert {k: sa[k] for k in ("out_of_grid", "fast", "nonfinite")} == \
        {k: sb[k] for k in ("out_of_grid", "fast", "nonfinite")} == dict(out_of_grid=0, fast=0, nonfinite=0)


# ---------------------------------------------------------------- full size, sampled
FULL = {
    "dam3d_dx0.004": lambda: scenes.dam_break_3d(dx=0.004),
    "dam3d_obst_dx0.0025": lambda: scenes.dam_break_3d(dx=0.0025, obstacles=8, seed=0),
    # the dam break with a wedge at the paper's dx = h_w/40 (5,721,296 particles)
    "wedge3d_res40": lambda: scenes.dam_break_wedge(res=40),
    # the differentiable 2-D dam break at its full size (80,000 + 6,018)
    "dam2d_dx0.005": lambda: scenes.dam_break_2d(dx=0.005),
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled_parity(solver_mod, name):
    # The workloads at full size in the launch configuration the bench
    # times (FP32, sph_step), two steps in; then one step stage by stage,
    # compared on sampled particles that the oracle evaluates one by one.
    sc = FULL[name]()
    print(f"[full] {name} nf={sc.n_fluid} nw={sc.n_wall}", flush=True)
    s = scales(sc)
    S = solver_mod.Solver(sc, "f32")
    S.step(2)
    P = O.params_from_scene(sc)
    rng = np.random.default_rng(5)
    e0, w0 = S.export(), S.export_walls()
    wx, wn = w0["pos"], w0["nrm"]
    near_wall = np.nonzero(e0["pos"][:, sc.dim - 1] < 3 * sc.dx)[0]
    qf = np.unique(np.concatenate([rng.choice(sc.n_fluid, 3000, replace=False),
                                   rng.choice(near_wall, min(1000, len(near_wall)), replace=False)]))
    qw = rng.choice(sc.n_wall, 2000, replace=False)
    # neighbour sets of the sampled particles, bit-exact: the oracle's pair
    # test in the kernel's precision (FP32 cell + offset, as the device holds
    # them) over candidates that the FP64 cell list finds within 2h (1 + 1e-5)
    cnt, off, lst = S.neighbours(0)
    raw = S.raw()
    nf = sc.n_fluid
    inv_f = np.empty(nf, dtype=np.int64)
    inv_f[raw["pid"][0]] = np.arange(nf)
    inv_w = np.empty(sc.n_wall, dtype=np.int64)
    inv_w[raw["wpid"]] = np.arange(sc.n_wall)
    cells = np.concatenate([S.cell_coords(raw["key"][0]), S.cell_coords(raw["wkey"])])
    offs = np.concatenate([raw["off"][0].T, raw["woff"].T]).astype(np.float64)
    sorted_of = lambda ids: np.where(ids < nf, inv_f[np.minimum(ids, nf - 1)],
                                     nf + inv_w[np.maximum(ids - nf, 0)])
    L = float(S.desc.cell)
    rc2 = float(np.float32(4.0 * sc.h * sc.h))
    allx = np.concatenate([e0["pos"], wx])
    ocnt, olst = O.neighbours(sc.dim, sc.h * (1 + 1e-5), e0["pos"][qf], allx)
    oo = np.concatenate([[0], np.cumsum(ocnt)])
    ncand = 0
    for a, i in enumerate(qf):
        cand = olst[oo[a]:oo[a + 1]].astype(np.int64)
        si, sj = sorted_of(np.array([i])), sorted_of(cand)
        hit = O.pairs_bruteforce(sc.dim, True, cells[si], offs[si], cells[sj], offs[sj], L, rc2)[0]
        got = set(lst[off[i]:off[i] + cnt[i]].tolist())
        ref = set(cand[hit.astype(bool)].tolist())
        assert got == ref, (i, sorted(got - ref)[:5], sorted(ref - got)[:5])
        ncand += len(cand)
    print(f"  {len(qf)} sampled neighbour sets bit-exact ({ncand} candidates tested in FP32)", flush=True)
    # density stage
    S.density()
    e_mid = S.export()   # rho: reinitialised, vel: half step (positions still r^n in copy 0)
    sig_o = O.sigma(P, e0["pos"], wx, query=qf)
    rt_o = O.reinit(P, sig_o, e0["rho"][qf])
    errs = dict(p_reinit=scaled(sc.c0 ** 2 * (e_mid["rho"][qf] - rt_o), 0, s["p"]),
                v_half=scaled(e_mid["vel"][qf], e0["vel"][qf] + 0.5 * sc.dt * e0["acc"][qf], s["v"]))
    S.build_cells()
    e1 = S.export()
    errs["x1"] = scaled(e1["pos"][qf], e0["pos"][qf] + sc.dt * e1["vel"][qf], s["x"])
    S.wall_bc()
    pw1 = S.export_walls()["pw"]
    errs["pw"] = scaled(pw1[qw], O.wall_pressure(P, wx, e1["pos"], e1["rho"], query=qw), s["p"])
    S.continuity()
    e2 = S.export()
    D_o = O.continuity(P, e1["pos"], e1["vel"], e1["rho"], wx, pw1, query=qf)
    errs["p_new"] = scaled(sc.c0 ** 2 * (e2["rho"][qf] - (e1["rho"][qf] + sc.dt * D_o)), 0, s["p"])
    S.momentum()
    e3 = S.export()
    A_o = O.momentum(P, e1["pos"], e1["vel"], e2["rho"], wx, pw1, wn, query=qf)
    errs["acc"] = scaled(e3["acc"][qf], A_o, max(G, np.abs(A_o).max()))
    errs["v_new"] = scaled(e3["vel"][qf], e1["vel"][qf] + 0.5 * sc.dt * A_o, s["v"])
    print("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), S.status(), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= TOL32}
    assert not bad, bad
    assert S.status() == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", ["box3d", "dam3d", "dam2d", "wedge3d"])
def test_lists_and_cell_walk_agree_bitwise(solver_mod, name, prec):
    # The sweeps read neighbour masks when present and walk the cells
    # otherwise: same pairs, same order, same arithmetic, same bits.
    sc = SMALL[name]()
    a = solver_mod.Solver(sc, prec, lists=True)
    b = solver_mod.Solver(sc, prec, lists=False)
    a.step(10)
    b.step(10)
    ea, eb = a.export(), b.export()
    for k in ("pos", "vel", "rho", "acc"):
        assert np.array_equal(ea[k], eb[k]), k
    assert np.array_equal(a.export_walls()["pw"], b.export_walls()["pw"])
    st = a.status()
    assert st["list_overflow"] == 0
    raw = a.raw()
    assert raw["cnt_ff"].min() >= 1      # itself at least; -1 would mark an overflow
    # the masks hold exactly the pairs the cell walk finds
    cnt, _, _ = a.neighbours(0)
    nfl = np.empty_like(raw["cnt_ff"])
    nfl[raw["pid"][0]] = raw["cnt_ff"] + raw["cnt_fw"]
    assert np.array_equal(cnt, nfl)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", ["box3d", "dam3d", "dam2d"])
def test_sigma_from_momentum_sweep_is_bitwise_the_gathered_sum(solver_mod, name, prec):
    # The momentum sweep sums sigma at the positions the next density update
    # starts from; the update must give the same bits as its own neighbour sum.
    from paper_2110_02621_amd import adjoint
    sc = SMALL[name]()
    S = solver_mod.Solver(sc, prec, keep_sigma=True)
    S.step(5)
    assert S.buf.sigma_ready == 1
    st = adjoint.save_state(S)
    S.density()                      # sigma handed over by the momentum sweep
    fused = S.raw()
    adjoint.load_state(S, st)        # clears sigma_ready: this density sums itself
    assert S.buf.sigma_ready == 0
    S.density()
    gathered = S.raw()
    assert np.array_equal(fused["sigma"], gathered["sigma"])
    for k in ("key", "pid", "off", "vel", "rho"):
        assert np.array_equal(fused[k], gathered[k]), k
