#!/usr/bin/env python3
"""Throughput of the WCSPH step on one MI355X: particle-steps/s of the 3-D
dam break with seeded obstacles (dx = 0.0025 m: 6.91M fluid + 1.90M wall
dummy particles), FP32, with the FP64 build of the same kernels timed
beside it and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  One step = density/reinit + kick/drift, cell sort,
wall pressure, continuity, momentum + kick: every row of the hot path.
Inputs are resident in HBM before the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (3-D dam break, 4M particles, FP32 vs FP64) + adjoint/fwd ratio"

# Useful (algorithmic) flops per interacting pair of each sweep in 3-D,
# counted operation by operation from the kernels' formulas (distance from
# cell + offset, kernel value or gradient, Riemann terms, accumulation);
# square root, reciprocal and reciprocal square root count as one each.
# Culled candidates (r >= 2h) are not counted.
FLOPS_PAIR = {
    "wall_bc": 33,        # sum W, sum p W, sum rho r W
    "continuity_ff": 39,  # Eq. (9) with the Riemann intermediate velocity
    "continuity_fw": 36,
    "momentum_ff": 68,    # Eq. (10) with p* of Eq. (8), viscous term
    "momentum_fw": 64,    # Eq. (11) p*, viscous, penalty test
    "momentum_sigma": 14,  # sigma += W(r) (compensated) for the next step, every pair incl. self
}
# Compulsory HBM bytes per fluid particle in FP32 of the cell sort
# (histogram 16, placement 16, in-cell ordering 8, gather 76) and per cell
# (count fill, scan read/write, cell table reads); of the density update
# (reads sigma, rho, v, dv/dt, offset, key, id: 52; writes rho, v, offset,
# key, id: 36).
SORT_BYTES_PARTICLE = 116
SORT_BYTES_CELL = 24
DENSITY_BYTES_PARTICLE = 88
# Compulsory HBM bytes (lower bounds, FP32, 3-D, every record read once)
# per fluid particle of the mask builder (reads offset record, key: 20;
# writes nine row words, two counts: 80), the continuity sweep (reads both
# records, key, count, nine row words: 112; writes the density and its
# record: 20) and the momentum sweep (the same reads: 112; writes dv/dt,
# velocity, its record, sigma: 44), and per wall particle of the wall
# pressure (key, record, count; writes p_w and the record: 44).  Second
# mask words and the fluid-wall rows are left out.
MASKS_BYTES_PARTICLE = 100
CONTINUITY_BYTES_PARTICLE = 132
MOMENTUM_BYTES_PARTICLE = 156
WALL_BC_BYTES_WALL = 44

# HBM bytes per launch of the two pair sweeps on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE scaled by 2.000 and WRITE_SIZE by 1.000,
# the factors a plain 1 GiB device copy gives): see
# profiles/kernels_dam_break_3d_dx0.0025_8obstacles_hbm.md.  They describe the
# kernel sources whose SHA-256 is recorded; once those change the traffic is
# reported as null until the counters are taken again.
TRAFFIC = {
    "sources_sha256": "9c77df0ca1b11de43dfb432510bc2795f871af7361802282fa9fac67fbc1f305",
    "momentum": 2085.0e6 + 269.6e6,
    "continuity": 2148.3e6 + 139.9e6,
}
KERNEL_SOURCES = ("sph_kernels.hip", "sph_device.h", "sph_host.h")

PEAK_FP32 = 157.3e12      # MI355X published FP32 vector peak (packed FMA)
PEAK_FP32_UNPACKED = 78.6e12  # 256 CU x 64 lanes x 2 flop x 2.4 GHz, one FMA per lane per clock
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dx", type=float, default=0.0025, help="particle spacing of the dam break")
    ap.add_argument("--obstacles", type=int, default=8)
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: --steps)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-4m", action="store_true", help="skip the dx = 0.003 m (4M fluid) point")
    ap.add_argument("--no-two-phase", action="store_true", help="skip the two-phase dam break point")
    ap.add_argument("--no-sloshing", action="store_true", help="skip the shaken two-phase tank points")
    ap.add_argument("--no-wedge", action="store_true", help="skip the dam break with a wedge point")
    ap.add_argument("--adjoint-only", action="store_true", help="time only the adjoint/forward ratio")
    ap.add_argument("--sloshing-only", type=float, default=None, metavar="DX",
                    help="time only the shaken two-phase tank at this dx (kernel profiles of that case)")
    ap.add_argument("--large-only", type=float, default=None, metavar="DX",
                    help="time only the dam break with obstacles at this (small) dx: throughput and device "
                         "memory of a large problem")
    ap.add_argument("--penalty-off", action="store_true",
                    help="the single-phase workloads without the wall penalty (the paper applies it to the light "
                         "phase only): the cost of that term")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle steps of the CPU baseline (about 3 s each)")
    ap.add_argument("--cpu-stride", type=int, default=16,
                    help="every n-th particle in the one-thread oracle sample")
    ap.add_argument("--cpu-sample-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward timing")
    ap.add_argument("--adj-steps", type=int, default=1000, help="steps of the differentiable 2-D dam break")
    ap.add_argument("--adj-dx", type=float, default=0.005)
    ap.add_argument("--adj-K", type=int, default=50, help="checkpoint interval of the adjoint")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also run one plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


def timed_run(solver_mod, scene, precision, steps, warmup):
    """Warm up, then time `steps` steps stage by stage with events on the
    stream the kernels run on.  Returns wall seconds and mean ms per stage."""
    import torch
    S = solver_mod.Solver(scene, precision)
    S.step(warmup)
    torch.cuda.synchronize()
    names = ["density", "sort", "wall_bc", "continuity", "momentum"]
    calls = [S.density, S.build_cells, S.wall_bc, S.continuity, S.momentum]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        e = ev[k]
        e[0].record()
        for j, fn in enumerate(calls):
            fn()
            e[j + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = {n: sum(ev[k][j].elapsed_time(ev[k][j + 1]) for k in range(steps)) / steps
                for j, n in enumerate(names)}
    return S, wall, stage_ms


def measured_traffic(kernel):
    """Counter-measured HBM bytes of `kernel` per launch, or None when the
    kernel sources differ from the ones the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2110_02621_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sources_sha256"]:
        return None
    return TRAFFIC.get(kernel)


def adjoint_timing(scenes, args, precision):
    """J, dJ/dtheta and the forward and backward times of the differentiable
    2-D dam break with a `precision` forward (after a short warm-up run)."""
    from paper_2110_02621_amd import adjoint
    sc4 = scenes.dam_break_2d(dx=args.adj_dx, steps=args.adj_steps)
    adjoint.probe_gradient(scenes.dam_break_2d(dx=args.adj_dx, steps=2 * args.adj_K),
                           precision=precision, K=args.adj_K)  # warm-up (kernels, allocator)
    r = adjoint.probe_gradient(sc4, precision=precision, K=args.adj_K, return_timings=True)
    return dict(workload=f"2-D dam break dx={args.adj_dx} m ({sc4.n_fluid} fluid + {sc4.n_wall} wall), "
                         f"{args.adj_steps} steps, checkpoint every {args.adj_K}",
                t_forward_s=r["t_forward"], t_backward_s=r["t_backward"],
                ratio=r["t_backward"] / r["t_forward"], J=r["J"], grad=r["grad"])


def copy_rate(torch, gib=2.0, reps=10):
    """Bytes read plus written per second of a plain device-to-device copy
    of `gib` GiB (the HBM rate a streaming kernel reaches in practice)."""
    a = torch.ones(int(gib * 2 ** 30) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    rate = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return rate


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), as lscpu reports it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_stage_sample(dx, obstacles, stride):
    """Seconds the FP64 oracle takes for the pair sums of one step (number
    density, wall pressure, continuity, momentum) of every stride-th fluid
    and wall particle of the benchmark workload, from its initial state.
    Run in a child process whose OpenMP thread count is fixed by its
    environment; prints one JSON line."""
    import numpy as np
    import oracle
    from paper_2110_02621_amd import scenes
    sc = scenes.dam_break_3d(dx=dx, obstacles=obstacles, seed=0)
    P = oracle.params_from_scene(sc)
    q = np.arange(0, sc.n_fluid, stride)
    qw = np.arange(0, sc.n_wall, stride)
    pw = np.zeros(sc.n_wall)
    wn = np.zeros((sc.n_wall, 3))
    t0 = time.perf_counter()
    oracle.sigma(P, sc.fluid_x, sc.wall_x, query=q)
    oracle.wall_pressure(P, sc.wall_x, sc.fluid_x, sc.fluid_rho, query=qw)
    oracle.continuity(P, sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x, pw, query=q)
    oracle.momentum(P, sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x, pw, wn, query=q)
    t = time.perf_counter() - t0
    print(json.dumps(dict(seconds=t, particles=int(len(q) + len(qw)), threads=oracle.num_threads())), flush=True)


def cpu_sample_in_child(args, threads):
    """cpu_stage_sample in a child process with OMP_NUM_THREADS = threads."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample-child", "--dx", str(args.dx),
           "--obstacles", str(args.obstacles), "--cpu-stride", str(args.cpu_stride)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"CPU sample child failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def pair_counts(S):
    """Interacting pairs of the current state: fluid-fluid (self excluded),
    fluid-wall, wall-fluid, and fluid-(fluid+wall) with self."""
    c = S.pair_counts()
    nf = S.scene.n_fluid
    return dict(ff=c["ff_with_self"] - nf, fw=c["fw"], wf=c["wf"],
                all_with_self=c["ff_with_self"] + c["fw"], max_ff=c["max_ff"])


def main():
    args = parse()
    if args.cpu_sample_child:  # the oracle's timed sample, in a child process (no GPU)
        cpu_stage_sample(args.dx, args.obstacles, args.cpu_stride)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the hot path here is "
              "the single-GPU sweep; multi-GPU sharding is design-only.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2110_02621_amd import scenes, solver

    if args.adjoint_only:
        adj = adjoint_timing(scenes, args, "f32")
        adj["f64"] = adjoint_timing(scenes, args, "f64")
        adj["f64"].pop("workload")
        print(json.dumps(adj), flush=True)
        return

    if args.sloshing_only:
        scs = scenes.sloshing_tank(dim=3, dx=args.sloshing_only, steps=args.steps)
        Ss, walls_, stages = timed_run(solver, scs, "f32", args.steps, args.warmup)
        ns = scs.n_fluid + scs.n_wall
        print(json.dumps(dict(workload=f"3-D two-phase sloshing tank, dx={args.sloshing_only} m: {scs.n_heavy} water "
                                       f"+ {scs.n_fluid - scs.n_heavy} air + {scs.n_wall} wall",
                              value=ns * args.steps / walls_, unit="particle-steps/s",
                              ms_per_step=1e3 * walls_ / args.steps, steps=args.steps,
                              stage_ms={k: round(v, 4) for k, v in stages.items()}, status=Ss.status())),
              flush=True)
        return

    if args.large_only:
        t0 = time.perf_counter()
        scl = scenes.dam_break_3d(dx=args.large_only, obstacles=args.obstacles, seed=0, steps=args.steps)
        t_scene = time.perf_counter() - t0
        print(f"[bench] large: {scl.n_fluid} fluid + {scl.n_wall} wall (scene {t_scene:.0f} s)", file=sys.stderr,
              flush=True)
        torch.cuda.reset_peak_memory_stats()
        Sl, walll, stages = timed_run(solver, scl, "f32", args.steps, args.warmup)
        nl = scl.n_fluid + scl.n_wall
        print(json.dumps(dict(workload=f"3-D dam break with {args.obstacles} seeded obstacles, dx={args.large_only} m: "
                                       f"{scl.n_fluid} fluid + {scl.n_wall} wall",
                              value=nl * args.steps / walll, unit="particle-steps/s",
                              ms_per_step=1e3 * walll / args.steps, steps=args.steps,
                              stage_ms={k: round(v, 4) for k, v in stages.items()}, status=Sl.status(),
                              device_gib=round(torch.cuda.max_memory_allocated() / 2 ** 30, 2),
                              bytes_per_particle=round(torch.cuda.max_memory_allocated() / nl, 1))),
              flush=True)
        return

    sc = scenes.dam_break_3d(dx=args.dx, obstacles=args.obstacles, seed=0, steps=args.steps)
    if args.penalty_off:
        sc = sc.with_params(penalty_all=False)
    nf, nw = sc.n_fluid, sc.n_wall
    n_tot = nf + nw
    print(f"[bench] workload dam_break_3d dx={args.dx} obstacles={args.obstacles}: "
          f"{nf} fluid + {nw} wall", file=sys.stderr, flush=True)

    S, wall, stage = timed_run(solver, sc, "f32", args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    value = n_tot * args.steps / wall
    st = S.status()
    pc = pair_counts(S)
    print(f"[bench] f32 {ms_step:.3f} ms/step  stages {stage}  pairs {pc}  status {st}",
          file=sys.stderr, flush=True)

    flops = {
        "wall_bc": FLOPS_PAIR["wall_bc"] * pc["wf"],
        "continuity": FLOPS_PAIR["continuity_ff"] * pc["ff"] + FLOPS_PAIR["continuity_fw"] * pc["fw"],
        "momentum": (FLOPS_PAIR["momentum_ff"] * pc["ff"] + FLOPS_PAIR["momentum_fw"] * pc["fw"]
                     + FLOPS_PAIR["momentum_sigma"] * pc["all_with_self"]),
    }
    kernels = {}
    for k, f in flops.items():
        t = stage[k] * 1e-3
        kernels[k] = dict(ms=round(stage[k], 4), tflops=round(f / t / 1e12, 3),
                          alu_frac=round(f / t / PEAK_FP32, 4))
        # the pair sweeps' HBM side: counter-measured bytes per launch over
        # the launch's duration, and per interacting fluid pair
        traffic = measured_traffic(k)
        if traffic is not None:
            kernels[k].update(hbm_gbps=round(traffic / t / 1e9, 1), hbm_frac=round(traffic / t / PEAK_HBM, 4),
                              hbm_bytes_per_pair=round(traffic / (pc["ff"] + pc["fw"]), 2))
    dens_bytes = DENSITY_BYTES_PARTICLE * nf
    kernels["density"] = dict(ms=round(stage["density"], 4),
                              gbps=round(dens_bytes / (stage["density"] * 1e-3) / 1e9, 1),
                              hbm_frac=round(dens_bytes / (stage["density"] * 1e-3) / PEAK_HBM, 4))
    # the cell stage is the counting sort plus the neighbour-mask build;
    # the bytes below are the sort's alone (the mask build culls candidates)
    sort_bytes = SORT_BYTES_PARTICLE * nf + SORT_BYTES_CELL * int(S.desc.n_cells)
    kernels["cells"] = dict(ms=round(stage["sort"], 4),
                            sort_gbps_lower_bound=round(sort_bytes / (stage["sort"] * 1e-3) / 1e9, 1))
    # compulsory bytes per stage and per step against the published peak and
    # the measured copy rate
    alg = {"density": dens_bytes, "sort": sort_bytes + MASKS_BYTES_PARTICLE * nf,
           "wall_bc": WALL_BC_BYTES_WALL * nw, "continuity": CONTINUITY_BYTES_PARTICLE * nf,
           "momentum": MOMENTUM_BYTES_PARTICLE * nf}
    copy_bw = copy_rate(torch)
    step_hbm = dict(compulsory_bytes=sum(alg.values()), copy_gbps=round(copy_bw / 1e9, 1))
    t_stages = sum(stage.values()) * 1e-3
    step_hbm.update(gbps=round(step_hbm["compulsory_bytes"] / t_stages / 1e9, 1),
                    hbm_frac=round(step_hbm["compulsory_bytes"] / t_stages / PEAK_HBM, 4),
                    copy_frac=round(step_hbm["compulsory_bytes"] / t_stages / copy_bw, 4),
                    by_stage={k: dict(bytes=v, gbps=round(v / (stage[k] * 1e-3) / 1e9, 1),
                                      hbm_frac=round(v / (stage[k] * 1e-3) / PEAK_HBM, 4),
                                      copy_frac=round(v / (stage[k] * 1e-3) / copy_bw, 4))
                              for k, v in alg.items()})
    dom = max(("continuity", "momentum"), key=lambda k: stage[k])
    ach = flops[dom] / (stage[dom] * 1e-3)
    roofline = dict(bound="alu", achieved=round(ach / 1e12, 3), peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                    frac=round(ach / PEAK_FP32, 4), traffic=measured_traffic(dom), kernel=dom)
    del S
    torch.cuda.empty_cache()

    # the same dam break at dx = 0.003 m: exactly 4,000,000 fluid particles
    m4 = None
    if not args.no_4m:
        sc4m = scenes.dam_break_3d(dx=0.003, obstacles=args.obstacles, seed=0, steps=args.steps)
        k4 = max(10, args.steps // 2)
        S4, wall4, _ = timed_run(solver, sc4m, "f32", k4, max(2, args.warmup // 2))
        m4 = dict(workload=f"3-D dam break with {args.obstacles} seeded obstacles, dx=0.003 m, "
                           f"{sc4m.n_fluid} fluid + {sc4m.n_wall} wall",
                  value=(sc4m.n_fluid + sc4m.n_wall) * k4 / wall4, ms_per_step=1e3 * wall4 / k4, steps=k4,
                  status=S4.status())
        print(f"[bench] 4M f32 {m4['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        del S4
        torch.cuda.empty_cache()

    # two-phase dam break: water column + air in the rest of the closed tank
    tp = None
    if not args.no_two_phase:
        sct = scenes.dam_break_3d_two_phase(dx=0.005, steps=args.steps)
        kt = max(10, args.steps // 2)
        St, wallt, staget = timed_run(solver, sct, "f32", kt, max(2, args.warmup // 2))
        nt = sct.n_fluid + sct.n_wall
        tp = dict(workload=f"3-D two-phase dam break dx=0.005 m: {sct.n_heavy} water + "
                           f"{sct.n_fluid - sct.n_heavy} air + {sct.n_wall} wall, rho 1000/1, one c0",
                  value=nt * kt / wallt, ms_per_step=1e3 * wallt / kt, steps=kt,
                  stage_ms={k: round(v, 4) for k, v in staget.items()}, status=St.status())
        print(f"[bench] two-phase f32 {tp['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        del St
        torch.cuda.empty_cache()

    # the shaken two-phase tank of Sec. 4.4 (moving walls, X(t) = A0 sin(2 pi f0 t)):
    # 243,432 particles at dx = 0.01 (the paper's kernel-profile case) and
    # 1,410,752 at dx = 0.005 (its sloshing run)
    slosh = None
    if not args.no_sloshing:
        slosh = []
        for dxs in (0.01, 0.005):
            scs = scenes.sloshing_tank(dim=3, dx=dxs, steps=args.steps)
            ks = max(10, args.steps // 2)
            Ss, walls_, stages = timed_run(solver, scs, "f32", ks, max(2, args.warmup // 2))
            ns = scs.n_fluid + scs.n_wall
            slosh.append(dict(workload=f"3-D two-phase sloshing tank 1.3 x 0.1 x 0.9 m, dx={dxs} m: "
                                       f"{scs.n_heavy} water + {scs.n_fluid - scs.n_heavy} air + "
                                       f"{scs.n_wall} wall, A0={scs.motion_amp[0]} m, f0={scs.motion_freq} Hz",
                              value=ns * ks / walls_, ms_per_step=1e3 * walls_ / ks, steps=ks,
                              stage_ms={k: round(v, 4) for k, v in stages.items()}, status=Ss.status()))
            print(f"[bench] sloshing dx={dxs} f32 {slosh[-1]['ms_per_step']:.3f} ms/step",
                  file=sys.stderr, flush=True)
            del Ss
            torch.cuda.empty_cache()

    # dam break with a wedge (Sec. 4.5) at the paper's dx = h_w/40: 5,721,296
    # particles (the paper's run: 5,734,250)
    wedge = None
    if not args.no_wedge:
        scw = scenes.dam_break_wedge(res=40, steps=args.steps)
        kw = max(10, args.steps // 2)
        Sw, wallw, stagew = timed_run(solver, scw, "f32", kw, max(2, args.warmup // 2))
        nwt = scw.n_fluid + scw.n_wall
        wedge = dict(workload=f"3-D dam break with a pi/3 wedge, h_w = 5.5 m, dx = h_w/40: {scw.n_fluid} fluid + "
                              f"{scw.n_wall} wall ({scw.meta['n_wedge_wall']} on the wedge)",
                     value=nwt * kw / wallw, ms_per_step=1e3 * wallw / kw, steps=kw,
                     stage_ms={k: round(v, 4) for k, v in stagew.items()}, status=Sw.status())
        print(f"[bench] wedge f32 {wedge['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        del Sw
        torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        k64 = args.fp64_steps or args.steps
        S64, wall64, stage64 = timed_run(solver, sc, "f64", k64, max(2, args.warmup // 2))
        fp64 = dict(value=n_tot * k64 / wall64, ms_per_step=1e3 * wall64 / k64, steps=k64,
                    stage_ms={k: round(v, 4) for k, v in stage64.items()})
        print(f"[bench] f64 {fp64['ms_per_step']:.3f} ms/step stages {stage64}", file=sys.stderr, flush=True)
        del S64
        torch.cuda.empty_cache()

    adj = None
    if not args.no_adjoint:
        adj = adjoint_timing(scenes, args, "f32")
        print(f"[bench] adjoint fwd {adj['t_forward_s']:.3f} s bwd {adj['t_backward_s']:.3f} s grad {adj['grad']}",
              file=sys.stderr, flush=True)
        # the same with an FP64 forward (its gradient agrees with FP64 central
        # differences to ~3e-5 at this size, the FP32 one to ~1e-3)
        adj["f64"] = adjoint_timing(scenes, args, "f64")
        adj["f64"].pop("workload")
        adj["ratio_note"] = ("ratio: FP32 forward and its FP64-accumulated backward (incl. recompute) over that "
                             "forward; f64.ratio: the FP64 adjoint over its own forward; adjoint_fwd_ratio: the "
                             "FP64 adjoint's backward over the FP32 forward")
        print(f"[bench] adjoint f64 fwd {adj['f64']['t_forward_s']:.3f} s bwd {adj['f64']['t_backward_s']:.3f} s",
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    if args.copy_gib > 0:
        n = int(args.copy_gib * 2 ** 30 // 4)
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu:
        import oracle
        P = oracle.params_from_scene(sc)
        t0 = time.perf_counter()
        ost = oracle.State(P, sc.fluid_x, sc.fluid_v, sc.fluid_rho, sc.wall_x)
        tinit = time.perf_counter() - t0
        t0 = time.perf_counter()
        ost.step(args.cpu_steps)
        tcpu = time.perf_counter() - t0
        cpu = dict(value=n_tot * args.cpu_steps / tcpu, unit="particle-steps/s", cores=oracle.num_threads(),
                   kind="oracle",
                   sample=f"{args.cpu_steps} FP64 oracle step(s) of the full workload "
                          f"({n_tot} particles), {tcpu:.1f} s (+{tinit:.1f} s initialisation, untimed)",
                   cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                   host_cpus_usable=len(os.sched_getaffinity(0)))
        print(f"[bench] cpu oracle {tcpu:.1f} s for {args.cpu_steps} step(s)", file=sys.stderr, flush=True)
        # the pair sums of one step on every stride-th particle, with one
        # thread and with all of them (child processes)
        one = cpu_sample_in_child(args, 1)
        allt = cpu_sample_in_child(args, oracle.num_threads())
        cpu["one_thread"] = dict(
            value=one["particles"] / one["seconds"], unit="particle-steps/s", threads=one["threads"],
            sample=f"FP64 oracle pair sums of one step (number density, wall pressure, continuity, momentum) "
                   f"on every {args.cpu_stride}th particle ({one['particles']} particles) of the same workload, "
                   f"{one['seconds']:.1f} s; the same sample with {allt['threads']} threads: "
                   f"{allt['seconds']:.2f} s ({one['seconds'] / allt['seconds']:.1f}x)")
        print(f"[bench] cpu oracle sample: 1 thread {one['seconds']:.2f} s, {allt['threads']} threads "
              f"{allt['seconds']:.2f} s", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3-D dam break with {args.obstacles} seeded obstacles, dx={args.dx} m, "
                               f"{nf} fluid + {nw} wall dummy particles",
                   "n_fluid": nf, "n_wall": nw, "dx": args.dx, "obstacles": args.obstacles,
                   "wall_penalty": not args.penalty_off, "parallelism": "single GPU"},
        "fluid_particle_steps_per_s": nf * args.steps / wall,
        "fp32_4M": m4,
        "fp32_two_phase": tp,
        "fp32_sloshing": slosh,
        "fp32_wedge": wedge,
        "fp64": fp64,
        "fp32_over_fp64": (value / fp64["value"]) if fp64 else None,
        # the gradient that meets 1e-3 on every component (FP64 forward and
        # backward) against the production FP32 forward of the same run
        "adjoint_fwd_ratio": (adj["f64"]["t_backward_s"] / adj["t_forward_s"]) if adj else None,
        "adjoint": adj,
        "roofline": roofline,
        "roofline_frac_unpacked_fp32": round(ach / PEAK_FP32_UNPACKED, 4),
        "step_hbm": step_hbm,
        "kernels": kernels,
        "pairs": pc,
        "status": st,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
