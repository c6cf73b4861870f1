"""Reverse-through-time derivatives of the wall-probe functional

    J = sum over steps n of dt * mean(p_w^n over the probe walls)

with respect to theta = (mu, gamma_p, c0, H) on the GPU.  The forward runs
the C-ABI step with checkpoints every K steps; the backward restores each
checkpoint in reverse, recomputes its K steps (bit for bit: same kernels,
same inputs) keeping one frame per step, and runs the hand-written backward
kernels (``sph_step_bwd``), ending with the initial state
(``sph_init_bwd``).  ``ProbeFunctional`` wraps both as a
``torch.autograd.Function`` of theta.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import abi, scenes
from .abi import check
from .solver import Solver, _p

THETA_NAMES = ("mu", "gamma_p", "c0", "H")


class Frame(C.Structure):
    _fields_ = [("key", C.c_void_p), ("pid", C.c_void_p), ("off", C.c_void_p), ("fstart", C.c_void_p),
                ("rho", C.c_void_p), ("sigma", C.c_void_p), ("vh", C.c_void_p), ("rt", C.c_void_p),
                ("pw", C.c_void_p),
                ("nbr_ff", C.c_void_p), ("nbr_fw", C.c_void_p), ("nbr_wf", C.c_void_p),
                ("cnt_ff", C.c_void_p), ("cnt_fw", C.c_void_p), ("cnt_wf", C.c_void_p),
                ("nstep", C.c_int64)]


class Adjoint(C.Structure):
    _fields_ = [("xb", C.c_void_p), ("vb", C.c_void_p), ("rhob", C.c_void_p), ("ab", C.c_void_p),
                ("theta", C.c_void_p), ("work", C.c_void_p), ("work_bytes", C.c_size_t)]


def _declare(L):
    if getattr(L, "_adjoint_declared", False):
        return
    dp, bp = C.POINTER(abi.Desc), C.POINTER(abi.Buffers)
    fp, ap = C.POINTER(Frame), C.POINTER(Adjoint)
    vp = C.c_void_p
    L.sph_adjoint_work_bytes.argtypes = [dp, C.c_int64, C.c_int64]
    L.sph_adjoint_work_bytes.restype = C.c_size_t
    L.sph_adjoint_zero.argtypes = [dp, bp, ap, vp]
    for name in ("sph_forces_bwd", "sph_wall_bc_bwd", "sph_density_bwd"):
        getattr(L, name).argtypes = [dp, bp, fp, ap, vp]
    L.sph_step_bwd.argtypes = [dp, bp, fp, fp, ap, vp]
    L.sph_step_frame.argtypes = [dp, bp, vp, fp, vp]
    L.sph_step_frame.restype = C.c_int
    L.sph_init_bwd.argtypes = [dp, bp, fp, C.c_double, ap, vp]
    for name in ("sph_adjoint_zero", "sph_forces_bwd", "sph_wall_bc_bwd", "sph_density_bwd",
                 "sph_step_bwd", "sph_init_bwd"):
        getattr(L, name).restype = C.c_int
    L._adjoint_declared = True


def _cur(S):
    """Views of the solver's current sorted state and fields."""
    t, b = S.t, S.buf
    return dict(key=t["key"][0], pid=t["pid"][0], off=t["off"][0], fstart=t["fstart"],
                vel=t["vel"][b.sel_vel], rho=t["rho"][b.sel_rho], acc=t["acc"], pw=t["pw"])


def save_state(S):
    """Everything needed to resume the forward from here (device copies)."""
    c = _cur(S)
    st = {k: c[k].clone() for k in ("key", "pid", "off", "fstart", "vel", "rho", "acc", "pw")}
    for k in ("nbr_ff", "nbr_fw", "nbr_wf", "cnt_ff", "cnt_fw", "cnt_wf"):
        st[k] = S.t[k].clone()
    st["nstep"] = int(S.buf.nstep)
    return st


def load_state(S, st):
    c = _cur(S)
    for k in ("key", "pid", "off", "fstart", "vel", "rho", "acc", "pw"):
        c[k].copy_(st[k])
    for k in ("nbr_ff", "nbr_fw", "nbr_wf", "cnt_ff", "cnt_fw", "cnt_wf"):
        S.t[k].copy_(st[k])
    S.buf.sigma_ready = 0  # the stored sigma belongs to the overwritten state
    S.buf.nstep = st["nstep"]


MASKS = ("nbr_ff", "nbr_fw", "nbr_wf", "cnt_ff", "cnt_fw", "cnt_wf")


class FramePool:
    """Device storage for the frames of one segment (reused by every
    segment): frame k holds the state at the segment's step k."""

    def __init__(self, S, nframes):
        t = S.t
        self.frames = []
        for k in range(nframes):
            f = {"sigma": torch.empty_like(t["rho"][0])}
            if k > 0:
                for name, src in (("key", t["key"][0]), ("pid", t["pid"][0]), ("off", t["off"][0]),
                                  ("fstart", t["fstart"]), ("vh", t["vel"][0]), ("rt", t["rho"][0]),
                                  ("rho", t["rho"][0]), ("pw", t["pw"])):
                    f[name] = torch.empty_like(src)
                for name in MASKS:
                    f[name] = torch.empty_like(t[name])
            self.frames.append(f)

    @staticmethod
    def struct(f):
        fr = Frame()
        for name, _ in Frame._fields_:
            if name == "nstep":
                fr.nstep = int(f.get("nstep", 0))
                continue
            v = f.get(name)
            setattr(fr, name, (_p(v).value or None) if v is not None else None)
        return fr


def recompute_segment(S, pool, start_state, nsteps, first_frame_extra=None):
    """Restore `start_state` and rerun nsteps steps, recording frames
    0..nsteps into the pool (frame 0 refers to the checkpoint's arrays)."""
    L = S.lib
    load_state(S, start_state)
    f0 = pool.frames[0]
    for k in ("key", "pid", "off", "fstart", "rho") + MASKS:
        f0[k] = start_state[k]
    f0.pop("vh", None)
    f0.pop("pw", None)
    f0["nstep"] = start_state["nstep"]
    if first_frame_extra:
        f0.update(first_frame_extra)
    stream = S._stream()
    for n in range(nsteps):
        nxt = FramePool.struct(pool.frames[n + 1])
        check(L.sph_step_frame(C.byref(S.desc), C.byref(S.buf), _p(pool.frames[n]["sigma"]),
                               C.byref(nxt), stream), "sph_step_frame")
        pool.frames[n + 1]["nstep"] = nxt.nstep
    return [FramePool.struct(f) for f in pool.frames[:nsteps + 1]]


class Tape:
    """What the forward leaves for the backward: the solver (walls, probe,
    buffers), the checkpoints (state every K steps, device copies), the
    initial half-step velocity and wall pressure, and J."""

    def __init__(self, S, scene, K, steps, ckpts, init_extra, J):
        self.S, self.scene, self.K, self.steps = S, scene, K, steps
        self.ckpts, self.init_extra, self.J = ckpts, init_extra, J


def forward(scene, precision="f32", K=50, steps=None, device="cuda") -> Tape:
    """Run `steps` steps (default scene.steps) of `scene`, keeping a
    checkpoint every K steps; J is read at the end."""
    steps = scene.steps if steps is None else steps
    S = Solver(scene, precision, device=device, probe=True, keep_sigma=True)
    _declare(S.lib)
    init_extra = dict(vh=_cur(S)["vel"].clone(), pw=S.t["pw"].clone())
    ckpts = []
    done = 0
    while done < steps:
        ckpts.append((done, save_state(S)))
        k = min(K, steps - done)
        S.step(k)
        done += k
    J = S.diag()["J"]
    return Tape(S, scene, K, steps, ckpts, init_extra, J)


def backward(tape: Tape):
    """dJ/dtheta (float64 device tensor [mu, gamma_p, c0, H]) from a tape:
    every segment, last first, is recomputed from its checkpoint with its
    frames recorded and then stepped backward; the initial state last."""
    S, scene, K, steps = tape.S, tape.scene, tape.K, tape.steps
    L = S.lib
    nf, nw, dim = scene.n_fluid, scene.n_wall, scene.dim
    f64 = dict(dtype=torch.float64, device=S.device)
    A = {k: torch.zeros((dim, nf) if k != "rhob" else (nf,), **f64) for k in ("xb", "vb", "rhob", "ab")}
    theta = torch.zeros(4, **f64)
    wb = int(L.sph_adjoint_work_bytes(C.byref(S.desc), nf, nw))
    work = torch.zeros(wb + 256, dtype=torch.uint8, device=S.device)
    adj = Adjoint()
    adj.xb, adj.vb, adj.rhob, adj.ab = (_p(A[k]).value for k in ("xb", "vb", "rhob", "ab"))
    adj.theta = _p(theta).value
    adj.work = (work.data_ptr() + 255) & ~255
    adj.work_bytes = wb
    stream = S._stream()
    pool = FramePool(S, min(K, steps) + 1)
    check(L.sph_adjoint_zero(C.byref(S.desc), C.byref(S.buf), C.byref(adj), stream), "sph_adjoint_zero")
    for seg in reversed(range(len(tape.ckpts))):
        start, st = tape.ckpts[seg]
        k = min(K, steps - start)
        structs = recompute_segment(S, pool, st, k, tape.init_extra if start == 0 else None)
        for n in reversed(range(k)):
            check(L.sph_step_bwd(C.byref(S.desc), C.byref(S.buf), C.byref(structs[n]),
                                 C.byref(structs[n + 1]), C.byref(adj), stream), "sph_step_bwd")
        if start == 0:
            check(L.sph_init_bwd(C.byref(S.desc), C.byref(S.buf), C.byref(structs[0]), float(scene.H),
                                 C.byref(adj), stream), "sph_init_bwd")
    return theta


def probe_gradient(scene, precision="f32", K=50, steps=None, device="cuda", return_timings=False):
    """J and dJ/dtheta for theta = (mu, gamma_p, c0, H) of `scene` over
    `steps` steps (default scene.steps), checkpoints every K steps."""
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tape = forward(scene, precision, K, steps, device)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t1 = time.perf_counter()
    theta = backward(tape)
    grad = theta.cpu().numpy().copy()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t1
    out = dict(J=tape.J, grad=dict(zip(THETA_NAMES, grad.tolist())), status=tape.S.status())
    if return_timings:
        out["t_forward"] = t_fwd
        out["t_backward"] = t_bwd
    return out


def scene_for(theta, base="dam_break_2d", **kw):
    """The scene of a parameter vector theta = (mu, gamma_p, c0, H)."""
    mu, gp, c0, H = (float(x) for x in theta)
    if base == "dam_break_2d":
        return scenes.dam_break_2d(mu=mu, gamma_p=gp, c0=c0, column_height=H, **kw)
    raise ValueError(base)


class ProbeFunctional(torch.autograd.Function):
    """J(theta) of the 2-D dam break with its hand-written adjoint.

    forward(theta: float64 tensor [mu, gamma_p, c0, H], precision, K, scene
    kwargs) runs the checkpointed forward only and keeps its tape on ctx;
    backward runs the adjoint (recomputation and backward kernels) once and
    releases the tape."""

    @staticmethod
    def forward(ctx, theta, precision="f32", K=50, scene_kw=None):
        sc = scene_for(theta.detach().cpu().numpy(), **(scene_kw or {}))
        tape = forward(sc, precision=precision, K=K)
        ctx.tape = tape
        return torch.tensor(tape.J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        tape = ctx.tape
        if tape is None:
            raise RuntimeError("ProbeFunctional: backward called twice on one forward")
        g = backward(tape)
        ctx.tape = None
        return gJ * g.to(gJ.device), None, None, None
