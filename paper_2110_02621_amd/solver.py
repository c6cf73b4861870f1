"""Thin Python front end of the C ABI: torch owns the device buffers and the
stream, every step of the method runs in the HIP kernels of ``libsph.so``.

    from paper_2110_02621_amd import scenes, solver
    s = solver.Solver(scenes.dam_break_3d(dx=0.004), precision="f32")
    s.step(100)
    print(s.diag())

Requires a ROCm GPU and the built library; raises otherwise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi
from .abi import check

_PREC = {"f32": (abi.SPH_F32, torch.float32), "f64": (abi.SPH_F64, torch.float64)}


def _p(t: torch.Tensor):
    return C.c_void_p(t.data_ptr()) if t.numel() > 0 else C.c_void_p(0)


def make_desc(scene, precision="f32") -> abi.Desc:
    d = abi.Desc()
    d.dim = scene.dim
    d.precision = _PREC[precision][0]
    d.penalty_all = 1 if scene.penalty_all else 0
    d.dx, d.h, d.rho0, d.c0 = scene.dx, scene.h, scene.rho0, scene.c0
    d.mu, d.gamma_p, d.dt = scene.mu, scene.gamma_p, scene.dt
    if getattr(scene, "rho0_light", None) is not None:
        d.two_phase = 1
        d.n_heavy = int(scene.n_heavy)
        d.rho0_light = float(scene.rho0_light)
        d.cross_phase = int(getattr(scene, "cross_phase", 0))
    d.motion_freq = float(getattr(scene, "motion_freq", 0.0))
    for k in range(3):
        d.motion_amp[k] = float(scene.motion_amp[k]) if d.motion_freq else 0.0
        d.g[k] = float(scene.g[k])
        d.a_wall[k] = 0.0
        d.lo[k] = float(scene.lo[k]) if k < scene.dim else 0.0
        d.hi[k] = float(scene.hi[k]) if k < scene.dim else 1.0
    check(abi.load().sph_configure(C.byref(d)), "sph_configure")
    return d


class Solver:
    """Device-resident state of one run and the calls of the C ABI."""

    # Neighbour masks: two 64-bit words per stencil row and query.
    MASK_ROWS = {2: 3, 3: 9}

    def __init__(self, scene, precision="f32", device="cuda", probe=True, keep_sigma=False,
                 lists=True):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = abi.load()
        self.scene = scene
        self.precision = precision
        self.device = torch.device(device)
        self.desc = make_desc(scene, precision)
        dim, T = scene.dim, _PREC[precision][1]
        self.dtype = T
        nf, nw = scene.n_fluid, scene.n_wall
        dev = self.device
        i32 = dict(dtype=torch.int32, device=dev)
        self.t = t = {}
        t["key"] = torch.zeros((2, nf), **i32)
        t["pid"] = torch.zeros((2, nf), **i32)
        t["off"] = torch.zeros((2, dim, nf), dtype=T, device=dev)
        t["vel"] = torch.zeros((2, dim, nf), dtype=T, device=dev)
        t["rho"] = torch.zeros((2, nf), dtype=T, device=dev)
        t["acc"] = torch.zeros((dim, nf), dtype=T, device=dev)
        t["wkey"] = torch.zeros(nw, **i32)
        t["wpid"] = torch.zeros(nw, **i32)
        t["woff"] = torch.zeros((dim, nw), dtype=T, device=dev)
        t["pw"] = torch.zeros(nw, dtype=T, device=dev)
        t["nrm"] = torch.zeros((dim, nw), dtype=T, device=dev)
        nc = int(self.desc.n_cells)
        t["fstart"] = torch.zeros(nc + 1, **i32)
        t["wstart"] = torch.zeros(nc + 1, **i32)
        sb = int(self.lib.sph_scratch_bytes(C.byref(self.desc), nf, nw))
        t["scratch"] = torch.zeros(sb + 256, dtype=torch.uint8, device=dev)
        t["status"] = torch.zeros(abi.SPH_STATUS_LEN, **i32)
        t["diag"] = torch.zeros(abi.SPH_DIAG_LEN, dtype=torch.float64, device=dev)
        t["sigma"] = torch.zeros(nf if keep_sigma else 0, dtype=T, device=dev)
        words = 2 * self.MASK_ROWS[dim] if lists else 0
        i64 = dict(dtype=torch.int64, device=dev)
        t["nbr_ff"] = torch.zeros((words, nf), **i64)
        t["nbr_fw"] = torch.zeros((words, nf), **i64)
        t["nbr_wf"] = torch.zeros((words, nw), **i64)
        t["cnt_ff"] = torch.zeros(nf if lists else 0, **i32)
        t["cnt_fw"] = torch.zeros(nf if lists else 0, **i32)
        t["cnt_wf"] = torch.zeros(nw if lists else 0, **i32)
        pr = scene.probe if (probe and len(scene.probe)) else np.zeros(0)
        t["probe"] = torch.as_tensor(np.asarray(pr, dtype=np.int32), device=dev)

        b = abi.Buffers()
        b.n_fluid, b.n_wall = nf, nw
        for c in range(2):
            b.key[c] = _p(t["key"][c]).value
            b.pid[c] = _p(t["pid"][c]).value
            b.off[c] = _p(t["off"][c]).value
            b.vel[c] = _p(t["vel"][c]).value
            b.rho[c] = _p(t["rho"][c]).value
        b.acc = _p(t["acc"]).value
        for name in ("wkey", "wpid", "woff", "pw", "nrm", "fstart", "wstart", "status", "diag"):
            setattr(b, name, _p(t[name]).value)
        base = t["scratch"].data_ptr()
        aligned = (base + 255) & ~255
        b.scratch = aligned if sb else base
        b.scratch_bytes = sb
        b.sigma_out = _p(t["sigma"]).value
        b.probe = _p(t["probe"]).value
        b.n_probe = int(t["probe"].numel())
        if lists:
            # a mask array of zero size (no fluid or no walls) still needs a
            # non-null pointer: point it at the (then unused) status words
            for name in ("nbr_ff", "nbr_fw", "nbr_wf", "cnt_ff", "cnt_fw", "cnt_wf"):
                setattr(b, name, _p(t[name]).value or _p(t["status"]).value)
        self.buf = b

        def soa(a, n):
            return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n, dim).T),
                                   device=dev)

        fpos = soa(scene.fluid_x, nf)
        fvel = soa(scene.fluid_v, nf)
        frho = torch.as_tensor(np.asarray(scene.fluid_rho, dtype=np.float64), device=dev)
        wpos = soa(scene.wall_x, nw)
        self._call("sph_init", self.lib.sph_init, _p(fpos), _p(fvel), _p(frho), _p(wpos))
        torch.cuda.current_stream(dev).synchronize()
        del fpos, fvel, frho, wpos

    # -- calls -------------------------------------------------------------
    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _call(self, name, fn, *args):
        check(fn(C.byref(self.desc), C.byref(self.buf), *args, self._stream()), name)

    def step(self, n=1):
        self._call("sph_step", self.lib.sph_step, int(n))
        return self

    def density(self):
        self._call("sph_density", self.lib.sph_density)

    def build_cells(self):
        self._call("sph_build_cells", self.lib.sph_build_cells)

    def wall_bc(self):
        self._call("sph_wall_bc", self.lib.sph_wall_bc)

    def continuity(self):
        self._call("sph_forces", self.lib.sph_forces, abi.SPH_CONTINUITY)

    def momentum(self, kick=True):
        self._call("sph_forces", self.lib.sph_forces, abi.SPH_MOMENTUM | (0 if kick else abi.SPH_NO_KICK))

    def synchronize(self):
        torch.cuda.current_stream(self.device).synchronize()

    # -- read back (host copies; for tests, diagnostics and output) --------
    def diag(self):
        self._call("sph_diag", self.lib.sph_diag)
        d = self.t["diag"].cpu().numpy()
        return dict(M=d[abi.SPH_DIAG_MASS], P=d[abi.SPH_DIAG_MOM:abi.SPH_DIAG_MOM + 3].copy(),
                    Ek=d[abi.SPH_DIAG_EKIN], Ep=d[abi.SPH_DIAG_EPOT], vmax=d[abi.SPH_DIAG_VMAX],
                    J=d[abi.SPH_DIAG_PROBE], steps=int(d[abi.SPH_DIAG_STEPS]))

    def status(self):
        s = self.t["status"].cpu().numpy().astype(np.int64)
        return dict(out_of_grid=int(s[abi.SPH_STATUS_OUT_OF_GRID]), fast=int(s[abi.SPH_STATUS_FAST]),
                    nonfinite=int(s[abi.SPH_STATUS_NONFINITE]),
                    list_overflow=int(s[abi.SPH_STATUS_LIST_OVERFLOW]))

    def export(self):
        """Fluid state in particle-id order: pos, vel, acc (n, dim), rho (n,)."""
        nf, dim = self.scene.n_fluid, self.scene.dim
        dev = self.device
        pos = torch.zeros((dim, nf), dtype=torch.float64, device=dev)
        vel = torch.zeros_like(pos)
        acc = torch.zeros_like(pos)
        rho = torch.zeros(nf, dtype=torch.float64, device=dev)
        self._call("sph_export", self.lib.sph_export, _p(pos), _p(vel), _p(rho), _p(acc))
        return dict(pos=pos.T.cpu().numpy(), vel=vel.T.cpu().numpy(), rho=rho.cpu().numpy(),
                    acc=acc.T.cpu().numpy())

    def export_walls(self):
        """Wall pressure (n,), normals and positions (n, dim) in wall-id order."""
        nw, dim = self.scene.n_wall, self.scene.dim
        dev = self.device
        pw = torch.zeros(nw, dtype=torch.float64, device=dev)
        nrm = torch.zeros((dim, nw), dtype=torch.float64, device=dev)
        pos = torch.zeros((dim, nw), dtype=torch.float64, device=dev)
        self._call("sph_export_walls", self.lib.sph_export_walls, _p(pw), _p(nrm), _p(pos))
        return dict(pw=pw.cpu().numpy(), nrm=nrm.T.cpu().numpy(), pos=pos.T.cpu().numpy())

    def neighbours(self, which=0):
        """Neighbour sets as the sweeps enumerate them: (count, offsets, ids)
        indexed by particle (which=0) or wall (which=1) id."""
        nq = self.scene.n_fluid if which == 0 else self.scene.n_wall
        dev = self.device
        count = torch.zeros(nq, dtype=torch.int32, device=dev)
        self._call("sph_neighbours", self.lib.sph_neighbours, int(which), C.c_void_p(0), _p(count),
                   C.c_void_p(0), 0)
        offset = torch.zeros(nq, dtype=torch.int64, device=dev)
        if nq > 1:
            offset[1:] = torch.cumsum(count.to(torch.int64), 0)[:-1]
        total = int(count.to(torch.int64).sum().item()) if nq else 0
        lst = torch.full((max(total, 1),), -1, dtype=torch.int32, device=dev)
        count2 = torch.zeros_like(count)
        self._call("sph_neighbours", self.lib.sph_neighbours, int(which), _p(offset), _p(count2),
                   _p(lst), total)
        return count.cpu().numpy(), offset.cpu().numpy(), lst[:total].cpu().numpy()

    def pair_counts(self):
        """Interacting pairs of the current sorted state from the neighbour
        list counts: fluid-fluid with self, fluid-wall, wall-fluid."""
        t = self.t
        if t["cnt_ff"].numel() == 0 and self.scene.n_fluid > 0:
            raise RuntimeError("pair_counts needs the neighbour lists (Solver(..., lists=True))")
        if any(int((t[k] < 0).sum()) for k in ("cnt_ff", "cnt_fw", "cnt_wf") if t[k].numel()):
            raise RuntimeError("pair_counts: some queries overflowed their masks")
        s = lambda x: int(x.to(torch.int64).sum().item()) if x.numel() else 0
        return dict(ff_with_self=s(t["cnt_ff"]), fw=s(t["cnt_fw"]), wf=s(t["cnt_wf"]),
                    max_ff=int(t["cnt_ff"].max().item()) if t["cnt_ff"].numel() else 0)

    def raw(self):
        """Host copies of the raw sorted buffers and the current-copy flags."""
        out = {k: v.cpu().numpy() for k, v in self.t.items() if k not in ("scratch", "nbr_ff", "nbr_fw", "nbr_wf")}
        out["sel_vel"] = int(self.buf.sel_vel)
        out["sel_rho"] = int(self.buf.sel_rho)
        return out

    def cell_coords(self, key):
        nx, ny = int(self.desc.grid[0]), int(self.desc.grid[1])
        key = np.asarray(key, dtype=np.int64)
        c = np.stack([key % nx, (key // nx) % ny, key // (nx * ny)], axis=1)
        return c[:, : self.scene.dim]

    def absolute(self, key, off):
        """Absolute positions (n, dim) of raw key / offset arrays (offset (dim, n))."""
        c = self.cell_coords(key)
        lo = np.array([self.desc.lo[k] for k in range(self.scene.dim)])
        return lo + c * float(self.desc.cell) + np.asarray(off, dtype=np.float64).T
