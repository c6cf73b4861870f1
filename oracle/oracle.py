"""ctypes front end of the FP64 oracle (``sph_oracle.c``).

Test infrastructure: the functions here take plain NumPy arrays (positions
and velocities row-major ``(n, dim)``, float64) and return NumPy arrays.  They
follow the paper's equations one by one; see the C file for the passage each
one implements.  Nothing here imports the HIP package.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libsph_oracle.so")


class OrcParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("penalty_on", C.c_int32),
        ("dx", C.c_double),
        ("h", C.c_double),
        ("rho0", C.c_double),
        ("c", C.c_double),
        ("mu", C.c_double),
        ("gamma_p", C.c_double),
        ("dt", C.c_double),
        ("g", C.c_double * 3),
        ("a_wall", C.c_double * 3),
        ("sigma0", C.c_double),
        ("two_phase", C.c_int32),
        ("cross_phase", C.c_int32),
        ("n_heavy", C.c_int64),
        ("rho0_light", C.c_double),
        ("wall_v", C.c_double * 3),
        ("motion_amp", C.c_double * 3),
        ("motion_freq", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        i64 = C.c_int64
        pp = C.POINTER(OrcParams)
        L.orc_W.restype = C.c_double
        L.orc_W.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_dW.restype = C.c_double
        L.orc_dW.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_counting_sort.argtypes = [i64, ip, C.c_int32, ip, ip]
        L.orc_neighbours.argtypes = [C.c_int, C.c_double, i64, dp, i64, dp, ip,
                                     C.POINTER(C.c_int64), ip]
        L.orc_pairs_bruteforce.argtypes = [C.c_int, C.c_int, i64, ip, dp, i64, ip, dp,
                                           C.c_double, C.c_double, C.POINTER(C.c_uint8)]
        L.orc_riemann.argtypes = [C.c_double] * 7 + [dp]
        L.orc_riemann.restype = None
        qp = C.POINTER(C.c_int64)
        L.orc_sigma.argtypes = [pp, i64, dp, i64, dp, i64, qp, dp]
        L.orc_reinit.argtypes = [pp, i64, dp, dp, dp]
        L.orc_reinit.restype = None
        L.orc_sigma0.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_sigma0.restype = C.c_double
        L.orc_wall_pressure.argtypes = [pp, i64, dp, i64, dp, dp, i64, qp, dp]
        L.orc_normals.argtypes = [pp, i64, dp, dp, dp]
        L.orc_continuity.argtypes = [pp, i64, dp, dp, dp, i64, dp, dp, i64, qp, dp]
        L.orc_momentum.argtypes = [pp, i64, dp, dp, dp, i64, dp, dp, dp, i64, qp, dp]
        L.orc_diag.argtypes = [pp, i64, dp, dp, dp]
        L.orc_diag.restype = None
        L.orc_step.argtypes = [pp, i64, dp, dp, dp, dp, i64, dp, dp, dp, dp, i64, C.c_int, ip,
                               C.c_int, dp, C.c_double]
        L.orc_tank_motion.argtypes = [pp, i64, dp, dp, dp]
        L.orc_tank_motion.restype = None
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, dim=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if dim is not None:
        a = a.reshape(-1, dim)
    return a


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def params(dim, dx, h, rho0, c, mu=0.0, gamma_p=1.0, dt=0.0, g=(0.0, 0.0, 0.0),
           a_wall=(0.0, 0.0, 0.0), sigma0=None, penalty_on=True, n_heavy=None,
           rho0_light=None, wall_v=(0.0, 0.0, 0.0), motion_amp=(0.0, 0.0, 0.0),
           motion_freq=0.0, cross_phase=0) -> OrcParams:
    """Parameter block.  sigma0 defaults to the lattice sum of Eq. (17).
    Two phases: fluid particles with index >= n_heavy have reference density
    rho0_light (both given, or neither for a single phase).  wall_v is the
    wall velocity seen by the pair functions; a time step takes it, and the
    wall positions and acceleration, from the tank motion
    X(t) = motion_amp sin(2 pi motion_freq t)."""
    p = OrcParams()
    p.dim = int(dim)
    p.penalty_on = 1 if penalty_on else 0
    p.dx, p.h, p.rho0, p.c, p.mu, p.gamma_p, p.dt = dx, h, rho0, c, mu, gamma_p, dt
    for k in range(3):
        p.g[k] = float(g[k]) if k < len(g) else 0.0
        p.a_wall[k] = float(a_wall[k]) if k < len(a_wall) else 0.0
    p.sigma0 = sigma0_lattice(dim, dx, h) if sigma0 is None else float(sigma0)
    p.two_phase = 1 if rho0_light is not None else 0
    p.cross_phase = int(cross_phase)
    p.n_heavy = int(n_heavy) if n_heavy is not None else 0
    p.rho0_light = float(rho0_light) if rho0_light is not None else float(rho0)
    for k in range(3):
        p.wall_v[k] = float(wall_v[k]) if k < len(wall_v) else 0.0
        p.motion_amp[k] = float(motion_amp[k]) if k < len(motion_amp) else 0.0
    p.motion_freq = float(motion_freq)
    return p


def params_from_scene(sc, **over) -> OrcParams:
    kw = dict(dim=sc.dim, dx=sc.dx, h=sc.h, rho0=sc.rho0, c=sc.c0, mu=sc.mu,
              gamma_p=sc.gamma_p, dt=sc.dt, g=tuple(sc.g), penalty_on=sc.penalty_all)
    if getattr(sc, "rho0_light", None) is not None:
        kw.update(n_heavy=sc.n_heavy, rho0_light=sc.rho0_light, cross_phase=getattr(sc, "cross_phase", 0))
    if getattr(sc, "motion_freq", 0.0):
        kw.update(motion_amp=tuple(sc.motion_amp), motion_freq=sc.motion_freq)
    kw.update(over)
    return params(**kw)


# ---------------------------------------------------------------- kernel
def W(r, h, dim):
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    L = lib()
    return np.array([L.orc_W(dim, h, float(x)) for x in r.ravel()]).reshape(r.shape)


def dW(r, h, dim):
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    L = lib()
    return np.array([L.orc_dW(dim, h, float(x)) for x in r.ravel()]).reshape(r.shape)


def sigma0_lattice(dim, dx, h) -> float:
    return float(lib().orc_sigma0(int(dim), float(dx), float(h)))


# ---------------------------------------------------------------- cells
def counting_sort(keys, nkey):
    """Stable counting sort: returns (start[nkey+1], order[n])."""
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    start = np.zeros(nkey + 1, dtype=np.int32)
    order = np.zeros(max(len(keys), 1), dtype=np.int32)
    _check(lib().orc_counting_sort(len(keys), _i(keys), int(nkey), _i(start), _i(order)), "sort")
    return start, order[: len(keys)]


def neighbours(dim, h, xa, xb):
    """List of (a, b) index pairs with |x_a - x_b| < 2h (FP64), via cells.

    Returns (count[na], flat list of b per a in cell order)."""
    xa = _f64(xa, dim)
    xb = _f64(xb, dim)
    na, nb = len(xa), len(xb)
    L = lib()
    count = np.zeros(max(na, 1), dtype=np.int32)
    _check(L.orc_neighbours(dim, h, na, _d(xa), nb, _d(xb), _i(count), None, None), "neighbours")
    count = count[:na]
    off = np.zeros(na + 1, dtype=np.int64)
    np.cumsum(count, out=off[1:])
    lst = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
    cnt2 = np.zeros(max(na, 1), dtype=np.int32)
    _check(L.orc_neighbours(dim, h, na, _d(xa), nb, _d(xb), _i(cnt2),
                            off.ctypes.data_as(C.POINTER(C.c_int64)), _i(lst)), "neighbours")
    return count, lst[: int(off[-1])]


def pairs_bruteforce(dim, single, cell_a, off_a, cell_b, off_b, L, rc2):
    """Boolean matrix [na, nb] of pairs decided in the kernel's precision."""
    ca = np.ascontiguousarray(cell_a, dtype=np.int32).reshape(-1, dim)
    cb = np.ascontiguousarray(cell_b, dtype=np.int32).reshape(-1, dim)
    oa = _f64(off_a, dim)
    ob = _f64(off_b, dim)
    na, nb = len(ca), len(cb)
    hit = np.zeros(max(na * nb, 1), dtype=np.uint8)
    _check(lib().orc_pairs_bruteforce(dim, 1 if single else 0, na, _i(ca), _d(oa), nb, _i(cb),
                                      _d(ob), float(L), float(rc2),
                                      hit.ctypes.data_as(C.POINTER(C.c_uint8))), "pairs")
    return hit[: na * nb].reshape(na, nb).astype(bool)


# ---------------------------------------------------------------- physics
def riemann(rhoL, UL, pL, rhoR, UR, pR, c):
    """Eq. (8): returns dict(Ustar, pstar, Ubar, Pbar, beta)."""
    out = np.zeros(5)
    lib().orc_riemann(rhoL, UL, pL, rhoR, UR, pR, c, _d(out))
    return dict(Ustar=out[0], pstar=out[1], Ubar=out[2], Pbar=out[3], beta=out[4])


def _query(query, n):
    """(count, pointer, keep-alive array) of an optional index subset."""
    if query is None:
        return n, None, None
    q = np.ascontiguousarray(query, dtype=np.int64)
    if len(q) and (q.min() < 0 or q.max() >= n):
        raise IndexError("query index out of range")
    return len(q), q.ctypes.data_as(C.POINTER(C.c_int64)), q


def sigma(P, fx, wx, query=None):
    """sigma_i = sum_j W_ij over fluid and walls (j = i included); query
    selects the fluid particles to evaluate (default all)."""
    fx = _f64(fx, P.dim)
    wx = _f64(wx, P.dim)
    nq, qp, _keep = _query(query, len(fx))
    out = np.zeros(max(nq, 1))
    _check(lib().orc_sigma(C.byref(P), len(fx), _d(fx), len(wx), _d(wx), nq, qp, _d(out)), "sigma")
    return out[:nq]


def reinit(P, sig, rho_star):
    sig = _f64(sig)
    rho_star = _f64(rho_star)
    out = np.zeros(max(len(sig), 1))
    lib().orc_reinit(C.byref(P), len(sig), _d(sig), _d(rho_star), _d(out))
    return out[: len(sig)]


def wall_pressure(P, wx, fx, frho, query=None):
    """Eq. (12) for every wall particle (or the query subset)."""
    wx = _f64(wx, P.dim)
    fx = _f64(fx, P.dim)
    frho = _f64(frho)
    nq, qp, _keep = _query(query, len(wx))
    out = np.zeros(max(nq, 1))
    _check(lib().orc_wall_pressure(C.byref(P), len(wx), _d(wx), len(fx), _d(fx), _d(frho),
                                   nq, qp, _d(out)), "wall_pressure")
    return out[:nq]


def normals(P, wx, with_psi=False):
    wx = _f64(wx, P.dim)
    n = np.zeros((max(len(wx), 1), P.dim))
    psi = np.zeros((max(len(wx), 1), P.dim))
    _check(lib().orc_normals(C.byref(P), len(wx), _d(wx), _d(n), _d(psi)), "normals")
    if with_psi:
        return n[: len(wx)], psi[: len(wx)]
    return n[: len(wx)]


def continuity(P, fx, fv, frho, wx, pw, query=None):
    """drho/dt of Eq. (9) for every fluid particle (or the query subset)."""
    fx = _f64(fx, P.dim)
    fv = _f64(fv, P.dim)
    frho = _f64(frho)
    wx = _f64(wx, P.dim)
    pw = _f64(pw)
    nq, qp, _keep = _query(query, len(fx))
    out = np.zeros(max(nq, 1))
    _check(lib().orc_continuity(C.byref(P), len(fx), _d(fx), _d(fv), _d(frho), len(wx), _d(wx),
                                _d(pw), nq, qp, _d(out)), "continuity")
    return out[:nq]


def momentum(P, fx, fv, frho, wx, pw, wn, query=None):
    """dv/dt of Eqs. (10)-(11), (13) + viscous + g (or the query subset)."""
    fx = _f64(fx, P.dim)
    fv = _f64(fv, P.dim)
    frho = _f64(frho)
    wx = _f64(wx, P.dim)
    pw = _f64(pw)
    wn = _f64(wn, P.dim)
    nq, qp, _keep = _query(query, len(fx))
    out = np.zeros((max(nq, 1), P.dim))
    _check(lib().orc_momentum(C.byref(P), len(fx), _d(fx), _d(fv), _d(frho), len(wx), _d(wx),
                              _d(pw), _d(wn), nq, qp, _d(out)), "momentum")
    return out[:nq]


def diag(P, fx, fv):
    fx = _f64(fx, P.dim)
    fv = _f64(fv, P.dim)
    out = np.zeros(8)
    lib().orc_diag(C.byref(P), len(fx), _d(fx), _d(fv), _d(out))
    return dict(M=out[0], P=out[1:4].copy(), Ek=out[4], Ep=out[5], vmax=out[6])


def tank_motion(P, step):
    """(X, V, A) of the prescribed tank motion at t = step dt, each (dim,)."""
    X, V, A = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_tank_motion(C.byref(P), int(step), _d(X), _d(V), _d(A))
    return X[: P.dim], V[: P.dim], A[: P.dim]


class State:
    """Oracle state of one run: fluid arrays are updated in place by step().

    wx0 are the wall dummies at t = 0; with a tank motion they sit at
    wx0 + X(t) (self.wx) and move with it."""

    def __init__(self, P, fx, fv, frho, wx, probe=None):
        d = P.dim
        self.P = P
        self.x = _f64(fx, d).copy()
        self.v = _f64(fv, d).copy()
        self.rho = _f64(frho).copy()
        self.wx0 = _f64(wx, d).copy()
        self.nstep = 0
        X, V, A = tank_motion(P, 0)
        self.wx = self.wx0 + X
        self.wn = normals(P, self.wx)
        # initial wall pressure and acceleration from the initial state, the
        # walls moving with X'(0) and accelerating with X''(0)
        Q = params_copy(P, wall_v=V, a_wall=np.array(P.a_wall[:d]) + A)
        self.pw = wall_pressure(Q, self.wx, self.x, self.rho)
        self.a = momentum(Q, self.x, self.v, self.rho, self.wx, self.pw, self.wn)
        self.probe = None if probe is None else np.ascontiguousarray(probe, dtype=np.int32)
        self.J = 0.0

    @classmethod
    def resume(cls, P, x, v, rho, a, wx0, nstep, pw=None, probe=None):
        """A state taken over mid-run: fluid arrays at step nstep (a = the
        dv/dt of the last momentum evaluation), walls at wx0 + X(t)."""
        d = P.dim
        st = cls.__new__(cls)
        st.P = P
        st.x = _f64(x, d).copy()
        st.v = _f64(v, d).copy()
        st.rho = _f64(rho).copy()
        st.a = _f64(a, d).copy()
        st.wx0 = _f64(wx0, d).copy()
        st.nstep = int(nstep)
        st.wx = st.wx0 + tank_motion(P, st.nstep)[0]
        st.wn = normals(P, st.wx)
        st.pw = np.zeros(len(st.wx)) if pw is None else _f64(pw).copy()
        st.probe = None if probe is None else np.ascontiguousarray(probe, dtype=np.int32)
        st.J = 0.0
        return st

    def step(self, n=1, damp=0.0):
        P = self.P
        Jb = np.zeros(1)
        pwb = np.zeros(max(len(self.wx), 1))
        pwb[: len(self.pw)] = self.pw
        nprobe = 0 if self.probe is None else len(self.probe)
        wxb = self.wx.copy()
        _check(lib().orc_step(C.byref(P), len(self.x), _d(self.x), _d(self.v), _d(self.rho),
                              _d(self.a), len(self.wx0), _d(self.wx0), _d(wxb), _d(self.wn),
                              _d(pwb), int(self.nstep), int(n),
                              _i(self.probe) if nprobe else None, nprobe, _d(Jb),
                              float(damp)), "step")
        self.wx = wxb
        self.pw = pwb[: len(self.wx)].copy()
        self.J += float(Jb[0])
        self.nstep += n
        return self

    def diag(self):
        return diag(self.P, self.x, self.v)


def params_copy(P, **over) -> OrcParams:
    """A copy of a parameter block with some fields replaced (vectors padded)."""
    q = OrcParams()
    C.pointer(q)[0] = P
    for k, v in over.items():
        if isinstance(getattr(q, k), C.Array):
            arr = getattr(q, k)
            for i in range(3):
                arr[i] = float(v[i]) if i < len(v) else 0.0
        else:
            setattr(q, k, v)
    return q


def num_threads() -> int:
    return int(lib().orc_num_threads())


def time_steps(P, fx, fv, frho, wx, nsteps=1):
    """Wall-clock seconds of nsteps oracle steps (initialisation excluded)."""
    st = State(P, fx, fv, frho, wx)
    t0 = time.perf_counter()
    st.step(nsteps)
    return time.perf_counter() - t0, st
