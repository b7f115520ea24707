"""ctypes binding of the FP64 oracle (oracle/sph_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  Nothing in the product package
imports this module; it shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FLUID, BUFFER, WALL, DEAD = 0, 1, 2, 3
DEC_NONE, DEC_RELABEL, DEC_INJECT, DEC_DELETE, DEC_REVERT, DEC_REVERT_RELABEL = range(6)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("turbulence", C.c_int32),
                ("obc_mode", C.c_int32), ("pad0", C.c_int32),
                ("dp", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
                ("c0", C.c_double), ("nu_l", C.c_double), ("eta", C.c_double),
                ("g", C.c_double * 3),
                ("C1", C.c_double), ("C2", C.c_double), ("Cmu", C.c_double),
                ("sigma_k", C.c_double), ("sigma_eps", C.c_double),
                ("k_floor", C.c_double), ("eps_floor", C.c_double),
                ("cfl_adv", C.c_double), ("cfl_ac", C.c_double),
                ("u_ref", C.c_double), ("cell_size", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("seed", C.c_uint64), ("tvf_alpha", C.c_double)]


class BufferDesc(C.Structure):
    _fields_ = [("id", C.c_int32), ("vel_mode", C.c_int32),
                ("p_mode", C.c_int32), ("turb_mode", C.c_int32),
                ("profile", C.c_int32), ("n_coef", C.c_int32),
                ("origin", C.c_double * 3), ("frame", C.c_double * 9),
                ("length", C.c_double), ("half_width", C.c_double * 2),
                ("fringe", C.c_double), ("p_ob", C.c_double),
                ("k_bc", C.c_double), ("eps_bc", C.c_double),
                ("u0", C.c_double), ("noise_amp", C.c_double),
                ("coef", C.c_double * 16), ("ramp_time", C.c_double)]


class StateC(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64),
                ("x", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
                ("rho", C.POINTER(C.c_double)), ("drho", C.POINTER(C.c_double)),
                ("k", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
                ("tag", C.POINTER(C.c_uint32)), ("pid", C.POINTER(C.c_uint32)),
                ("next_pid", C.c_uint64), ("step", C.c_int64), ("t", C.c_double)]


class RatesC(C.Structure):
    _fields_ = [(nm, C.POINTER(C.c_double)) for nm in
                ("p", "vol", "ap", "drho", "anu", "gradv", "dk", "deps", "shift")]


class StepInfo(C.Structure):
    _fields_ = [("dt_adv", C.c_double), ("dt_ac", C.c_double),
                ("vmax", C.c_double), ("numax", C.c_double),
                ("n_ac", C.c_int32), ("pad", C.c_int32), ("n_pairs", C.c_int64)]


class Objective(C.Structure):
    _fields_ = [("slab_origin", C.c_double * 3), ("slab_normal", C.c_double * 3),
                ("slab_width", C.c_double), ("shear_dir", C.c_double * 3),
                ("wall_length", C.c_double)]


def make_objective(d: dict) -> Objective:
    o = Objective()
    for f in ("slab_origin", "slab_normal", "shear_dir"):
        for k, a in enumerate(d[f]):
            getattr(o, f)[k] = float(a)
    o.slab_width = float(d["slab_width"])
    o.wall_length = float(d["wall_length"])
    return o


class Counts(C.Structure):
    _fields_ = [("n_relabel", C.c_int32 * 256), ("n_inject", C.c_int32 * 256),
                ("n_delete", C.c_int32 * 256), ("n_revert", C.c_int32 * 256),
                ("n_real", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        u32p = C.POINTER(C.c_uint32)
        u8p = C.POINTER(C.c_uint8)
        PP, BP, SP = C.POINTER(Params), C.POINTER(BufferDesc), C.POINTER(StateC)
        sig = {
            "ora_set_threads": (None, [C.c_int]),
            "ora_get_threads": (C.c_int, []),
            "ora_splitmix64": (C.c_uint64, [C.c_uint64]),
            "ora_uniform": (C.c_double, [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32]),
            "ora_kernel_W": (C.c_double, [C.c_double, C.c_double, C.c_int]),
            "ora_kernel_dW": (C.c_double, [C.c_double, C.c_double, C.c_int]),
            "ora_neighbors_brute": (C.c_int64, [PP, C.c_int64, dp, i64p, i64p, C.c_int64]),
            "ora_neighbors_cll": (C.c_int64, [PP, C.c_int64, dp, i64p, i64p, C.c_int64]),
            "ora_correction": (C.c_int, [PP, BP, C.c_int, SP, C.c_int, dp, dp]),
            "ora_ghosts": (C.c_int64, [PP, BP, C.c_int, SP, C.c_int64, dp, dp, C.c_int64]),
            "ora_rates_eval": (C.c_int, [PP, BP, C.c_int, SP, dp, C.POINTER(RatesC)]),
            "ora_time_step": (C.c_int, [PP, SP, C.POINTER(StepInfo)]),
            "ora_advection_step": (C.c_int, [PP, BP, C.c_int, SP, C.c_double, C.c_int,
                                             C.POINTER(StepInfo)]),
            "ora_buffer_decisions": (C.c_int, [PP, BP, C.c_int, SP, u32p]),
            "ora_buffer_update": (C.c_int, [PP, BP, C.c_int, SP, C.POINTER(Counts), u32p]),
            "ora_velocity_bc": (C.c_int, [PP, BP, C.c_int, SP]),
            "ora_objective_eval": (C.c_int, [PP, SP, C.POINTER(Objective), u8p, u8p, dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


def make_params(p: dict) -> Params:
    P = Params()
    for name, _ in Params._fields_:
        if name == "pad0":
            continue
        val = p.get(name, 0.0) if name == "tvf_alpha" else p[name]
        if name in ("g", "lo", "hi"):
            for k in range(3):
                getattr(P, name)[k] = float(val[k])
        else:
            setattr(P, name, val)
    return P


def make_buffers(bufs) -> "C.Array":
    arr = (BufferDesc * max(1, len(bufs)))()
    for q, b in enumerate(bufs):
        d = arr[q]
        d.id, d.vel_mode, d.p_mode = b.id, b.vel_mode, b.p_mode
        d.turb_mode, d.profile, d.n_coef = b.turb_mode, b.profile, len(b.coef)
        for k in range(3):
            d.origin[k] = b.origin[k]
            for c in range(3):
                d.frame[3 * k + c] = b.frame[k][c]
        d.length = b.length
        d.half_width[0], d.half_width[1] = b.half_width
        d.fringe = b.fringe
        d.p_ob, d.k_bc, d.eps_bc = b.p_ob, b.k_bc, b.eps_bc
        d.u0, d.noise_amp = b.u0, b.noise_amp
        for m, a in enumerate(b.coef):
            d.coef[m] = a
        d.ramp_time = b.ramp_time
    return arr


class OracleSim:
    """Oracle state (numpy arrays, with a reserved tail for injection)."""

    def __init__(self, case, capacity=None, threads=1, params=None, buffers=None):
        self.case = case
        self.pdict = dict(case.params if params is None else params)
        self.P = make_params(self.pdict)
        self.bufs = list(case.buffers if buffers is None else buffers)
        self.B = make_buffers(self.bufs)
        self.nbuf = len(self.bufs)
        n = case.n
        cap = case.capacity() if capacity is None else capacity
        self.cap = cap
        self.x = np.zeros((cap, 3))
        self.v = np.zeros((cap, 3))
        self.rho = np.zeros(cap)
        self.drho = np.zeros(cap)
        self.k = np.zeros(cap)
        self.eps = np.zeros(cap)
        self.tag = np.zeros(cap, dtype=np.uint32)
        self.pid = np.zeros(cap, dtype=np.uint32)
        self.x[:n] = case.x
        self.v[:n] = case.v
        self.rho[:n] = case.rho
        self.k[:n] = case.k
        self.eps[:n] = case.eps
        self.tag[:n] = case.tag
        self.pid[:n] = case.pid
        if getattr(case, "drho", None) is not None:
            self.drho[:n] = case.drho
        self.S = StateC()
        self.S.n, self.S.cap = n, cap
        self.S.x, self.S.v = _ptr(self.x), _ptr(self.v)
        self.S.rho, self.S.drho = _ptr(self.rho), _ptr(self.drho)
        self.S.k, self.S.eps = _ptr(self.k), _ptr(self.eps)
        self.S.tag, self.S.pid = _ptr(self.tag, C.c_uint32), _ptr(self.pid, C.c_uint32)
        self.S.next_pid = case.next_pid
        self.S.step = int(getattr(case, "step", 0))
        self.S.t = float(getattr(case, "t", 0.0))
        lib().ora_set_threads(int(threads))

    # -- views -------------------------------------------------------------
    @property
    def n(self):
        return int(self.S.n)

    def snapshot(self):
        n = self.n
        return dict(x=self.x[:n].copy(), v=self.v[:n].copy(),
                    rho=self.rho[:n].copy(), drho=self.drho[:n].copy(),
                    k=self.k[:n].copy(), eps=self.eps[:n].copy(),
                    tag=self.tag[:n].copy(), pid=self.pid[:n].copy())

    def load(self, snap, step=None):
        n = snap["x"].shape[0]
        for f in ("x", "v", "rho", "drho", "k", "eps", "tag", "pid"):
            getattr(self, f)[:n] = snap[f]
        self.S.n = n
        if step is not None:
            self.S.step = step

    # -- operations ---------------------------------------------------------
    def correction(self, mirror=None):
        n = self.n
        mirror = (self.pdict["obc_mode"] >= 3) if mirror is None else mirror
        Bm = np.zeros((n, 9))
        sW = np.zeros(n)
        err = lib().ora_correction(C.byref(self.P), self.B, self.nbuf,
                                   C.byref(self.S), int(bool(mirror)),
                                   _ptr(Bm), _ptr(sW))
        if err:
            raise RuntimeError(f"ora_correction failed ({err})")
        return Bm, sW

    def ghosts(self, i, cap=4096):
        gx = np.zeros((cap, 3))
        gv = np.zeros(cap)
        m = lib().ora_ghosts(C.byref(self.P), self.B, self.nbuf, C.byref(self.S),
                             int(i), _ptr(gx), _ptr(gv), cap)
        if m < 0 or m > cap:
            raise RuntimeError("ora_ghosts failed")
        return gx[:m], gv[:m]

    def rates(self, Bm=None):
        n = self.n
        if Bm is None:
            if self.pdict["obc_mode"] >= 2:
                Bm, _ = self.correction()
            else:
                Bm = np.tile(np.eye(3).ravel(), (n, 1))
                if self.pdict["dim"] == 2:
                    Bm[:, 8] = 0.0
        out = dict(p=np.zeros(n), vol=np.zeros(n), ap=np.zeros((n, 3)),
                   drho=np.zeros(n), anu=np.zeros((n, 3)),
                   gradv=np.zeros((n, 9)), dk=np.zeros(n), deps=np.zeros(n),
                   shift=np.zeros((n, 3)))
        R = RatesC(*[_ptr(out[f]) for f in ("p", "vol", "ap", "drho", "anu",
                                            "gradv", "dk", "deps", "shift")])
        err = lib().ora_rates_eval(C.byref(self.P), self.B, self.nbuf,
                                   C.byref(self.S), _ptr(np.ascontiguousarray(Bm)),
                                   C.byref(R))
        if err:
            raise RuntimeError(f"ora_rates_eval failed ({err})")
        out["B"] = Bm
        return out

    def time_step(self):
        I = StepInfo()
        err = lib().ora_time_step(C.byref(self.P), C.byref(self.S), C.byref(I))
        if err:
            raise RuntimeError(f"ora_time_step failed ({err})")
        return I

    def step(self, dt_adv=0.0, n_ac=0):
        I = StepInfo()
        err = lib().ora_advection_step(C.byref(self.P), self.B, self.nbuf,
                                       C.byref(self.S), float(dt_adv), int(n_ac),
                                       C.byref(I))
        if err:
            raise RuntimeError(f"ora_advection_step failed ({err})")
        return I

    def decisions(self):
        dec = np.zeros(max(1, self.n), dtype=np.uint32)
        err = lib().ora_buffer_decisions(C.byref(self.P), self.B, self.nbuf,
                                         C.byref(self.S), _ptr(dec, C.c_uint32))
        if err:
            raise RuntimeError(f"ora_buffer_decisions failed ({err})")
        return dec[:self.n]

    def buffer_update(self, forced=None):
        Cn = Counts()
        f = None
        if forced is not None:
            forced = np.ascontiguousarray(forced, dtype=np.uint32)
            f = _ptr(forced, C.c_uint32)
        err = lib().ora_buffer_update(C.byref(self.P), self.B, self.nbuf,
                                      C.byref(self.S), C.byref(Cn), f)
        if err:
            raise RuntimeError(f"ora_buffer_update failed ({err})")
        return Cn

    def velocity_bc(self):
        lib().ora_velocity_bc(C.byref(self.P), self.B, self.nbuf, C.byref(self.S))

    def objective(self, desc: dict, member=None):
        """([J_Q, J_tau], slab membership) of the current state; `member`
        (0/1 per particle) freezes the slab membership."""
        n = self.n
        J = np.zeros(2)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        m_in = None
        if member is not None:
            member = np.ascontiguousarray(member, dtype=np.uint8)
            m_in = _ptr(member, C.c_uint8)
        err = lib().ora_objective_eval(C.byref(self.P), C.byref(self.S),
                                       C.byref(make_objective(desc)), m_in,
                                       _ptr(out, C.c_uint8), _ptr(J))
        if err:
            raise RuntimeError(f"ora_objective_eval failed ({err})")
        return J, out[:n]


# ---------------------------------------------------------------------------
# Inlet-profile sensitivity reference: rollouts with a frozen event log and
# central finite differences of the step-averaged objectives.
# ---------------------------------------------------------------------------
def with_coef(buffers, bid, coef):
    """Copy of the buffer list with buffer `bid`'s profile coefficients set."""
    import dataclasses
    out = []
    for b in buffers:
        if b.id == bid:
            b = dataclasses.replace(b, coef=tuple(float(a) for a in coef))
        out.append(b)
    return out


def rollout(case, steps, objective, buffers=None, replay=None, threads=1):
    """Run `steps` advection steps (step, objective, buffer update) and return
    the mean over steps of [J_Q, J_tau] with the run's event log.

    replay: a log from an earlier rollout; its time steps, slab memberships
    and buffer decisions are imposed (frozen) instead of being recomputed."""
    sim = OracleSim(case, threads=threads, buffers=buffers)
    J = np.zeros(2)
    log = []
    for s in range(steps):
        if replay is None:
            I = sim.step()
            dt_adv, n_ac = I.dt_adv, I.n_ac
        else:
            dt_adv, n_ac = replay[s]["dt_adv"], replay[s]["n_ac"]
            sim.step(dt_adv, n_ac)
        Js, member = sim.objective(objective, None if replay is None else replay[s]["member"])
        J += Js
        n = sim.n
        if replay is None:
            dec = sim.decisions().copy()
        else:
            dec = replay[s]["dec"]
        log.append(dict(dt_adv=float(dt_adv), n_ac=int(n_ac), dec=dec, member=member.copy(),
                        pid=sim.pid[:n].copy(), next_pid=int(sim.S.next_pid)))
        sim.buffer_update(forced=dec)
    return J / max(steps, 1), log, sim


def fd_gradient(case, steps, objective, bid, eps=1e-4, log=None, threads=1, coefs=None):
    """Central differences d[J_Q, J_tau]/d a_m of the step-averaged objectives
    with respect to the profile coefficients of buffer `bid`, decisions and
    time steps frozen to `log` (the unperturbed run's, by default)."""
    base = [b for b in case.buffers if b.id == bid][0]
    a0 = np.array(base.coef, dtype=np.float64)
    if coefs is None:
        coefs = range(len(a0))
    if log is None:
        _, log, _ = rollout(case, steps, objective, threads=threads)
    g = np.zeros((len(a0), 2))
    for m in coefs:
        Jp = []
        for sgn in (1.0, -1.0):
            a = a0.copy()
            a[m] += sgn * eps
            J, _, _ = rollout(case, steps, objective, with_coef(case.buffers, bid, a),
                              replay=log, threads=threads)
            Jp.append(J)
        g[m] = (Jp[0] - Jp[1]) / (2.0 * eps)
    return g, log


def neighbors(params: dict, x: np.ndarray, brute=False):
    """CSR neighbour lists (j sorted ascending)."""
    P = make_params(params)
    n = x.shape[0]
    x = np.ascontiguousarray(x, dtype=np.float64)
    cap = max(64, n * (150 if params["dim"] == 3 else 40))
    off = np.zeros(n + 1, dtype=np.int64)
    idx = np.zeros(cap, dtype=np.int64)
    f = lib().ora_neighbors_brute if brute else lib().ora_neighbors_cll
    m = f(C.byref(P), n, _ptr(x), _ptr(off, C.c_int64), _ptr(idx, C.c_int64), cap)
    if m < 0:
        raise RuntimeError("neighbour search failed")
    if brute:
        pass
    return off, idx[:m].copy()


def kernel_W(r, h, dim):
    return lib().ora_kernel_W(float(r), float(h), int(dim))


def kernel_dW(r, h, dim):
    return lib().ora_kernel_dW(float(r), float(h), int(dim))


def splitmix64(z):
    return int(lib().ora_splitmix64(C.c_uint64(z)))


def uniform(seed, pid, step, comp=0):
    return float(lib().ora_uniform(seed, pid, step, comp))
