"""Python binding of the gfx950 SPH library (include/sph.h, libsphx.so).

Argument marshalling only: every step of the pipeline runs in the HIP
kernels of libsphx.so.  PyTorch supplies device memory (one workspace
tensor per context, plus the exchange arrays) and the stream.  There is no
fallback: if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphx.so")

SPH_OK, SPH_E_ARG, SPH_E_CAPACITY, SPH_E_HIP, SPH_E_NUMERIC, SPH_E_STATE = range(6)
SPH_FP64, SPH_FP32_MIXED = 0, 1
SPH_FLUID, SPH_BUFFER, SPH_WALL, SPH_DEAD = 0, 1, 2, 3
(SPH_K_CELLS, SPH_K_CORRECTION, SPH_K_ADVECTION, SPH_K_PRESSURE, SPH_K_DENSITY,
 SPH_K_BUFFER, SPH_K_REDUCE) = range(7)
KERNEL_NAMES = ["cells", "correction", "advection", "pressure", "density",
                "buffer", "reduce"]
STATUS = {0: "SPH_OK", 1: "SPH_E_ARG", 2: "SPH_E_CAPACITY", 3: "SPH_E_HIP",
          4: "SPH_E_NUMERIC", 5: "SPH_E_STATE"}


class SphError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class sph_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32),
                ("turbulence", C.c_int32), ("obc_mode", C.c_int32),
                ("dp", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
                ("c0", C.c_double), ("nu_l", C.c_double), ("eta", C.c_double),
                ("g", C.c_double * 3), ("C1", C.c_double), ("C2", C.c_double),
                ("Cmu", C.c_double), ("sigma_k", C.c_double),
                ("sigma_eps", C.c_double), ("k_floor", C.c_double),
                ("eps_floor", C.c_double), ("cfl_adv", C.c_double),
                ("cfl_ac", C.c_double), ("u_ref", C.c_double),
                ("cell_size", C.c_double), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("capacity", C.c_int64),
                ("seed", C.c_uint64), ("tvf_alpha", C.c_double)]


class sph_buffer_desc(C.Structure):
    _fields_ = [("id", C.c_int32), ("vel_mode", C.c_int32), ("p_mode", C.c_int32),
                ("turb_mode", C.c_int32), ("profile", C.c_int32),
                ("n_coef", C.c_int32), ("origin", C.c_double * 3),
                ("frame", C.c_double * 9), ("length", C.c_double),
                ("half_width", C.c_double * 2), ("fringe", C.c_double),
                ("p_ob", C.c_double), ("k_bc", C.c_double), ("eps_bc", C.c_double),
                ("u0", C.c_double), ("noise_amp", C.c_double),
                ("coef", C.c_double * 16), ("ramp_time", C.c_double)]


class sph_particles(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in
                ("x", "v", "rho", "drho", "k", "eps", "tag", "pid")]


class sph_rates(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in
                ("ap", "drho", "anu", "gradv", "dk", "deps", "B", "p", "shift")]


class sph_buffer_counts(C.Structure):
    _fields_ = [("n_relabel", C.c_int32 * 256), ("n_inject", C.c_int32 * 256),
                ("n_delete", C.c_int32 * 256), ("n_revert", C.c_int32 * 256),
                ("n_real", C.c_int64), ("n_total", C.c_int64)]


class sph_step_ctrl(C.Structure):
    _fields_ = [("dt_adv", C.c_double), ("n_ac", C.c_int32), ("pad", C.c_int32)]


class sph_step_info(C.Structure):
    _fields_ = [("dt_adv", C.c_double), ("dt_ac", C.c_double), ("vmax", C.c_double),
                ("numax", C.c_double), ("t", C.c_double), ("n_ac", C.c_int32),
                ("list_outgrown", C.c_int32), ("step", C.c_int64)]


class sph_kernel_stats(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("launches", C.c_int64),
                ("bytes", C.c_double), ("particles", C.c_double)]


class sph_objective_desc(C.Structure):
    _fields_ = [("slab_origin", C.c_double * 3), ("slab_normal", C.c_double * 3),
                ("slab_width", C.c_double), ("shear_dir", C.c_double * 3),
                ("wall_length", C.c_double), ("control_buffer", C.c_int32),
                ("pad", C.c_int32)]


class sph_adjoint_ctrl(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("next_pid", C.c_uint64),
                ("dt_adv", C.c_double), ("n_ac", C.c_int32), ("pad", C.c_int32),
                ("dec_by_pid", C.c_void_p), ("member_by_pid", C.c_void_p),
                ("pid_cap", C.c_int64), ("w_flux", C.c_double), ("w_shear", C.c_double)]


EXPORTS = {
    "sph_workspace_size": (C.c_size_t, [C.POINTER(sph_params), C.POINTER(sph_buffer_desc), C.c_int32]),
    "sph_create": (C.c_int, [C.POINTER(sph_params), C.POINTER(sph_buffer_desc), C.c_int32,
                             C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "sph_destroy": (C.c_int, [C.c_void_p]),
    "sph_last_error": (C.c_char_p, [C.c_void_p]),
    "sph_set_particles": (C.c_int, [C.c_void_p, C.c_int64, C.c_uint64, C.POINTER(sph_particles)]),
    "sph_get_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sph_get_particles": (C.c_int, [C.c_void_p, C.POINTER(sph_particles)]),
    "sph_set_clock": (C.c_int, [C.c_void_p, C.c_int64, C.c_double]),
    "sph_build_cells": (C.c_int, [C.c_void_p]),
    "sph_correction": (C.c_int, [C.c_void_p]),
    "sph_step": (C.c_int, [C.c_void_p, C.POINTER(sph_step_ctrl), C.POINTER(sph_step_info)]),
    "sph_buffer_update": (C.c_int, [C.c_void_p, C.POINTER(sph_buffer_counts)]),
    "sph_advance": (C.c_int, [C.c_void_p, C.POINTER(sph_step_ctrl), C.POINTER(sph_step_info),
                              C.POINTER(sph_buffer_counts)]),
    "sph_buffer_decisions": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sph_eval_rates": (C.c_int, [C.c_void_p, C.POINTER(sph_rates)]),
    "sph_neighbors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                C.POINTER(C.c_int64)]),
    "sph_field_offset": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_size_t),
                                   C.POINTER(C.c_int32)]),
    "sph_set_count": (C.c_int, [C.c_void_p, C.c_int64, C.c_uint64]),
    "sph_step_pairs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.POINTER(C.c_int64)]),
    "sph_neighbors_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.POINTER(C.c_int64)]),
    "sph_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "sph_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(sph_kernel_stats)]),
    "sph_pair_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "sph_get_clock": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                C.POINTER(C.c_uint64)]),
    "sph_buffer_update_ex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.POINTER(sph_buffer_counts)]),
    "sph_set_profile_coef": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "sph_objective": (C.c_int, [C.c_void_p, C.POINTER(sph_objective_desc), C.c_void_p,
                                C.c_void_p, C.c_int64, C.c_void_p]),
    "sph_adjoint_workspace_size": (C.c_size_t, [C.c_void_p, C.c_int32]),
    "sph_adjoint_step": (C.c_int, [C.c_void_p, C.POINTER(sph_particles), C.c_int64,
                                   C.POINTER(sph_objective_desc), C.POINTER(sph_adjoint_ctrl),
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "sph_adjoint_forward": (C.c_int, [C.c_void_p, C.POINTER(sph_adjoint_ctrl), C.c_void_p,
                                      C.c_size_t, C.POINTER(C.c_int64)]),
    "sph_adjoint_reverse": (C.c_int, [C.c_void_p, C.POINTER(sph_objective_desc),
                                      C.POINTER(sph_adjoint_ctrl), C.c_int64, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_size_t]),
}

_lib = None


def lib():
    """Loads libsphx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------
def _check(ctx, st):
    if st != SPH_OK:
        msg = lib().sph_last_error(ctx)
        raise SphError(st, msg.decode() if msg else "")


def sph_workspace_size(params, bufs, nbuf):
    return lib().sph_workspace_size(C.byref(params), bufs, nbuf)


def sph_create(params, bufs, nbuf, ws_ptr, ws_bytes, stream_ptr):
    out = C.c_void_p()
    st = lib().sph_create(C.byref(params), bufs, nbuf, C.c_void_p(ws_ptr), ws_bytes,
                          C.c_void_p(stream_ptr), C.byref(out))
    if st != SPH_OK:
        raise SphError(st, "sph_create failed (invalid parameters, buffers or workspace)")
    return out


def sph_destroy(ctx):
    _check(ctx, lib().sph_destroy(ctx))


def sph_set_particles(ctx, n, next_pid, parts):
    _check(ctx, lib().sph_set_particles(ctx, n, next_pid, C.byref(parts)))


def sph_get_count(ctx):
    a, b = C.c_int64(), C.c_int64()
    _check(ctx, lib().sph_get_count(ctx, C.byref(a), C.byref(b)))
    return a.value, b.value


def sph_get_particles(ctx, parts):
    _check(ctx, lib().sph_get_particles(ctx, C.byref(parts)))


def sph_set_clock(ctx, step, t):
    _check(ctx, lib().sph_set_clock(ctx, step, t))


def sph_build_cells(ctx):
    _check(ctx, lib().sph_build_cells(ctx))


def sph_correction(ctx):
    _check(ctx, lib().sph_correction(ctx))


def sph_step(ctx, ctrl=None):
    info = sph_step_info()
    st = lib().sph_step(ctx, C.byref(ctrl) if ctrl is not None else None, C.byref(info))
    _check(ctx, st)
    return info


def sph_buffer_update(ctx):
    cnt = sph_buffer_counts()
    _check(ctx, lib().sph_buffer_update(ctx, C.byref(cnt)))
    return cnt


def sph_advance(ctx, ctrl=None):
    info, cnt = sph_step_info(), sph_buffer_counts()
    st = lib().sph_advance(ctx, C.byref(ctrl) if ctrl is not None else None, C.byref(info),
                           C.byref(cnt))
    _check(ctx, st)
    return info, cnt


def sph_buffer_decisions(ctx, dec_ptr):
    _check(ctx, lib().sph_buffer_decisions(ctx, C.c_void_p(dec_ptr)))


def sph_eval_rates(ctx, rates):
    _check(ctx, lib().sph_eval_rates(ctx, C.byref(rates)))


def sph_neighbors(ctx, row_ptr, col_ptr, cap):
    n = C.c_int64()
    _check(ctx, lib().sph_neighbors(ctx, C.c_void_p(row_ptr), C.c_void_p(col_ptr), cap,
                                    C.byref(n)))
    return n.value


def sph_neighbors_noalloc(ctx, row_ptr, col_ptr, cap):
    n = C.c_int64()
    _check(ctx, lib().sph_neighbors_noalloc(ctx, C.c_void_p(row_ptr), C.c_void_p(col_ptr), cap,
                                            C.byref(n)))
    return n.value


FIELDS = {"x0": 0, "x1": 1, "x2": 2, "v0": 3, "v1": 4, "v2": 5, "rho": 6, "drho": 7, "k": 8,
          "eps": 9, "tag": 10, "pid": 11}


def sph_field_offset(ctx, field):
    off, dt = C.c_size_t(), C.c_int32()
    _check(ctx, lib().sph_field_offset(ctx, int(field), C.byref(off), C.byref(dt)))
    return off.value, dt.value


def sph_set_count(ctx, n_total, next_pid):
    _check(ctx, lib().sph_set_count(ctx, int(n_total), int(next_pid)))


def sph_step_pairs(ctx, row_ptr, col_ptr, cap):
    n = C.c_int64()
    _check(ctx, lib().sph_step_pairs(ctx, C.c_void_p(row_ptr), C.c_void_p(col_ptr), cap,
                                     C.byref(n)))
    return n.value


def sph_profile_enable(ctx, on):
    _check(ctx, lib().sph_profile_enable(ctx, int(on)))


def sph_profile_read(ctx, kernel):
    s = sph_kernel_stats()
    _check(ctx, lib().sph_profile_read(ctx, kernel, C.byref(s)))
    return s


def sph_pair_count(ctx):
    n = C.c_int64()
    _check(ctx, lib().sph_pair_count(ctx, C.byref(n)))
    return n.value


def sph_get_clock(ctx):
    a, b, c = C.c_int64(), C.c_double(), C.c_uint64()
    _check(ctx, lib().sph_get_clock(ctx, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def sph_buffer_update_ex(ctx, forced_ptr, log_ptr, pid_cap):
    cnt = sph_buffer_counts()
    _check(ctx, lib().sph_buffer_update_ex(ctx, C.c_void_p(forced_ptr), C.c_void_p(log_ptr),
                                           int(pid_cap), C.byref(cnt)))
    return cnt


def sph_set_profile_coef(ctx, buffer_id, coef):
    a = np.ascontiguousarray(coef, dtype=np.float64)
    _check(ctx, lib().sph_set_profile_coef(ctx, int(buffer_id), int(a.size),
                                           a.ctypes.data_as(C.POINTER(C.c_double))))


def sph_objective(ctx, desc, member_in_ptr, member_out_ptr, pid_cap, J_ptr):
    _check(ctx, lib().sph_objective(ctx, C.byref(desc), C.c_void_p(member_in_ptr),
                                    C.c_void_p(member_out_ptr), int(pid_cap),
                                    C.c_void_p(J_ptr)))


def sph_adjoint_workspace_size(ctx, max_nac):
    return lib().sph_adjoint_workspace_size(ctx, int(max_nac))


def sph_adjoint_step(ctx, pre, n_pre, desc, ctrl, lam_ptr, grad_ptr, ws_ptr, ws_bytes):
    _check(ctx, lib().sph_adjoint_step(ctx, C.byref(pre), int(n_pre), C.byref(desc),
                                       C.byref(ctrl), C.c_void_p(lam_ptr), C.c_void_p(grad_ptr),
                                       C.c_void_p(ws_ptr), int(ws_bytes)))


def sph_adjoint_forward(ctx, ctrl, ws_ptr, ws_bytes):
    n = C.c_int64(0)
    _check(ctx, lib().sph_adjoint_forward(ctx, C.byref(ctrl), C.c_void_p(ws_ptr), int(ws_bytes),
                                          C.byref(n)))
    return int(n.value)


def sph_adjoint_reverse(ctx, desc, ctrl, n_step, lam_ptr, grad_ptr, ws_ptr, ws_bytes):
    _check(ctx, lib().sph_adjoint_reverse(ctx, C.byref(desc), C.byref(ctrl), int(n_step),
                                          C.c_void_p(lam_ptr), C.c_void_p(grad_ptr),
                                          C.c_void_p(ws_ptr), int(ws_bytes)))


def make_objective(d: dict, control_buffer: int) -> sph_objective_desc:
    o = sph_objective_desc()
    for f in ("slab_origin", "slab_normal", "shear_dir"):
        for k, a in enumerate(d[f]):
            getattr(o, f)[k] = float(a)
    o.slab_width = float(d["slab_width"])
    o.wall_length = float(d["wall_length"])
    o.control_buffer = int(control_buffer)
    return o


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def make_params(p: dict, precision: int, capacity: int) -> sph_params:
    P = sph_params()
    P.dim, P.precision = int(p["dim"]), int(precision)
    P.turbulence, P.obc_mode = int(p["turbulence"]), int(p["obc_mode"])
    for name in ("dp", "h", "rho0", "c0", "nu_l", "eta", "C1", "C2", "Cmu", "sigma_k",
                 "sigma_eps", "k_floor", "eps_floor", "cfl_adv", "cfl_ac", "u_ref",
                 "cell_size"):
        setattr(P, name, float(p[name]))
    for k in range(3):
        P.g[k], P.lo[k], P.hi[k] = p["g"][k], p["lo"][k], p["hi"][k]
    P.capacity = int(capacity)
    P.seed = int(p["seed"])
    P.tvf_alpha = float(p.get("tvf_alpha", 0.0))
    return P


def make_buffers(bufs):
    arr = (sph_buffer_desc * max(1, len(bufs)))()
    for q, b in enumerate(bufs):
        d = arr[q]
        d.id, d.vel_mode, d.p_mode, d.turb_mode = b.id, b.vel_mode, b.p_mode, b.turb_mode
        d.profile, d.n_coef = b.profile, len(b.coef)
        for k in range(3):
            d.origin[k] = b.origin[k]
            for c in range(3):
                d.frame[3 * k + c] = b.frame[k][c]
        d.length = b.length
        d.half_width[0], d.half_width[1] = b.half_width
        d.fringe, d.p_ob, d.k_bc, d.eps_bc = b.fringe, b.p_ob, b.k_bc, b.eps_bc
        d.u0, d.noise_amp, d.ramp_time = b.u0, b.noise_amp, b.ramp_time
        for m, a in enumerate(b.coef):
            d.coef[m] = a
    return arr


class Simulation:
    """One context on the current torch device and stream.

    ``case`` supplies ``params`` (dict), ``buffers`` and the particle arrays
    (x, v [n][3], rho, k, eps, tag, pid).  State is exchanged as FP64 numpy
    arrays ordered like the library's current (cell-sorted) order.
    """

    def __init__(self, case, precision=SPH_FP32_MIXED, capacity=None, device=None,
                 params=None, buffers=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the SPH library needs a GPU (torch.cuda is not available)")
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.case = case
        self.pdict = dict(case.params if params is None else params)
        self.bufs = list(case.buffers if buffers is None else buffers)
        self.capacity = case.capacity() if capacity is None else int(capacity)
        self.precision = precision
        self.turbulence = bool(self.pdict.get("turbulence", 0))
        self.P = make_params(self.pdict, precision, self.capacity)
        self.B = make_buffers(self.bufs)
        self.nbuf = len(self.bufs)
        nbytes = sph_workspace_size(self.P, self.B, self.nbuf)
        if nbytes == 0:
            raise SphError(SPH_E_ARG, "invalid parameters or buffers")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            self.ws_ptr = (base + 255) & ~255
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = sph_create(self.P, self.B, self.nbuf, self.ws_ptr, nbytes,
                                  self.stream.cuda_stream)
        self.load(case.x, case.v, case.rho, case.k, case.eps, case.tag, case.pid,
                  case.next_pid, drho=getattr(case, "drho", None),
                  step=int(getattr(case, "step", 0)), t=float(getattr(case, "t", 0.0)))

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                lib().sph_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    # -- state exchange -----------------------------------------------------
    def _dev(self, a, dtype):
        t = self.torch.as_tensor(np.ascontiguousarray(a), dtype=dtype)
        return t.to(self.device)

    def load(self, x, v, rho, k, eps, tag, pid, next_pid, drho=None, step=0, t=0.0):
        torch = self.torch
        n = int(np.asarray(x).shape[0])
        f64 = torch.float64
        self._in = dict(
            x=self._dev(np.asarray(x, dtype=np.float64).T.copy(), f64),
            v=self._dev(np.asarray(v, dtype=np.float64).T.copy(), f64),
            rho=self._dev(np.asarray(rho, dtype=np.float64), f64),
            drho=self._dev(np.zeros(n) if drho is None else np.asarray(drho, np.float64), f64),
            k=self._dev(np.asarray(k, dtype=np.float64), f64),
            eps=self._dev(np.asarray(eps, dtype=np.float64), f64),
            tag=self._dev(np.asarray(tag, dtype=np.uint32).view(np.int32), torch.int32),
            pid=self._dev(np.asarray(pid, dtype=np.uint32).view(np.int32), torch.int32))
        parts = sph_particles(*[self._in[f].data_ptr() for f in
                                ("x", "v", "rho", "drho", "k", "eps", "tag", "pid")])
        sph_set_particles(self.ctx, n, int(next_pid), parts)
        sph_set_clock(self.ctx, int(step), float(t))
        self._in = None

    def state(self):
        torch = self.torch
        n, _ = sph_get_count(self.ctx)
        f64 = dict(dtype=torch.float64, device=self.device)
        out = dict(x=torch.zeros(3, max(n, 1), **f64), v=torch.zeros(3, max(n, 1), **f64),
                   rho=torch.zeros(max(n, 1), **f64), drho=torch.zeros(max(n, 1), **f64),
                   k=torch.zeros(max(n, 1), **f64), eps=torch.zeros(max(n, 1), **f64),
                   tag=torch.zeros(max(n, 1), dtype=torch.int32, device=self.device),
                   pid=torch.zeros(max(n, 1), dtype=torch.int32, device=self.device))
        parts = sph_particles(*[out[f].data_ptr() for f in
                                ("x", "v", "rho", "drho", "k", "eps", "tag", "pid")])
        sph_get_particles(self.ctx, parts)
        res = {}
        for f, t in out.items():
            a = t.cpu().numpy()
            if f in ("x", "v"):
                a = a[:, :n].T.copy()
            else:
                a = a[:n].copy()
            if f in ("tag", "pid"):
                a = a.view(np.uint32)
            res[f] = a
        return res

    @property
    def n(self):
        return sph_get_count(self.ctx)[0]

    # -- pipeline -------------------------------------------------------------
    def build_cells(self):
        sph_build_cells(self.ctx)

    def correction(self):
        sph_correction(self.ctx)

    def step(self, dt_adv=0.0, n_ac=0):
        ctrl = None
        if dt_adv > 0:
            ctrl = sph_step_ctrl(float(dt_adv), int(n_ac), 0)
        return sph_step(self.ctx, ctrl)

    def buffer_update(self):
        return sph_buffer_update(self.ctx)

    def advance(self, dt_adv=0.0, n_ac=0):
        """build cells, correction, one advection step, buffer update (one
        library call; leaves the updated state built and corrected)."""
        ctrl = None
        if dt_adv > 0:
            ctrl = sph_step_ctrl(float(dt_adv), int(n_ac), 0)
        return sph_advance(self.ctx, ctrl)

    def decisions(self):
        torch = self.torch
        n = self.n
        d = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        sph_buffer_decisions(self.ctx, d.data_ptr())
        return d.cpu().numpy()[:n].view(np.uint32)

    def rates(self):
        torch = self.torch
        n = self.n
        f64 = dict(dtype=torch.float64, device=self.device)
        out = dict(ap=torch.zeros(3, n, **f64), drho=torch.zeros(n, **f64),
                   anu=torch.zeros(3, n, **f64), gradv=torch.zeros(9, n, **f64),
                   dk=torch.zeros(n, **f64), deps=torch.zeros(n, **f64),
                   B=torch.zeros(9, n, **f64), p=torch.zeros(n, **f64),
                   shift=torch.zeros(3, n, **f64))
        turb = bool(self.pdict["turbulence"])
        tvf = float(self.pdict.get("tvf_alpha", 0.0)) != 0.0
        ptr = lambda f: out[f].data_ptr() if ((turb or f not in ("gradv", "dk", "deps"))
                                              and (tvf or f != "shift")) else None
        R = sph_rates(*[ptr(f) for f in ("ap", "drho", "anu", "gradv", "dk", "deps", "B", "p",
                                         "shift")])
        sph_eval_rates(self.ctx, R)
        self.stream.synchronize()
        res = {f: t.cpu().numpy() for f, t in out.items()}
        for f in ("ap", "anu", "gradv", "B", "shift"):
            res[f] = res[f].T.copy()
        return res

    def neighbors(self):
        torch = self.torch
        n = self.n
        row = torch.zeros(n + 1, dtype=torch.int32, device=self.device)
        cap = max(64, n * (160 if self.pdict["dim"] == 3 else 48))
        col = torch.zeros(cap, dtype=torch.int32, device=self.device)
        m = sph_neighbors(self.ctx, row.data_ptr(), col.data_ptr(), cap)
        return row.cpu().numpy(), col.cpu().numpy()[:m]

    def field_view(self, name):
        """In-place tensor view (capacity entries) of a live particle array;
        valid until the next call that moves the arrays (build, step,
        update, advance, set)."""
        torch = self.torch
        off, dt = sph_field_offset(self.ctx, FIELDS[name])
        tdt, size = {0: (torch.float64, 8), 1: (torch.float32, 4), 2: (torch.int32, 4)}[dt]
        start = (self.ws_ptr - self.ws.data_ptr()) + off
        return self.ws[start:start + self.capacity * size].view(tdt)

    def set_count(self, n_total, next_pid):
        sph_set_count(self.ctx, n_total, next_pid)

    def step_pairs(self):
        """CSR (row_ptr, col) of the pairs the step's pair passes visit."""
        torch = self.torch
        n = self.n
        row = torch.zeros(n + 1, dtype=torch.int32, device=self.device)
        cap = max(64, n * (160 if self.pdict["dim"] == 3 else 48))
        col = torch.zeros(cap, dtype=torch.int32, device=self.device)
        m = sph_step_pairs(self.ctx, row.data_ptr(), col.data_ptr(), cap)
        return row.cpu().numpy(), col.cpu().numpy()[:m]

    def profile(self, on=True):
        sph_profile_enable(self.ctx, on)

    def kernel_stats(self):
        return {KERNEL_NAMES[k]: sph_profile_read(self.ctx, k) for k in range(len(KERNEL_NAMES))}

    def pair_count(self):
        return sph_pair_count(self.ctx)

    # -- sensitivity ------------------------------------------------------------
    def clock(self):
        """(step, t, next_pid) of the current state."""
        return sph_get_clock(self.ctx)

    def save(self):
        """Device copy of the whole state (checkpoint): particle arrays in the
        current order, their count and the clock."""
        torch = self.torch
        n, _ = sph_get_count(self.ctx)
        m = max(n, 1)
        f64 = dict(dtype=torch.float64, device=self.device)
        i32 = dict(dtype=torch.int32, device=self.device)
        snap = dict(x=torch.zeros(3, m, **f64), v=torch.zeros(3, m, **f64),
                    rho=torch.zeros(m, **f64), drho=torch.zeros(m, **f64),
                    k=torch.zeros(m, **f64), eps=torch.zeros(m, **f64),
                    tag=torch.zeros(m, **i32), pid=torch.zeros(m, **i32))
        sph_get_particles(self.ctx, self.parts_of(snap))
        snap["n"] = n
        snap["clock"] = self.clock()
        return snap

    def restore(self, snap):
        step, t, next_pid = snap["clock"]
        sph_set_particles(self.ctx, snap["n"], next_pid, self.parts_of(snap))
        sph_set_clock(self.ctx, step, t)

    @staticmethod
    def parts_of(snap):
        return sph_particles(*[snap[f].data_ptr() for f in
                               ("x", "v", "rho", "drho", "k", "eps", "tag", "pid")])

    def set_profile_coef(self, buffer_id, coef):
        sph_set_profile_coef(self.ctx, buffer_id, coef)

    def objective(self, desc, J, member_in=None, member_out=None, pid_cap=0):
        """Adds [J_Q, J_tau] of the current state to the device tensor J."""
        sph_objective(self.ctx, desc, 0 if member_in is None else member_in.data_ptr(),
                      0 if member_out is None else member_out.data_ptr(), pid_cap,
                      J.data_ptr())

    def buffer_update_ex(self, forced=None, log=None, pid_cap=0):
        return sph_buffer_update_ex(self.ctx, 0 if forced is None else forced.data_ptr(),
                                    0 if log is None else log.data_ptr(), pid_cap)
