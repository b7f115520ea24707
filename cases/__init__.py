"""Seeded synthetic inputs for the WCSPH / k-epsilon RANS open-boundary step.

This module only builds *inputs*: particle lattices, wall bands, buffer
boxes and physical parameters for the five workloads (straight channel,
U-channel, plane jet, 3D micro-mixer, adjoint channel).  It holds none of
the method's arithmetic (no kernel, no operator, no buffer predicate); both
the FP64 oracle and the HIP path consume the arrays produced here.

All particles start FLUID (or WALL); labelling particles that start inside a
buffer box is left to the first buffer update of whichever implementation
runs the case.

Geometry conventions (shared interface of both implementations):
  * positions are float64 [n][3] (z = 0 in 2D);
  * tag = kind | (buffer_id << 8), kind 0 fluid, 1 buffer, 2 wall;
  * a buffer box is given by the centre of its open face (``origin``), an
    orthonormal frame whose row 0 is the unit normal pointing into the fluid,
    its length L_b along that normal, its transverse half widths and the
    fringe offset of the particle-generation line (0.5 dp).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

FLUID, BUFFER, WALL = 0, 1, 2

VEL_EXTRAPOLATE, VEL_PRESCRIBED = 0, 1
P_NONE, P_PRESCRIBED, P_EXTRAPOLATE = 0, 1, 2
TURB_ZERO_GRADIENT, TURB_FREESTREAM = 0, 1
PROFILE_UNIFORM, PROFILE_PARABOLIC, PROFILE_SINE = 0, 1, 2

# Table A of the paper (standard k-epsilon constants).
KEPS = dict(C1=1.44, C2=1.92, Cmu=0.09, sigma_k=1.0, sigma_eps=1.3)


def make_tag(kind: int, bid: int = 0) -> int:
    return int(kind) | (int(bid) << 8)


@dataclasses.dataclass
class Buffer:
    id: int
    origin: tuple
    frame: tuple            # 3 rows, row 0 = inward normal n_b
    length: float
    half_width: tuple       # (w1, w2); w2 unused in 2D
    fringe: float
    vel_mode: int = VEL_EXTRAPOLATE
    p_mode: int = P_NONE
    turb_mode: int = TURB_ZERO_GRADIENT
    p_ob: float = 0.0
    k_bc: float = 0.0
    eps_bc: float = 0.0
    profile: int = PROFILE_UNIFORM
    u0: float = 0.0
    coef: tuple = ()
    noise_amp: float = 0.0
    ramp_time: float = 0.0


@dataclasses.dataclass
class Case:
    name: str
    params: dict
    buffers: List[Buffer]
    x: np.ndarray
    v: np.ndarray
    rho: np.ndarray
    k: np.ndarray
    eps: np.ndarray
    tag: np.ndarray
    pid: np.ndarray
    steps: int
    note: str = ""
    drho: np.ndarray = None       # last continuity rate (None: zero)
    npid: int = None              # id of the next injected particle
    step: int = 0                 # step counter of the state
    t: float = 0.0                # physical time of the state
    objective: dict = None        # objective descriptor of a sensitivity case

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_wall(self) -> int:
        return int(np.count_nonzero((self.tag & 3) == WALL))

    @property
    def n_fluid(self) -> int:
        return self.n - self.n_wall

    @property
    def next_pid(self) -> int:
        if self.npid is not None:
            return int(self.npid)
        return int(self.pid.max()) + 1 if self.n else 0

    def capacity(self, factor: float = 1.25, extra: int = 4096) -> int:
        return int(self.n * factor) + extra


def base_params(dim, dp, rho0=1.0, c0=10.0, nu_l=1e-3, u_ref=1.0,
                turbulence=0, obc_mode=4, seed=0):
    h = 1.3 * dp
    p = dict(dim=dim, turbulence=turbulence, obc_mode=obc_mode, dp=dp, h=h,
             rho0=rho0, c0=c0, nu_l=nu_l, eta=3.0, g=(0.0, 0.0, 0.0),
             k_floor=1e-10, eps_floor=1e-10, cfl_adv=0.25, cfl_ac=0.6,
             u_ref=u_ref, cell_size=2.6 * h, lo=(0.0, 0.0, 0.0),
             hi=(0.0, 0.0, 0.0), seed=seed)
    p.update(KEPS)
    return p


def _set_bounds(params, pts, pad_cells=3):
    cs = params["cell_size"]
    lo = pts.min(axis=0) - pad_cells * cs
    hi = pts.max(axis=0) + pad_cells * cs
    if params["dim"] == 2:
        lo[2], hi[2] = -cs, cs
    params["lo"] = tuple(float(a) for a in lo)
    params["hi"] = tuple(float(a) for a in hi)


def lattice2(x0, x1, y0, y1, dp):
    """Lattice points ((i+1/2)dp, (j+1/2)dp) with x0 <= x < x1, y0 <= y < y1,
    for x0, y0 multiples of dp."""
    i0, i1 = int(round(x0 / dp)), int(round(x1 / dp))
    j0, j1 = int(round(y0 / dp)), int(round(y1 / dp))
    xs = (np.arange(i0, i1) + 0.5) * dp
    ys = (np.arange(j0, j1) + 0.5) * dp
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pts = np.zeros((X.size, 3))
    pts[:, 0] = X.ravel()
    pts[:, 1] = Y.ravel()
    return pts


def _assemble(name, params, buffers, fluid, wall, steps, *, v=None, k0=0.0,
              eps0=0.0, note="", pad_cells=3):
    nf, nw = fluid.shape[0], wall.shape[0]
    x = np.concatenate([fluid, wall]).astype(np.float64)
    n = nf + nw
    vel = np.zeros((n, 3))
    if v is not None:
        vel[:nf] = v
    rho = np.full(n, params["rho0"])
    k = np.zeros(n)
    eps = np.zeros(n)
    if params["turbulence"]:
        k[:nf] = k0
        eps[:nf] = eps0
    tag = np.zeros(n, dtype=np.uint32)
    tag[nf:] = WALL
    pid = np.arange(n, dtype=np.uint32)
    _set_bounds(params, x, pad_cells)
    return Case(name, params, buffers, x, vel, rho, k, eps, tag, pid,
                steps, note)


def _frame2(nx, ny):
    n = np.array([nx, ny, 0.0])
    t = np.array([-ny, nx, 0.0])
    return (tuple(n), tuple(t), (0.0, 0.0, 1.0))


# ----------------------------------------------------------------------------
# 2D straight channel (Poiseuille): domain L x H, parabolic velocity inlet,
# zero-pressure outlet, 3 layers of wall particles above and below.
# ----------------------------------------------------------------------------
def make_channel(H=1.0, L=10.0, dp=None, Re=100.0, Umax=1.0, c0=10.0,
                 steps=200, profile=PROFILE_PARABOLIC, coef=(), obc_mode=4,
                 name="channel", seed=0, ramp_time=10.0, p_out=0.0):
    dp = H / 20 if dp is None else dp
    nu = (2.0 / 3.0) * Umax * H / Re          # Re on the bulk velocity
    P = base_params(2, dp, c0=c0, nu_l=nu, u_ref=Umax, obc_mode=obc_mode,
                    seed=seed)
    fluid = lattice2(0.0, L, 0.0, H, dp)
    ext = 4 * dp
    wall = np.concatenate([lattice2(-ext, L + ext, -3 * dp, 0.0, dp),
                           lattice2(-ext, L + ext, H, H + 3 * dp, dp)])
    Lb = 4 * dp
    inlet = Buffer(1, (0.0, H / 2, 0.0), _frame2(1.0, 0.0), Lb, (H / 2, 0.0),
                   0.5 * dp, vel_mode=VEL_PRESCRIBED, p_mode=P_EXTRAPOLATE,
                   profile=profile, u0=Umax, coef=tuple(coef),
                   ramp_time=ramp_time)
    outlet = Buffer(2, (L, H / 2, 0.0), _frame2(-1.0, 0.0), Lb, (H / 2, 0.0),
                    0.5 * dp, vel_mode=VEL_EXTRAPOLATE, p_mode=P_PRESCRIBED,
                    p_ob=p_out)
    # the outlet frame's transverse axis is -y; the profile is symmetric
    return _assemble(name, P, [inlet, outlet], fluid, wall, steps,
                     note=f"{L}Hx{H} channel dp={dp} Re={Re}")


def make_adjoint_channel(dp=None, seed=4, steps=100, n_coef=16, amp=0.1, length=20.0,
                         Umax=1.0):
    """length x H channel (H = 1), Re 200, started from the developed Poiseuille
    profile; inlet profile 4 Umax s(1-s) + sum a_m sin(m pi s) (s = y / H) with
    a_m ~ U[-amp, amp] (seeded), no start-up ramp.  Objective slab: 4dp just
    upstream of the outlet buffer; wall length: both walls over the length."""
    H = 1.0
    dp = H / 80 if dp is None else dp
    rng = np.random.default_rng(seed)
    coef = tuple(float(a) for a in rng.uniform(-amp, amp, n_coef))
    c = make_channel(H=H, L=length, dp=dp, Re=200.0, Umax=Umax, steps=steps,
                     profile=PROFILE_SINE, coef=coef, name="adjoint_channel",
                     seed=seed, ramp_time=0.0)
    fl = (c.tag & 3) != WALL
    y = c.x[fl, 1]
    c.v[fl, 0] = 4.0 * Umax * y * (H - y) / (H * H)
    Lb = 4 * dp
    c.objective = dict(slab_origin=(length - Lb - 4 * dp, 0.0, 0.0),
                       slab_normal=(1.0, 0.0, 0.0), slab_width=4 * dp,
                       shear_dir=(1.0, 0.0, 0.0), wall_length=2.0 * length)
    c.note = (f"{length}Hx{H} channel dp={dp} Re=200, developed start, "
              f"{n_coef} sine coefficients")
    return c


# ----------------------------------------------------------------------------
# 2D U-channel: two straight legs joined by a 180-degree bend of inner radius
# H; pressure inlet (p=1) on the lower leg, pressure outlet (p=0) on the upper
# leg, both open faces at x = 0.
# ----------------------------------------------------------------------------
def make_uchannel(dp=None, H=1.0, Lleg=13.275, p_in=1.0, Re=50.0, c0=10.0,
                  noise=1e-3, seed=1, steps=2000, ramp_time=5.0, inlet="velocity",
                  tvf_alpha=0.0):
    """U-channel with legs of length Lleg joined by a 180-degree bend.

    The driving pressure drop p_in sets the Poiseuille estimate of the mean
    velocity U (and so nu from Re).  inlet="velocity" prescribes that flow as a
    parabolic velocity inlet (mean U, ramped); inlet="pressure" prescribes
    p = p_in at the inlet buffer instead.  The outlet buffer has p = 0.
    """
    dp = H / 40 if dp is None else dp
    R_in = H
    cy = R_in + H                      # bend centre (Lleg, cy)
    # Poiseuille estimate: mean velocity U with Re = U H / nu and the
    # pressure drop over the centreline length balancing 12 mu U / H^2.
    Lpath = 2 * Lleg + math.pi * (R_in + H / 2)
    G = p_in / Lpath
    nu = math.sqrt(G * H * H / (12.0 * Re))
    U = Re * nu / H
    P = base_params(2, dp, c0=c0, nu_l=nu, u_ref=U, seed=seed)
    P["tvf_alpha"] = tvf_alpha
    ext = 4 * dp
    x0 = -ext
    span = lattice2(x0, Lleg + cy + H + 4 * dp, -4 * dp, 2 * cy + 4 * dp, dp)
    X, Y = span[:, 0], span[:, 1]
    r = np.hypot(X - Lleg, Y - cy)

    def region(dil, xmin):
        lower = (X >= xmin) & (X < Lleg) & (Y > -dil) & (Y < H + dil)
        upper = (X >= xmin) & (X < Lleg) & (Y > 2 * cy - H - dil) & \
            (Y < 2 * cy + dil)
        bend = (X >= Lleg) & (r > R_in - dil) & (r < R_in + H + dil)
        return lower | upper | bend

    fl = region(0.0, 0.0)
    fext = region(0.0, x0)
    wl = region(3 * dp, x0) & ~fext
    fluid, wall = span[fl], span[wl]
    rng = np.random.default_rng(seed)
    Umax = 1.5 * U
    v = np.zeros((fluid.shape[0], 3))
    v[:, :2] = noise * Umax * rng.uniform(-1.0, 1.0, (fluid.shape[0], 2))
    Lb = 4 * dp
    if inlet == "pressure":
        inb = Buffer(1, (0.0, H / 2, 0.0), _frame2(1.0, 0.0), Lb, (H / 2, 0.0),
                     0.5 * dp, vel_mode=VEL_EXTRAPOLATE, p_mode=P_PRESCRIBED,
                     p_ob=p_in, ramp_time=ramp_time)
    else:
        inb = Buffer(1, (0.0, H / 2, 0.0), _frame2(1.0, 0.0), Lb, (H / 2, 0.0),
                     0.5 * dp, vel_mode=VEL_PRESCRIBED, p_mode=P_EXTRAPOLATE,
                     profile=PROFILE_PARABOLIC, u0=Umax, ramp_time=ramp_time)
    outlet = Buffer(2, (0.0, 2 * cy - H / 2, 0.0), _frame2(1.0, 0.0), Lb,
                    (H / 2, 0.0), 0.5 * dp, vel_mode=VEL_EXTRAPOLATE,
                    p_mode=P_PRESCRIBED, p_ob=0.0)
    return _assemble("uchannel", P, [inb, outlet], fluid, wall, steps, v=v,
                     note=f"U-channel H={H} dp={dp} legs={Lleg} Re={Re} "
                          f"nu={nu:.4g} U_ref={U:.4g} {inlet} inlet")


# ----------------------------------------------------------------------------
# 2D turbulent plane jet in a compact 20D x 20D box with six buffers:
# 1 slot inlet, 2 outlet, 3/4 side inflow at zero velocity, 5/6 top/bottom
# far-field.  k-epsilon on; no walls.
# ----------------------------------------------------------------------------
def make_jet(dp=None, D=1.0, L=20.0, W=10.0, U=1.0, Re=1e4, c0=10.0,
             turb_int=0.05, mix_len=0.07, noise=0.05, seed=2, steps=5000, turbulence=1,
             tvf_alpha=0.2, corner_overhang=0.0, pad_cells=3, p_far=0.0):
    """Plane jet with the six buffers of Table 3 and the transport-velocity
    shift (tvf_alpha; without it the shear layers at the slot lips cavitate
    within about 500 steps).  p_far is the pressure of the outlet and the two
    far-field buffers (Table 3 names a far-field pressure without a value);
    the ambient starts at rest at that pressure.  corner_overhang widens the
    outlet buffer's transverse box past y = +-W (the corner cells it shares
    with the far-field buffers): a slow particle there that moves out through
    the top or bottom stays an outlet particle instead of turning into a
    fluid particle outside every buffer.  pad_cells widens the cell grid
    around the domain for long runs."""
    dp = D / 20 if dp is None else dp
    nu = U * D / Re
    P = base_params(2, dp, c0=c0, nu_l=nu, u_ref=U, turbulence=turbulence, seed=seed)
    P["tvf_alpha"] = tvf_alpha
    k_in = 1.5 * (turb_int * U) ** 2
    eps_in = P["Cmu"] ** 0.75 * k_in ** 1.5 / (mix_len * D)
    k_a, eps_a = 1e-3 * k_in, 1e-3 * eps_in
    fluid = lattice2(0.0, L, -W, W, dp)
    Lb = 4 * dp
    f = 0.5 * dp
    ex = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    b1 = Buffer(1, (0.0, 0.0, 0.0), ex, Lb, (D / 2, 0.0), f,
                vel_mode=VEL_PRESCRIBED, p_mode=P_EXTRAPOLATE,
                turb_mode=TURB_FREESTREAM, k_bc=k_in, eps_bc=eps_in,
                profile=PROFILE_UNIFORM, u0=U, noise_amp=noise)
    b2 = Buffer(2, (L, 0.0, 0.0), _frame2(-1.0, 0.0), Lb, (W + corner_overhang, 0.0), f,
                vel_mode=VEL_EXTRAPOLATE, p_mode=P_PRESCRIBED, p_ob=p_far)
    hw_side = (W - D / 2) / 2
    b3 = Buffer(3, (0.0, D / 2 + hw_side, 0.0), ex, Lb, (hw_side, 0.0), f,
                vel_mode=VEL_PRESCRIBED, p_mode=P_EXTRAPOLATE,
                turb_mode=TURB_FREESTREAM, k_bc=k_a, eps_bc=eps_a,
                profile=PROFILE_UNIFORM, u0=0.0)
    b4 = dataclasses.replace(b3, id=4, origin=(0.0, -(D / 2 + hw_side), 0.0))
    hw_tb = L / 2 - Lb
    b5 = Buffer(5, (L / 2, W, 0.0), _frame2(0.0, -1.0), Lb, (hw_tb, 0.0), f,
                vel_mode=VEL_EXTRAPOLATE, p_mode=P_PRESCRIBED, p_ob=p_far)
    b6 = Buffer(6, (L / 2, -W, 0.0), _frame2(0.0, 1.0), Lb, (hw_tb, 0.0), f,
                vel_mode=VEL_EXTRAPOLATE, p_mode=P_PRESCRIBED, p_ob=p_far)
    wall = np.zeros((0, 3))
    c = _assemble("jet", P, [b1, b2, b3, b4, b5, b6], fluid, wall, steps,
                  k0=k_a, eps0=eps_a, pad_cells=pad_cells,
                  note=f"plane jet D={D} {L}x{2 * W} dp={dp} Re={Re:g} "
                       f"k_in={k_in:.4g} eps_in={eps_in:.4g}")
    if p_far:
        c.rho[:] = P["rho0"] * (1.0 + p_far / (P["rho0"] * c0 * c0))
    return c


def make_laminar_jet(nf=10, Re=40.0, tvf_alpha=0.2, steps=20000, seed=2, p_far=0.0):
    """Laminar plane jet of Sec. 4.3: slot width D = 2, domain 40 D long and
    2 x 20 D wide, nf particles across the slot, uniform inlet speed 1, the
    six buffers of Table 3, no inlet noise, with the transport-velocity
    shift (particle regularity in the low-pressure shear layers at the slot
    lips and in the outlet buffer's backflow).  The grid is padded for runs
    of some 10^4 steps."""
    D = 2.0
    dp = D / nf
    return make_jet(dp=dp, D=D, L=40 * D, W=20 * D, U=1.0, Re=Re, noise=0.0, seed=seed,
                    steps=steps, turbulence=0, tvf_alpha=tvf_alpha, pad_cells=20, p_far=p_far)


# ----------------------------------------------------------------------------
# 3D self-rotating micro-mixer: cylinder (diameter 1, height 0.5), four
# tangential square inlets (side 0.1) with uniform velocity buffers, one axial
# circular outlet (diameter 0.2) with a p=0 buffer.
# ----------------------------------------------------------------------------
def make_mixer(dp=0.005, R=0.5, Hc=0.5, a=0.1, Lin=0.2, r_out=0.1,
               L_out=0.2, U=1.0, Re=50.0, c0=10.0, seed=3, steps=500):
    nu = U * a / Re
    P = base_params(3, dp, c0=c0, nu_l=nu, u_ref=U, seed=seed)
    rc = R - a / 2                    # inlet centre line distance to the axis
    s_face = math.sqrt(R * R - (R - a) ** 2) + Lin
    ext = 4 * dp
    wall_t = 3 * dp
    lim = R + s_face + ext + wall_t + dp
    zmin, zmax = -wall_t - dp, Hc + L_out + ext + wall_t + dp
    i0, i1 = int(math.floor(-lim / dp)), int(math.ceil(lim / dp))
    k0, k1 = int(math.floor(zmin / dp)), int(math.ceil(zmax / dp))
    xs = (np.arange(i0, i1) + 0.5) * dp
    zs = (np.arange(k0, k1) + 0.5) * dp
    fluid_parts, wall_parts = [], []
    thetas = [0.5 * math.pi * q for q in range(4)]
    for z in zs:                       # slab by slab to bound memory
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        X, Y = X.ravel(), Y.ravel()
        rr = np.hypot(X, Y)

        def region(dil, extend):
            zz = z
            cham = (rr < R + dil) & (zz > -dil) & (zz < Hc + dil)
            top = Hc + L_out + (ext if extend else 0.0)
            outl = (rr < r_out + dil) & (zz >= Hc - dil) & (zz < top + dil)
            m = cham | outl
            for th in thetas:
                c = np.array([rc * math.cos(th), rc * math.sin(th)])
                d = np.array([-math.sin(th), math.cos(th)])
                nrm = np.array([math.cos(th), math.sin(th)])
                rel0, rel1 = X - c[0], Y - c[1]
                s = -(rel0 * d[0] + rel1 * d[1])      # distance behind c
                t = rel0 * nrm[0] + rel1 * nrm[1]
                smax = s_face + (ext if extend else 0.0)
                m |= (s >= -dil) & (s < smax + (dil if not extend else 0.0)) \
                    & (np.abs(t) < a / 2 + dil) & (zz > -dil) & (zz < a + dil)
            return m

        fl = region(0.0, False)
        fe = region(0.0, True)
        wl = region(wall_t, True) & ~fe
        if fl.any():
            fluid_parts.append(np.stack([X[fl], Y[fl], np.full(fl.sum(), z)], 1))
        if wl.any():
            wall_parts.append(np.stack([X[wl], Y[wl], np.full(wl.sum(), z)], 1))
    fluid = np.concatenate(fluid_parts)
    wall = np.concatenate(wall_parts)
    Lb = 4 * dp
    bufs = []
    for q, th in enumerate(thetas):
        c = np.array([rc * math.cos(th), rc * math.sin(th), a / 2])
        d = np.array([-math.sin(th), math.cos(th), 0.0])
        nrm = np.array([math.cos(th), math.sin(th), 0.0])
        o = c - s_face * d
        bufs.append(Buffer(q + 1, tuple(o), (tuple(d), tuple(nrm),
                                             (0.0, 0.0, 1.0)),
                           Lb, (a / 2, a / 2), 0.5 * dp,
                           vel_mode=VEL_PRESCRIBED, p_mode=P_EXTRAPOLATE,
                           profile=PROFILE_UNIFORM, u0=U))
    bufs.append(Buffer(5, (0.0, 0.0, Hc + L_out),
                       ((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)),
                       Lb, (r_out, r_out), 0.5 * dp, vel_mode=VEL_EXTRAPOLATE,
                       p_mode=P_PRESCRIBED, p_ob=0.0))
    return _assemble("mixer", P, bufs, fluid, wall, steps,
                     note=f"3D mixer dp={dp} R={R} Hc={Hc} inlets 4x{a} "
                          f"outlet r={r_out} Re={Re}")


def make_duct3d(dp=0.05, L=1.0, H=0.5, W=0.3, Umax=1.0, Re=100.0, c0=10.0, seed=5,
                steps=20, n_coef=16, amp=0.1):
    """3D rectangular duct along x (L x H x W), three wall layers on the four
    side faces, SINE-profile velocity inlet at x = 0 (s = y / H; the profile
    has no z factor) with a_m ~ U[-amp, amp] (seeded), zero-pressure outlet at
    x = L, started from u = 4 Umax s (1 - s), no start-up ramp; objective slab
    4dp upstream of the outlet buffer, wall area 2 (H + W) L."""
    nu = Umax * H / Re
    P = base_params(3, dp, c0=c0, nu_l=nu, u_ref=Umax, seed=seed)
    ext = 4 * dp
    wt = 3 * dp

    def lattice3(x0, x1, y0, y1, z0, z1):
        xs = (np.arange(int(round(x0 / dp)), int(round(x1 / dp))) + 0.5) * dp
        ys = (np.arange(int(round(y0 / dp)), int(round(y1 / dp))) + 0.5) * dp
        zs = (np.arange(int(round(z0 / dp)), int(round(z1 / dp))) + 0.5) * dp
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)

    fluid = lattice3(0.0, L, 0.0, H, 0.0, W)
    box = lattice3(-ext, L + ext, -wt, H + wt, -wt, W + wt)
    inner = (box[:, 1] > 0.0) & (box[:, 1] < H) & (box[:, 2] > 0.0) & (box[:, 2] < W)
    wall = box[~inner]
    rng = np.random.default_rng(seed)
    coef = tuple(float(a) for a in rng.uniform(-amp, amp, n_coef))
    Lb = 4 * dp
    frame = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    inlet = Buffer(1, (0.0, H / 2, W / 2), frame, Lb, (H / 2, W / 2), 0.5 * dp,
                   vel_mode=VEL_PRESCRIBED, p_mode=P_EXTRAPOLATE, profile=PROFILE_SINE,
                   u0=Umax, coef=coef, ramp_time=0.0)
    outlet = Buffer(2, (L, H / 2, W / 2), ((-1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)),
                    Lb, (H / 2, W / 2), 0.5 * dp, vel_mode=VEL_EXTRAPOLATE,
                    p_mode=P_PRESCRIBED, p_ob=0.0)
    s_ = fluid[:, 1] / H
    v = np.zeros((fluid.shape[0], 3))
    v[:, 0] = 4.0 * Umax * s_ * (1.0 - s_)
    c = _assemble("duct3d", P, [inlet, outlet], fluid, wall, steps, v=v,
                  note=f"3D duct {L}x{H}x{W} dp={dp} Re={Re}, sine inlet")
    c.objective = dict(slab_origin=(L - Lb - 4 * dp, 0.0, 0.0), slab_normal=(1.0, 0.0, 0.0),
                       slab_width=4 * dp, shear_dir=(1.0, 0.0, 0.0),
                       wall_length=2.0 * (H + W) * L)
    return c


def jittered(case: Case, amp: float, seed: int = 7) -> Case:
    """Copy of ``case`` with fluid positions jittered by amp*dp (uniform)."""
    rng = np.random.default_rng(seed)
    c = dataclasses.replace(case, x=case.x.copy(), v=case.v.copy(),
                            rho=case.rho.copy(), k=case.k.copy(),
                            eps=case.eps.copy(),
                            tag=case.tag.copy(), pid=case.pid.copy(),
                            params=dict(case.params))
    fl = (c.tag & 3) != WALL
    dim = c.params["dim"]
    c.x[fl, :dim] += amp * c.params["dp"] * rng.uniform(-1, 1,
                                                          (fl.sum(), dim))
    return c


def perturbed_state(case: Case, seed: int = 11, dv=0.05, drho=0.01,
                    dk=0.2) -> Case:
    """Copy of ``case`` with seeded velocity, density and k/eps fields, so
    that every pair term of a rate evaluation is exercised."""
    rng = np.random.default_rng(seed)
    c = jittered(case, 0.1, seed + 1)
    fl = (c.tag & 3) != WALL
    nf = int(fl.sum())
    dim = c.params["dim"]
    c.v[fl, :dim] = dv * rng.uniform(-1, 1, (nf, dim)) * c.params["u_ref"]
    c.rho[fl] = c.params["rho0"] * (1.0 + drho * rng.uniform(-1, 1, nf))
    if c.params["turbulence"]:
        c.k[fl] *= 1.0 + dk * rng.uniform(-1, 1, nf)
        c.eps[fl] *= 1.0 + dk * rng.uniform(-1, 1, nf)
    return c


WORKLOADS = {
    "channel": make_channel,
    "uchannel": make_uchannel,
    "jet": make_jet,
    "mixer": make_mixer,
    "adjoint_channel": make_adjoint_channel,
}
