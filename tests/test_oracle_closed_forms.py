"""Pins of the oracle parts that the operator tests leave open: the k and
epsilon diffusion sums (Eqs. (k-discretized-equ), (epsilon-discretized-equ)),
the guarded inverse of the correction moment (Eq. (equ-B-matrix) with the
singular-support reading), the dual-criteria time step (Sec. 2.3), the
effective pressure p + 2/3 rho k (Table 1) and the prescribed inlet profiles
(Table 3, Sec. 2.4.2).

Every expected value comes from mathematics outside the oracle: Taylor
moments of a lattice (the diffusion sum of a quadratic field is its second
derivative times the kernel moment A = B^-1), exactness of the corrected
pressure gradient for linear fields, a conservation law, limits of the
harmonic mean, textbook parabolas and the cosine ramp, and brute-force
moments of crafted supports.
"""
import dataclasses

import numpy as np
import pytest

import cases
from tests.helpers import block_case, interior_mask


def _sim(ora, case):
    return ora.OracleSim(case, threads=4)


def _moment(Bm, i, dim):
    return np.linalg.inv(Bm[i].reshape(3, 3)[:dim, :dim])


def _with_params(case, **kw):
    p = dict(case.params)
    p.update(kw)
    return dataclasses.replace(case, params=p)


# --------------------------------------------------------------------------
# k / epsilon diffusion (Eqs. k-discretized-equ, epsilon-discretized-equ)
# --------------------------------------------------------------------------
# On a full lattice the odd kernel moments vanish, so for any field phi the
# pair sum S_i = sum_j V_j f_ij (phi_i - phi_j) of a quadratic phi is
# -phi''/2 sum_j V_j f_ij r_y^2 = (phi''/2) A_yy (A = B^-1, the moment of
# Eq. equ-B-matrix): the discrete diffusion of a quadratic field equals the
# continuous one, D phi'' A_yy (2 / rho) with A ~ I.  Linear fields diffuse
# nothing.  With v = 0 the production G_k vanishes, so dk = -eps + diff_k and
# deps = -C2 eps^2 / k + diff_eps.

def _interior(c, n_side, dp, margin):
    return np.where(interior_mask(c.x, (0, 0), (n_side * dp, n_side * dp), margin))[0]


def test_keps_diffusion_of_quadratic_fields_with_molecular_viscosity(ora):
    # C_mu = 0: nu_t = 0 everywhere, D_k = D_eps = nu_l uniform; k quadratic in
    # y plus a linear part in x, eps quadratic in x plus a linear part in y.
    n_side, dp = 14, 0.1
    c = block_case(dim=2, n_side=n_side, dp=dp, turbulence=1, nu_l=2e-2)
    c = _with_params(c, Cmu=0.0)
    x, y = c.x[:, 0], c.x[:, 1]
    a, b = 0.7, 0.3
    c.k = 0.05 + a * y * y + 0.02 * x
    c.eps = 0.04 + b * x * x - 0.01 * y
    s = _sim(ora, c)
    Bm, _ = s.correction(mirror=False)
    r = s.rates(Bm)
    nu = c.params["nu_l"]
    inner = _interior(c, n_side, dp, 0.35)
    assert inner.size > 20
    for i in inner:
        A = _moment(Bm, i, 2)
        exp_k = 2.0 / s.rho[i] * nu * a * A[1, 1]
        exp_e = 2.0 / s.rho[i] * nu * b * A[0, 0]
        diff_k = r["dk"][i] + c.eps[i]
        diff_e = r["deps"][i] + c.params["C2"] * c.eps[i] ** 2 / c.k[i]
        assert abs(diff_k - exp_k) < 1e-11 * exp_k
        assert abs(diff_e - exp_e) < 1e-11 * exp_e
        # the continuous limit: A ~ I on the h = 1.3 dp lattice
        assert abs(diff_k / (2.0 * nu * a) - 1.0) < 0.03


def test_k_diffusion_coefficient_carries_sigma_k(ora):
    # uniform nu_t (eps = C_mu k^2 / nu_t0) with k = k0 + a y^2:
    # diff_k = (2 / rho) (nu_l + nu_t0 / sigma_k) a A_yy.  sigma_k = 1.7 here
    # (Table A has 1.0, where a missing division would not show).
    n_side, dp = 14, 0.1
    c = block_case(dim=2, n_side=n_side, dp=dp, turbulence=1, nu_l=1e-3)
    c = _with_params(c, sigma_k=1.7)
    nut0, a = 4e-3, 0.8
    y = c.x[:, 1]
    c.k = 0.02 + a * y * y
    c.eps = c.params["Cmu"] * c.k ** 2 / nut0
    s = _sim(ora, c)
    Bm, _ = s.correction(mirror=False)
    r = s.rates(Bm)
    Dk = c.params["nu_l"] + nut0 / 1.7
    inner = _interior(c, n_side, dp, 0.35)
    for i in inner:
        A = _moment(Bm, i, 2)
        exp = 2.0 / s.rho[i] * Dk * a * A[1, 1]
        assert abs(r["dk"][i] + c.eps[i] - exp) < 1e-11 * exp


def test_linear_k_does_not_diffuse_and_eps_diffusion_carries_sigma_eps(ora):
    # uniform nu_t with k = k0 + g y (linear): no k diffusion; then
    # eps = (C_mu / nu_t0) k^2 is quadratic with eps'' = 2 (C_mu / nu_t0) g^2
    # and diff_eps = (2 / rho) (nu_l + nu_t0 / sigma_eps) (eps'' / 2) A_yy.
    n_side, dp = 14, 0.1
    c = block_case(dim=2, n_side=n_side, dp=dp, turbulence=1, nu_l=1e-3)
    nut0, g = 5e-3, 0.06
    Cmu, C2, se = c.params["Cmu"], c.params["C2"], c.params["sigma_eps"]
    c.k = 0.03 + g * c.x[:, 1]
    c.eps = Cmu * c.k ** 2 / nut0
    s = _sim(ora, c)
    Bm, _ = s.correction(mirror=False)
    r = s.rates(Bm)
    De = c.params["nu_l"] + nut0 / se
    inner = _interior(c, n_side, dp, 0.35)
    for i in inner:
        A = _moment(Bm, i, 2)
        assert abs(r["dk"][i] + c.eps[i]) < 1e-12 * c.eps[i]
        exp = 2.0 / s.rho[i] * De * (Cmu / nut0) * g * g * A[1, 1]
        diff_e = r["deps"][i] + C2 * c.eps[i] ** 2 / c.k[i]
        assert abs(diff_e - exp) < 1e-10 * exp


def test_keps_diffusion_conserves_total_k_and_eps(ora):
    # With a symmetric pair coefficient the diffusion sums are antisymmetric in
    # (i, j): sum_i V_i rho_i diff_i = 2 sum_i sum_j V_i V_j D_ij (phi_i -
    # phi_j) f_ij = 0 for any cloud and any non-uniform nu_t.  A coefficient
    # that depended on i or j alone would break it.
    c = block_case(dim=2, n_side=12, dp=0.1, jitter=0.3, seed=3, turbulence=1)
    rng = np.random.default_rng(5)
    c.k = 1e-3 * (1.0 + rng.uniform(0, 4, c.n))
    c.eps = 1e-3 * (1.0 + rng.uniform(0, 4, c.n))
    c.rho = 1.0 + 0.005 * rng.uniform(-1, 1, c.n)
    s = _sim(ora, c)
    r = s.rates()
    P = c.params
    V = r["vol"]
    diff_k = r["dk"] + c.eps
    diff_e = r["deps"] + P["C2"] * c.eps ** 2 / c.k
    for d in (diff_k, diff_e):
        tot = np.sum(V * c.rho * d)
        assert abs(tot) < 1e-13 * np.sum(np.abs(V * c.rho * d))
        assert np.abs(d).max() > 0.0


def test_keps_diffusion_uses_the_harmonic_mean(ora):
    # Two particles, j nearly inviscid (nu_l ~ 0, nu_t,j ~ 1e-13): the
    # harmonic mean 2 D_i D_j / (D_i + D_j) -> 2 D_j ~ 0, so k and eps barely
    # diffuse into i although D_i is large (an arithmetic mean would give
    # about D_i / 2).
    c = block_case(dim=2, n_side=2, dp=0.1, turbulence=1, nu_l=1e-14)
    x = np.array([[1.0, 1.0, 0.0], [1.1, 1.0, 0.0]])
    c = dataclasses.replace(c, x=x, v=np.zeros((2, 3)), rho=np.ones(2),
                            k=np.array([1e-2, 1e-6]), eps=np.array([1e-3, 1.0]),
                            tag=np.zeros(2, np.uint32), pid=np.arange(2, dtype=np.uint32))
    cases._set_bounds(c.params, x)
    r = _sim(ora, c).rates()
    P = c.params
    diff_k = r["dk"][0] + c.eps[0]
    nut_i = P["Cmu"] * c.k[0] ** 2 / c.eps[0]
    f = ora.kernel_dW(0.1, P["h"], 2) / 0.1
    arith = 2.0 * (0.5 * nut_i) * (c.k[0] - c.k[1]) * f * r["vol"][1]
    assert abs(arith) > 1e-6
    assert abs(diff_k) < 1e-8 * abs(arith)


# --------------------------------------------------------------------------
# guarded inverse of the correction moment (Eq. equ-B-matrix; singular and
# nearly singular supports)
# --------------------------------------------------------------------------
def _star_case(dim, arms, dp=0.1):
    """Particle 0 at the centre of a star: for each axis k, two neighbours at
    +-arms[k] * h (arms[k] = 0: none on that axis)."""
    c = block_case(dim=dim, n_side=2, dp=dp)
    h = c.params["h"]
    ctr = np.array([1.0, 1.0, 0.0 if dim == 2 else 1.0])
    pts = [ctr.copy()]
    for k in range(dim):
        if arms[k] > 0:
            for sgn in (1.0, -1.0):
                p = ctr.copy()
                p[k] += sgn * arms[k] * h
                pts.append(p)
    x = np.array(pts)
    n = x.shape[0]
    c = dataclasses.replace(c, x=x, v=np.zeros((n, 3)), rho=np.ones(n), k=np.zeros(n),
                            eps=np.zeros(n), tag=np.zeros(n, np.uint32),
                            pid=np.arange(n, dtype=np.uint32))
    cases._set_bounds(c.params, x)
    return c


def _brute_moment(ora, c, i):
    """A_i = -sum_j V_j r_ij (x) r_ij W'(r) / r by brute force (V = dp^dim at
    rho0 = 1)."""
    dim, h, dp = c.params["dim"], c.params["h"], c.params["dp"]
    A = np.zeros((dim, dim))
    for j in range(c.n):
        if j == i:
            continue
        r = (c.x[i] - c.x[j])[:dim]
        rr = np.linalg.norm(r)
        if rr >= 2.0 * h:
            continue
        A -= dp ** dim * np.outer(r, r) * ora.kernel_dW(rr, h, dim) / rr
    return A


@pytest.mark.parametrize("dim", [2, 3])
def test_isolated_and_collinear_supports_give_identity(ora, dim):
    # no neighbour: A = 0; neighbours on one line: rank-one A, det = 0
    for arms in ([0.0] * dim, [1.0] + [0.0] * (dim - 1)):
        c = _star_case(dim, arms)
        Bm, _ = _sim(ora, c).correction(mirror=False)
        eye = np.eye(3)
        if dim == 2:
            eye[2, 2] = 0.0
        assert np.abs(Bm[0].reshape(3, 3) - eye).max() == 0.0


@pytest.mark.parametrize("dim,arms", [(2, (1.0, 1.8)), (2, (1.0, 1.75)),
                                      (3, (1.0, 1.0, 1.78))])
def test_nearly_singular_support_blends_inverse_with_identity(ora, dim, arms):
    # d = det A / (tr A / dim)^dim below 0.25: B = w A^-1 + (1 - w) I with
    # w = (d / 0.25)^2 -- the reading of the guard, with A from brute force
    c = _star_case(dim, arms)
    A = _brute_moment(ora, c, 0)
    d = np.linalg.det(A) / (np.trace(A) / dim) ** dim
    assert 0.0 < d < 0.25
    w = (d / 0.25) ** 2
    exp = w * np.linalg.inv(A) + (1.0 - w) * np.eye(dim)
    Bm, _ = _sim(ora, c).correction(mirror=False)
    B = Bm[0].reshape(3, 3)[:dim, :dim]
    assert np.abs(B - exp).max() < 1e-10 * np.abs(exp).max()
    # a blended B is no longer the inverse of the moment
    assert np.abs(B @ A - np.eye(dim)).max() > 0.1


@pytest.mark.parametrize("dim,arms", [(2, (1.0, 1.2)), (3, (1.0, 1.1, 1.2))])
def test_healthy_anisotropic_support_gives_exact_inverse(ora, dim, arms):
    c = _star_case(dim, arms)
    A = _brute_moment(ora, c, 0)
    d = np.linalg.det(A) / (np.trace(A) / dim) ** dim
    assert d >= 0.25
    Bm, _ = _sim(ora, c).correction(mirror=False)
    B = Bm[0].reshape(3, 3)[:dim, :dim]
    assert np.abs(B @ A - np.eye(dim)).max() < 1e-12


# --------------------------------------------------------------------------
# dual-criteria time step (Sec. 2.3)
# --------------------------------------------------------------------------
def _dt_case(v_fast, k_fluid, eps_fluid, wall_v=100.0, wall_nut_k=None):
    c = block_case(dim=2, n_side=8, dp=0.1, turbulence=1, walls=True, nu_l=1e-3)
    fl = np.where((c.tag & 3) == 0)[0]
    wl = np.where((c.tag & 3) == 2)[0]
    c.v = np.zeros((c.n, 3))
    c.v[fl, 0] = 0.1
    c.v[fl[17], :2] = v_fast
    c.v[wl[3], 0] = wall_v                 # walls do not enter the criteria
    c.k = np.zeros(c.n)
    c.eps = np.zeros(c.n)
    c.k[fl], c.eps[fl] = 1e-4, 1e-2
    c.k[fl[5]], c.eps[fl[5]] = k_fluid, eps_fluid
    if wall_nut_k is not None:
        c.k[wl[0]], c.eps[wl[0]] = wall_nut_k, 1e-6
    return c


def test_time_step_is_advection_limited_by_the_fastest_particle(ora):
    c = _dt_case((3.0, 4.0), 1e-4, 1e-2, wall_nut_k=10.0)
    P = c.params
    I = _sim(ora, c).time_step()
    h, vmax = P["h"], 5.0
    assert abs(I.vmax - vmax) < 1e-15
    assert I.dt_adv == pytest.approx(0.25 * h / vmax, rel=1e-15)
    assert I.dt_ac == pytest.approx(0.6 * h / (P["c0"] + vmax), rel=1e-15)
    # every acoustic sub-step keeps the acoustic CFL number, and no fewer
    # sub-steps would
    n = I.n_ac
    assert n == 2
    assert (I.dt_adv / n) * (P["c0"] + vmax) / h <= 0.6 * (1 + 1e-15)
    assert (I.dt_adv / (n - 1)) * (P["c0"] + vmax) / h > 0.6


def test_time_step_is_viscosity_limited_by_the_largest_eddy_viscosity(ora):
    # nu_t = C_mu k^2 / eps = 0.09 * 1 / 1e-3 = 90 at one fluid particle
    c = _dt_case((0.3, 0.0), 1.0, 1e-3)
    P = c.params
    nu = P["nu_l"] + P["Cmu"] * 1.0 / 1e-3
    I = _sim(ora, c).time_step()
    h = P["h"]
    assert I.numax == pytest.approx(nu, rel=1e-15)
    assert I.dt_adv == pytest.approx(0.25 * h * h / (2.0 * nu), rel=1e-15)
    assert I.n_ac == 1


def test_time_step_uses_the_reference_speed_below_it(ora):
    c = _dt_case((0.3, 0.4), 1e-4, 1e-2)
    P = c.params
    I = _sim(ora, c).time_step()
    h = P["h"]
    assert I.vmax == pytest.approx(0.5, rel=1e-15)
    assert I.dt_adv == pytest.approx(0.25 * h / P["u_ref"], rel=1e-15)
    assert I.dt_ac == pytest.approx(0.6 * h / (P["c0"] + 0.5), rel=1e-15)
    assert I.n_ac == int(np.ceil(I.dt_adv / I.dt_ac)) == 5


def test_time_step_counts_buffer_particles(ora):
    # buffer particles are real: their speed enters the criteria
    c = _dt_case((0.3, 0.0), 1e-4, 1e-2)
    fl = np.where((c.tag & 3) == 0)[0]
    c.tag = c.tag.copy()
    c.tag[fl[40]] = cases.make_tag(cases.BUFFER, 7)
    c.v[fl[40], :2] = (0.0, -2.0)
    I = _sim(ora, c).time_step()
    assert I.vmax == pytest.approx(2.0, rel=1e-15)


# --------------------------------------------------------------------------
# effective pressure p + 2/3 rho k (Table 1)
# --------------------------------------------------------------------------
def test_effective_pressure_adds_two_thirds_rho_k(ora):
    c = block_case(dim=2, n_side=6, dp=0.1, turbulence=1)
    rng = np.random.default_rng(2)
    c.rho = 1.0 + 0.004 * rng.uniform(-1, 1, c.n)
    c.k = 0.05 * (1.0 + rng.uniform(0, 1, c.n))
    c.eps = np.full(c.n, 1e-2)
    P = c.params
    r = _sim(ora, c).rates()
    lam = dataclasses.replace(c, params={**c.params, "turbulence": 0})
    r0 = _sim(ora, lam).rates()
    # laminar: the linear equation of state p = rho0 c0^2 (rho / rho0 - 1)
    assert np.allclose(r0["p"], P["c0"] ** 2 * (c.rho - 1.0), rtol=1e-12, atol=1e-15)
    assert np.allclose(r["p"] - r0["p"], 2.0 / 3.0 * c.rho * c.k, rtol=1e-12, atol=1e-16)


def test_turbulent_kinetic_energy_gradient_drives_the_pressure_force(ora):
    # rho = rho0 (no acoustic pressure), v = 0, k = k0 + g y: p_eff = 2/3 rho0 k
    # is linear, and the corrected pair sum of Eq. (eq-discretize-momentum-p-
    # RKGC) is exact for a linear pressure where every neighbour shares the
    # particle's B (lattice interior, 4h from the edges):
    # a_p = -grad p_eff / rho = -(2/3) g e_y.
    n_side, dp = 18, 0.1
    c = block_case(dim=2, n_side=n_side, dp=dp, turbulence=1)
    g = 0.4
    c.k = 0.05 + g * c.x[:, 1]
    c.eps = np.full(c.n, 1e-2)
    s = _sim(ora, c)
    r = s.rates()
    h = c.params["h"]
    inner = _interior(c, n_side, dp, 4.0 * h)
    assert inner.size >= 16
    ap = r["ap"][inner]
    assert np.abs(ap[:, 1] + 2.0 / 3.0 * g).max() < 1e-11
    assert np.abs(ap[:, 0]).max() < 1e-11


# --------------------------------------------------------------------------
# prescribed inlet profiles (Table 3, Sec. 2.4.2: buffer boundary values)
# --------------------------------------------------------------------------
def _frame3_rotated():
    n = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    t1 = np.array([-1.0, 1.0, 0.0]) / np.sqrt(2.0)
    t2 = np.array([0.0, 0.0, 1.0])
    return n, t1, t2


def _profile_case(dim, profile, s_t, u0=1.3, coef=(), ramp=0.0, t=0.0, noise=0.0, seed=0):
    """Buffer particles of one prescribed-velocity buffer placed at local
    coordinates (y0 = L/2, s, t): s, t in [0, 1] across the two transverse
    widths."""
    dp = 0.05
    P = cases.base_params(dim, dp, seed=seed)
    if dim == 3:
        n, t1, t2 = _frame3_rotated()
    else:
        n = np.array([np.cos(0.3), np.sin(0.3), 0.0])
        t1 = np.array([-n[1], n[0], 0.0])
        t2 = np.array([0.0, 0.0, 1.0])
    hw = (0.2, 0.15)
    org = np.array([1.0, 1.0, 1.0 if dim == 3 else 0.0])
    L = 4 * dp
    b = cases.Buffer(3, tuple(org), (tuple(n), tuple(t1), tuple(t2)), L, hw, 0.5 * dp,
                     vel_mode=cases.VEL_PRESCRIBED, profile=profile, u0=u0,
                     coef=tuple(coef), ramp_time=ramp, noise_amp=noise)
    pts = []
    for (s, tt) in s_t:
        y1 = (2.0 * s - 1.0) * hw[0]
        y2 = (2.0 * tt - 1.0) * hw[1] if dim == 3 else 0.0
        pts.append(org + 0.5 * L * n + y1 * t1 + y2 * t2)
    fluid = np.array(pts)
    c = cases._assemble("profile", P, [b], fluid, np.zeros((0, 3)), 1)
    c.tag[:] = cases.make_tag(cases.BUFFER, 3)
    c.t = t
    return c, n


def _apply_bc(ora, c):
    s = _sim(ora, c)
    s.velocity_bc()
    return s.v[:s.n]


def test_parabolic_inlet_profile_3d_is_the_product_of_two_parabolas(ora):
    # u = u0 16 s (1 - s) t (1 - t) along n_b: u0 at the centre, 0 on the box
    # edges; values at quarter points are products of 3/4
    st = [(0.5, 0.5), (0.25, 0.5), (0.5, 0.75), (0.25, 0.25), (0.0, 0.5), (0.5, 1.0),
          (0.75, 0.25), (0.1, 0.9)]
    exp = [1.0, 0.75, 0.75, 0.5625, 0.0, 0.0, 0.5625, 0.36 * 0.36]
    c, n = _profile_case(3, cases.PROFILE_PARABOLIC, st)
    v = _apply_bc(ora, c)
    u0 = 1.3
    for q, e in enumerate(exp):
        assert np.abs(v[q] - u0 * e * n).max() < 1e-14


def test_parabolic_and_sine_inlet_profiles_2d(ora):
    st = [(0.5, 0), (0.25, 0), (0.0, 0), (0.9, 0)]
    c, n = _profile_case(2, cases.PROFILE_PARABOLIC, st)
    v = _apply_bc(ora, c)
    for q, e in enumerate([1.0, 0.75, 0.0, 0.36]):
        assert np.abs(v[q] - 1.3 * e * n).max() < 1e-14
    # parabola + a_1 sin(pi s) + a_2 sin(2 pi s): at s = 1/2 the second mode
    # vanishes, at s = 1/4 both are sin(pi/4) and sin(pi/2)
    c, n = _profile_case(2, cases.PROFILE_SINE, [(0.5, 0), (0.25, 0)], coef=(0.1, 0.05))
    v = _apply_bc(ora, c)
    assert np.abs(v[0] - (1.3 + 0.1) * n).max() < 1e-14
    e1 = 1.3 * 0.75 + 0.1 * np.sqrt(0.5) + 0.05
    assert np.abs(v[1] - e1 * n).max() < 1e-14


def test_inlet_ramp_and_noise(ora):
    # ramp 0.5 (1 - cos(pi t / T)): 1/4 at t = T/3, 1/2 at T/2, 1 after T
    for t, f in ((2.0, 0.25), (3.0, 0.5), (7.0, 1.0)):
        c, n = _profile_case(2, cases.PROFILE_UNIFORM, [(0.3, 0)], ramp=6.0, t=t)
        v = _apply_bc(ora, c)
        assert np.abs(v[0] - 1.3 * f * n).max() < 1e-14
    # noise: u0 (1 + a U), U the counter-based uniform of (seed, pid, step, 0)
    c, n = _profile_case(2, cases.PROFILE_UNIFORM, [(0.3, 0), (0.6, 0)], noise=0.05, seed=9)
    v = _apply_bc(ora, c)
    for q in range(2):
        u = 1.3 * (1.0 + 0.05 * ora.uniform(9, int(c.pid[q]), 0, 0))
        assert np.abs(v[q] - u * n).max() < 1e-14
