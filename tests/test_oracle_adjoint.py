"""Pins of the oracle's sensitivity reference: the objectives (slab mass flux
and mean wall shear stress) and the central finite differences of their
step averages with respect to the inlet-profile coefficients, with the
run's events (time steps, buffer decisions, slab membership) frozen.

Expected values come from closed forms: the midpoint rule of the Poiseuille
profile for the flux, the analytic wall shear 4 mu Umax / H for the wall
force (within the dummy-wall discretisation error, shrinking with dp), and
the exact derivative of the prescribed inlet velocity for a slab that holds
only inlet-buffer particles.
"""
import math

import numpy as np
import pytest

import cases

WALL = cases.WALL


def poiseuille_channel(dp, L=2.0, uniform=None):
    c = cases.make_channel(H=1.0, L=L, dp=dp, Re=100.0)
    fl = (c.tag & 3) != WALL
    y = c.x[fl, 1]
    c.v[fl, 0] = 4.0 * y * (1.0 - y) if uniform is None else uniform
    return c


def slab(x0, w, L):
    return dict(slab_origin=(x0, 0.0, 0.0), slab_normal=(1.0, 0.0, 0.0), slab_width=w,
                shear_dir=(1.0, 0.0, 0.0), wall_length=2.0 * L)


@pytest.mark.parametrize("dp", [1 / 20, 1 / 40])
def test_flux_uniform_flow_is_rho_u_h(ora, dp):
    # a slab 4dp wide over the full height holds 4 * (H / dp) particles
    c = poiseuille_channel(dp, uniform=0.75)
    J, mem = ora.OracleSim(c).objective(slab(1.0 + 1e-9, 4 * dp, 2.0))
    assert abs(J[0] - 1.0 * 0.75 * 1.0) < 1e-12
    assert int(mem.sum()) == 4 * round(1.0 / dp)


@pytest.mark.parametrize("dp", [1 / 20, 1 / 40, 1 / 80])
def test_flux_poiseuille_equals_midpoint_rule(ora, dp):
    # rows at y = (j + 1/2) dp: the midpoint rule of int 4 y (1 - y) dy is
    # 2/3 + dp^2 / 3 exactly (its error is -dp^2/24 int u'' dy)
    c = poiseuille_channel(dp)
    J, _ = ora.OracleSim(c).objective(slab(1.0 + 1e-9, 4 * dp, 2.0))
    assert abs(J[0] - (2.0 / 3.0 + dp * dp / 3.0)) < 1e-12


def test_wall_shear_approaches_poiseuille_value(ora):
    # tau_w = mu du/dy at the wall = 4 mu Umax / H for the parabolic profile;
    # the dummy-wall sum approaches it from below as dp shrinks
    ratios = []
    for dp in (1 / 20, 1 / 40, 1 / 80):
        c = poiseuille_channel(dp)
        mu = c.params["rho0"] * c.params["nu_l"]
        J, _ = ora.OracleSim(c).objective(slab(1.0, 4 * dp, 2.0))
        ratios.append(J[1] / (4.0 * mu))
    assert 0.93 < ratios[0] < ratios[1] < ratios[2] < 1.0
    assert abs(ratios[2] - 1.0) < 0.04


def test_wall_shear_sign_follows_the_flow(ora):
    c = poiseuille_channel(1 / 20)
    c.v[:, 0] *= -1.0
    J, _ = ora.OracleSim(c).objective(slab(1.0, 0.2, 2.0))
    assert J[1] < 0.0 and J[0] < 0.0


def test_frozen_membership_replaces_the_predicate(ora):
    c = poiseuille_channel(1 / 20)
    sim = ora.OracleSim(c)
    d = slab(1.0 + 1e-9, 0.2, 2.0)
    J, mem = sim.objective(d)
    J2, mem2 = sim.objective(d, member=mem)
    assert np.array_equal(mem, mem2) and np.array_equal(J, J2)
    J0, _ = sim.objective(d, member=np.zeros_like(mem))
    assert J0[0] == 0.0 and J0[1] == J[1]


def test_objective_rejects_turbulent_runs(ora):
    c = cases.make_jet(dp=0.25)
    with pytest.raises(RuntimeError):
        ora.OracleSim(c).objective(slab(1.0, 0.2, 2.0))


def adjoint_case(steps=1, length=1.0):
    return cases.make_adjoint_channel(dp=1 / 20, length=length, steps=steps)


def test_fd_gradient_of_inlet_slab_flux_is_the_profile_derivative(ora):
    # The inlet region is relabelled into the buffer by the first update, so
    # in step 2 a slab over the inlet buffer holds only prescribed-velocity
    # particles.  Their velocity after the step is u(s) = 4 Umax s (1 - s) +
    # sum a_m sin(m pi s) along +x with s = y / H (unchanged in the step and
    # by the recycling shift along x), and step 1 does not depend on a:
    # d mean(J_Q) / d a_m = (1/2) sum_i m sin(m pi s_i) / w over the frozen
    # slab members of step 2.
    c = adjoint_case(steps=2)
    dp = c.params["dp"]
    d = slab(1e-9, 4 * dp, 1.0)
    g, log = ora.fd_gradient(c, 2, d, 1, eps=1e-5, threads=4)
    _, _, sim = ora.rollout(c, 2, d, replay=log, threads=4)
    mem = log[1]["member"].astype(bool)
    pid_in = log[1]["pid"][mem]
    n = sim.n
    y_of = {int(p): y for p, y in zip(sim.pid[:n], sim.x[:n, 1])}
    tag_of = {int(p): int(t) for p, t in zip(sim.pid[:n], sim.tag[:n])}
    assert mem.sum() > 0
    assert all((tag_of[int(p)] & 3) == cases.BUFFER for p in pid_in)
    s = np.array([y_of[int(p)] for p in pid_in])
    m = c.params["rho0"] * dp * dp
    w = 4 * dp
    exact = np.array([0.5 * np.sum(m * np.sin((k + 1) * math.pi * s)) / w for k in range(16)])
    assert np.max(np.abs(g[:, 0] - exact)) < 1e-8 * np.max(np.abs(exact))


def test_fd_gradient_is_step_size_consistent(ora):
    # with every event frozen the rollout is smooth in a: differences at two
    # step sizes agree to far better than the 1e-4 parity bar
    c = adjoint_case(steps=12)
    cf = [0, 1, 4, 9]
    g1, log = ora.fd_gradient(c, 12, c.objective, 1, eps=1e-5, threads=4, coefs=cf)
    g2, _ = ora.fd_gradient(c, 12, c.objective, 1, eps=2e-6, log=log, threads=4, coefs=cf)
    for k in range(2):
        scale = np.max(np.abs(g1[cf, k]))
        assert scale > 0.0
        assert np.max(np.abs(g1[cf, k] - g2[cf, k])) < 1e-6 * scale


def test_fd_gradient_of_outlet_flux_is_positive_for_the_first_mode(ora):
    # raising the first sine mode adds inflow; after the acoustic signal has
    # crossed the unit-length channel the outlet flux rises with it, while
    # the even modes (zero net inflow) move it much less
    c = adjoint_case(steps=30)
    g, _ = ora.fd_gradient(c, 30, c.objective, 1, eps=1e-5, threads=4, coefs=[0, 1])
    assert g[0, 0] > 0.3
    assert abs(g[1, 0]) < 0.1 * g[0, 0]
