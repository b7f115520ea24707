"""Pins of the oracle's transport-velocity shift.

The paper uses the transport-velocity formulation for particle regularity
(Sec. 2.3) and cites it without a formula; the oracle states the standard
position-correction form dx_i = -alpha h^2 sum_j 2 V_j grad_i W_ij for the
particles that move with the flow (fluid, and buffer particles of buffers
that extrapolate their velocity), evaluated on the start-of-step state and
added to the positions at the end of the advection step.  The expected values below come from
symmetry, antisymmetry of the kernel gradient, the divergence theorem in
the continuum limit, and the structure of the step, not from the oracle.
"""
import dataclasses

import numpy as np
import pytest
from scipy import integrate

import cases
from tests.helpers import block_case, interior_mask

ALPHA = 0.2


def _tvf(case, alpha=ALPHA):
    c = dataclasses.replace(case)
    c.params = dict(case.params, tvf_alpha=alpha)
    return c


def _shift(ora, case):
    return ora.OracleSim(_tvf(case), threads=4).rates()["shift"]


@pytest.mark.parametrize("dim,n_side", [(2, 16), (3, 8)])
def test_shift_vanishes_inside_a_uniform_lattice(ora, dim, n_side):
    # every neighbour at +r has a partner at -r: the gradient sum cancels
    c = block_case(dim=dim, n_side=n_side, dp=0.1)
    dx = _shift(ora, c)
    h = c.params["h"]
    inner = interior_mask(c.x, (0,) * dim, (n_side * 0.1,) * dim, 2 * h + 0.01)
    assert inner.sum() > 0
    assert np.abs(dx[inner]).max() < 1e-15
    # the edge rows do move (the sum is not zero by construction)
    assert np.abs(dx[~inner]).max() > 1e-4 * 0.1


def test_shift_pushes_a_pair_apart_along_its_axis(ora):
    # two particles: dx_i is along x_i - x_j, equal and opposite
    c = block_case(dim=2, n_side=1, dp=0.1)
    h = c.params["h"]
    x = np.array([[0.5, 0.5, 0.0], [0.5 + 0.8 * h, 0.5 + 0.3 * h, 0.0]])
    c = dataclasses.replace(c, x=x, v=np.zeros((2, 3)), rho=np.ones(2), drho=np.zeros(2),
                            k=np.zeros(2), eps=np.zeros(2), tag=np.zeros(2, np.uint32),
                            pid=np.arange(2, dtype=np.uint32))
    dx = _shift(ora, c)
    e = (x[0] - x[1]) / np.linalg.norm(x[0] - x[1])
    assert dx[0] @ e > 0 and dx[1] @ e < 0
    assert np.linalg.norm(np.cross(dx[0], e)) < 1e-14 * np.linalg.norm(dx[0])
    assert np.allclose(dx[0], -dx[1], rtol=0, atol=1e-16)


def test_volume_weighted_shift_sums_to_zero(ora):
    # sum_i V_i dx_i = -2 alpha h^2 sum_ij V_i V_j grad_i W_ij = 0 because
    # grad_i W_ij = -grad_j W_ji; unequal volumes make the weighting visible
    c = block_case(dim=2, n_side=12, dp=0.1, jitter=0.3, seed=4)
    rng = np.random.default_rng(2)
    c.rho = rng.uniform(0.8, 1.25, c.x.shape[0])
    dx = _shift(ora, c)
    V = c.params["rho0"] * 0.1 ** 2 / c.rho
    tot = (V[:, None] * dx).sum(axis=0)
    scale = (V[:, None] * np.abs(dx)).sum(axis=0).max()
    assert scale > 0
    assert np.abs(tot).max() < 1e-13 * scale


def test_shift_restores_a_displaced_particle(ora):
    # one particle moved by eps from its lattice site is pushed back, and the
    # response is linear in eps for small eps
    base = block_case(dim=2, n_side=16, dp=0.1)
    i = int(np.argmin(np.linalg.norm(base.x[:, :2] - 0.8, axis=1)))
    out = []
    for eps in (0.01, 0.02):
        x = base.x.copy()
        x[i, 0] += eps * 0.1
        x[i, 1] += 0.5 * eps * 0.1
        out.append(_shift(ora, dataclasses.replace(base, x=x))[i])
    d = np.array([1.0, 0.5, 0.0])
    assert out[0] @ d < 0 and out[1] @ d < 0
    assert abs(np.linalg.norm(out[1]) / np.linalg.norm(out[0]) - 2.0) < 0.01


def test_shift_at_a_lattice_edge_matches_the_divergence_theorem(ora):
    # A particle in the top row of a half-plane lattice, dp/2 below the
    # surface the lattice cells fill: sum_j V_j grad_i W_ij approximates
    # int_D grad_x W(x - y) dy = -n int_{surface} W dS (divergence theorem),
    # so dx_i = 2 alpha h^2 n Lambda, Lambda = int W(sqrt(s^2 + (dp/2)^2)) ds,
    # n the outward normal: the edge particle moves outward.
    dp, n_side = 0.1, 24
    c = block_case(dim=2, n_side=n_side, dp=dp)
    h = c.params["h"]
    dx = _shift(ora, c)
    top = np.abs(c.x[:, 1] - (n_side - 0.5) * dp) < 1e-9
    mid = top & (np.abs(c.x[:, 0] - 0.5 * n_side * dp) < 3 * dp)
    lam, _ = integrate.quad(lambda s: ora.kernel_W(np.hypot(s, 0.5 * dp), h, 2),
                            -2 * h, 2 * h, limit=200)
    expect = 2 * ALPHA * h * h * lam
    got = dx[mid]
    assert np.abs(got[:, 0]).max() < 1e-15
    assert np.abs(got[:, 1] / expect - 1.0).max() < 0.03


def test_step_adds_the_start_of_step_shift_to_flow_particles_only(ora):
    # With the shift on, the step differs from the plain step only in the
    # positions of fluid particles and of the outlet buffer's (extrapolated
    # velocity), by exactly the shift of the start state; the inlet buffer's
    # particles (prescribed velocity) and the walls do not move by it.
    c0 = cases.make_channel(H=0.5, L=1.5, dp=0.05, Re=50.0, Umax=1.0)
    s0 = ora.OracleSim(c0, threads=4)
    s0.buffer_update()
    sn = s0.snapshot()
    c = dataclasses.replace(c0, **{f: sn[f] for f in ("x", "v", "rho", "drho", "k", "eps",
                                                        "tag", "pid")},
                            npid=int(s0.S.next_pid))
    plain = ora.OracleSim(c, threads=4)
    tvf = ora.OracleSim(_tvf(c), threads=4)
    dx = tvf.rates()["shift"]
    I = plain.time_step()
    plain.step(I.dt_adv, I.n_ac)
    tvf.step(I.dt_adv, I.n_ac)
    a, b = plain.snapshot(), tvf.snapshot()
    kind, bid = c.tag & 3, (c.tag >> 8) & 0xFF
    outlet = [q.id for q in c.buffers if q.vel_mode == cases.VEL_EXTRAPOLATE]
    fluid = (kind == 0) | ((kind == 1) & np.isin(bid, outlet))
    assert (kind == 1).sum() > 0 and ((kind == 1) & ~fluid).sum() > 0
    assert ((kind == 1) & fluid).sum() > 0 and (kind == 2).sum() > 0
    for f in ("v", "rho", "drho", "tag", "pid"):
        assert np.array_equal(a[f], b[f]), f
    assert np.array_equal(a["x"][~fluid], b["x"][~fluid])
    assert np.abs(dx[~fluid]).max() == 0.0
    assert np.abs(dx[fluid]).max() > 0
    assert np.abs((b["x"] - a["x"]) - dx)[fluid].max() < 1e-15
    # outlet-buffer particles move only along the open face (normal removed)
    for q in c.buffers:
        if q.vel_mode != cases.VEL_EXTRAPOLATE:
            continue
        sel = (kind == 1) & (bid == q.id)
        n = np.array(q.frame[0])
        assert np.abs(dx[sel] @ n).max() < 1e-18
        assert np.abs(dx[sel]).max() > 0
        # none within 2h of the ends of the transverse extent
        y1 = (c.x - np.array(q.origin)) @ np.array(q.frame[1])
        ends = sel & (np.abs(y1) > q.half_width[0] - 2 * c.params["h"])
        assert ends.sum() > 0 and np.abs(dx[ends]).max() == 0.0
