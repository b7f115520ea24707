"""End-to-end pins of the oracle's advection step plus buffer update.

Steady plane Poiseuille flow between dummy-particle walls with a parabolic
velocity inlet and a zero-pressure outlet (Sec. 4.1 set-up): the
time-averaged cross-section profile must match u = 4 Umax y (H - y) / H^2
within 2 % (L2), the centre-line pressure gradient must match
-8 mu Umax / H^2, and the numbers of injected and deleted particles must
balance once the flow is steady.
"""
import numpy as np
import pytest

import cases


@pytest.mark.slow
def test_poiseuille_steady_state_and_buffer_balance(ora):
    L, dp, nsteps, navg = 4.0, 0.05, 3000, 600
    c = cases.make_channel(L=L, dp=dp)
    s = ora.OracleSim(c, threads=8)
    s.buffer_update()
    nb = int(round(1.0 / dp))
    acc = np.zeros(nb)
    cnt = np.zeros(nb)
    pa = np.zeros(2)
    pc = np.zeros(2)
    inj = dele = 0
    for k in range(nsteps):
        s.step()
        cn = s.buffer_update()
        if k < nsteps - navg:
            continue
        inj += cn.n_inject[1] + cn.n_inject[2]
        dele += cn.n_delete[1] + cn.n_delete[2]
        n = s.n
        x, v, tag = s.x[:n], s.v[:n], s.tag[:n]
        fl = (tag & 3) != 2
        sel = fl & (x[:, 0] > 0.4 * L) & (x[:, 0] < 0.8 * L)
        b = np.clip((x[sel, 1] / dp).astype(int), 0, nb - 1)
        np.add.at(acc, b, v[sel, 0])
        np.add.at(cnt, b, 1)
        cen = fl & (np.abs(x[:, 1] - 0.5) < 0.15)
        for q, xc in enumerate((0.3 * L, 0.7 * L)):
            m = cen & (np.abs(x[:, 0] - xc) < 0.1)
            pa[q] += np.sum(100.0 * (s.rho[:n][m] - 1.0))
            pc[q] += m.sum()
    u = acc / cnt
    y = (np.arange(nb) + 0.5) * dp
    ua = 4.0 * y * (1.0 - y)
    l2 = np.sqrt(np.mean((u - ua) ** 2)) / np.sqrt(np.mean(ua ** 2))
    assert l2 < 0.02
    # pressure gradient: p = rho0 c0^2 (rho/rho0 - 1) with c0^2 = 100
    grad = (pa[0] / pc[0] - pa[1] / pc[1]) / (0.4 * L)
    mu = c.params["nu_l"] * c.params["rho0"]
    assert abs(grad - 8.0 * mu) < 0.1 * 8.0 * mu
    # steady state: particles in == particles out (within a handful)
    assert inj > 100
    assert abs(inj - dele) <= max(5, 0.02 * inj)
