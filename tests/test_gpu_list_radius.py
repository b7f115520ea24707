"""The relative-motion radius of the neighbour list built by sph_advance.

sph_advance builds each step's list from the coming step's time step: j is
listed for i when |r_ij| < 2h + s_i + s_j + |u_c(i) - u_c(j)| dt_adv, with
u_c the mean velocity of a particle's build cell and s_i its allowed
deviation from drifting with it; the pressure pass checks every particle's
displacement against that allowance after each sub-step and falls back to
the cell stencil for the rest of the step when one exceeds it.  The pairs
within 2h are then the same as with the cell-size radius at every sub-step,
so both runs give the same state up to the order of the pair sums (FP64).
"""
import os

import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25702_amd import sph
    return sph


def _sim(sph, case, tight):
    old = os.environ.get("SPHX_LIST_TIGHT")
    os.environ["SPHX_LIST_TIGHT"] = "1" if tight else "0"
    try:
        g = sph.Simulation(case, precision=sph.SPH_FP64)
    finally:
        if old is None:
            del os.environ["SPHX_LIST_TIGHT"]
        else:
            os.environ["SPHX_LIST_TIGHT"] = old
    g.build_cells()
    g.buffer_update()
    return g


def _by_pid(st):
    o = np.argsort(st["pid"])
    return {k: v[o] for k, v in st.items()}


def _run(sph, case, steps, tight, ctrl=None):
    g = _sim(sph, case, tight)
    info = None
    for _ in range(steps):
        info, _ = g.advance(*(ctrl or (0.0, 0)))
    return _by_pid(g.state()), info


def _compare(a, b, name, h):
    assert np.array_equal(a["pid"], b["pid"]) and np.array_equal(a["tag"], b["tag"])
    dx = np.abs(a["x"] - b["x"]).max() / h
    vmax = max(np.abs(b["v"]).max(), 1e-12)
    dv = np.abs(a["v"] - b["v"]).max() / vmax
    drho = np.abs(a["rho"] - b["rho"]).max()
    print(f"{name}: x {dx:.2e} h, v {dv:.2e} vmax, rho {drho:.2e}", flush=True)
    assert dx <= 1e-9 and dv <= 1e-8 and drho <= 1e-10


CASES = {
    "uchannel": (lambda: cases.make_uchannel(ramp_time=0.0), 20),
    "jet": (lambda: cases.make_jet(), 20),
    "mixer_dp0125": (lambda: cases.make_mixer(dp=0.0125), 40),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_relative_motion_radius_gives_the_cell_radius_state(sph, name):
    make, steps = CASES[name]
    c = make()
    a, _ = _run(sph, c, steps, True)
    b, _ = _run(sph, c, steps, False)
    _compare(a, b, name, c.params["h"])


def test_a_longer_step_than_the_list_was_built_for_falls_back(sph):
    # a caller-set advection step 1.1 times the one the list was built for
    # (a particle then moves up to 0.275h, inside the cell skin of 0.3h):
    # the elapsed-time check outgrows the list, the passes scan the stencil
    c = cases.make_jet()
    g = _sim(sph, c, True)
    info, _ = g.advance()
    ctrl = (1.1 * info.dt_adv, 2 * info.n_ac)
    a, _ = _run(sph, c, 6, True, ctrl)
    b, _ = _run(sph, c, 6, False, ctrl)
    _compare(a, b, "jet, longer step", c.params["h"])
