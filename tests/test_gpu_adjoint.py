"""Parity of the sensitivity path (objectives, recorded replay, adjoint) of
the HIP library with the FP64 oracle, through the C ABI.

Bars:
  * objectives of a state: within 1e-12 of the oracle, slab membership
    bit-exact (by particle id);
  * a GPU rollout that replays the oracle's events (time steps, buffer
    decisions, slab membership): step-averaged objectives within 1e-10;
  * adjoint gradient d mean(J) / d a against the oracle's central finite
    differences with the same frozen events: max |g - g_fd| <= 1e-4 max |g_fd|
    for each objective; the same bar against central differences of the
    GPU's own FP64 rollout (at the full adjoint-channel size too);
  * checkpointed and unsegmented reverse sweeps agree bit for bit.
"""
import os

import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", n)), n))


THREADS = _threads()


@pytest.fixture(scope="module")
def sph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    from paper_2510_25702_amd import sph as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def sens():
    from paper_2510_25702_amd import sensitivity as s
    return s


@pytest.fixture(scope="module")
def ora():
    import oracle
    oracle.lib()
    return oracle


BID = 1   # the inlet buffer of the channel cases


def small_case(steps=20, length=1.0, dp=1 / 20, mode=4):
    c = cases.make_adjoint_channel(dp=dp, length=length, steps=steps)
    c.params["obc_mode"] = mode
    return c


def dev_u8(torch, a, n):
    t = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t[: len(a)] = torch.as_tensor(np.asarray(a, np.uint8), device="cuda")
    return t


def oracle_records(torch, sens, log, pid_cap):
    """The oracle's event log as GPU step records (indexed by particle id)."""
    recs = []
    for r in log:
        dec = np.zeros(pid_cap, np.uint32)
        mem = np.zeros(pid_cap, np.uint8)
        dec[r["pid"]] = r["dec"]
        mem[r["pid"]] = r["member"]
        recs.append(sens.StepRecord(0, 0.0, 0, r["dt_adv"], r["n_ac"],
                                    torch.as_tensor(dec.view(np.int32), device="cuda"),
                                    torch.as_tensor(mem, device="cuda")))
    return recs


def gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, recs, coef=None):
    import torch
    sim.restore(start)
    if coef is not None:
        sim.set_profile_coef(BID, coef)
    J, out, ckpts = sens.rollout(sim, steps, desc, pid_cap, replay=recs)
    return (J / steps).cpu().numpy(), out


def gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, gJ, K):
    """Adjoint gradient of gJ . mean(J) along the recorded events."""
    import torch
    sim.restore(start)
    J, out, ckpts = sens.rollout(sim, steps, desc, pid_cap, replay=recs, checkpoint_every=K)
    g = sens.adjoint(sim, desc, out, ckpts, pid_cap,
                     torch.as_tensor(np.asarray(gJ, np.float64)), steps, K)
    return g.cpu().numpy()


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


# ---------------------------------------------------------------------------
def test_objective_matches_oracle(sph, ora):
    import torch
    c = small_case(length=2.0)
    # a developed state with a non-trivial slab and wall field
    s_o = ora.OracleSim(c, threads=8)
    for _ in range(5):
        s_o.step()
        s_o.buffer_update()
    s_o.step()
    J_o, mem_o = s_o.objective(c.objective)
    snap = s_o.snapshot()
    import dataclasses
    c2 = dataclasses.replace(c, x=snap["x"], v=snap["v"], rho=snap["rho"], drho=snap["drho"],
                             tag=snap["tag"], pid=snap["pid"], npid=int(s_o.S.next_pid))
    sim = sph.Simulation(c2, precision=sph.SPH_FP64)
    sim.build_cells()
    pid_cap = int(s_o.S.next_pid) + 16
    J = torch.zeros(2, dtype=torch.float64, device="cuda")
    mem = torch.zeros(pid_cap, dtype=torch.uint8, device="cuda")
    sim.objective(sph.make_objective(c.objective, BID), J, member_out=mem, pid_cap=pid_cap)
    J = J.cpu().numpy()
    mem = mem.cpu().numpy()
    assert np.array_equal(mem[snap["pid"]], mem_o)
    assert int(mem.sum()) == int(mem_o.sum()) > 0
    assert abs(J[0] - J_o[0]) <= 1e-12 * abs(J_o[0])
    assert abs(J[1] - J_o[1]) <= 1e-12 * abs(J_o[1])


def test_replay_of_oracle_events_matches_oracle(sph, sens, ora):
    steps = 20
    c = small_case(steps)
    J_o, log, _ = ora.rollout(c, steps, c.objective, threads=8)
    import torch
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    recs = oracle_records(torch, sens, log, pid_cap)
    J, _ = gpu_rollout(sph, sens, sim, start, sph.make_objective(c.objective, BID), pid_cap,
                       steps, recs)
    assert np.abs(J - J_o).max() <= 1e-10 * np.abs(J_o).max()


@pytest.mark.parametrize("mode", [4, 3, 2, 1])
def test_adjoint_matches_oracle_finite_differences(sph, sens, ora, mode):
    import torch
    steps = 20
    c = small_case(steps, mode=mode)
    g_fd, log = ora.fd_gradient(c, steps, c.objective, BID, eps=1e-5, threads=8)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    recs = oracle_records(torch, sens, log, pid_cap)
    desc = sph.make_objective(c.objective, BID)
    for k in range(2):
        gJ = [1.0, 0.0] if k == 0 else [0.0, 1.0]
        g = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, gJ, K=7)
        err = rel_max(g, g_fd[:, k])
        print(f"mode {mode} objective {k}: max rel err {err:.3e}", flush=True)
        assert err <= 1e-4


def test_fp32_forward_adjoint_against_oracle_finite_differences(sph, sens, ora):
    # FP32 pair arithmetic in the forward, FP64 snapshots and reverse sweep:
    # the gradient of the FP64 scheme at the FP32 trajectory, held to the
    # same 1e-4 bar against the oracle's frozen-event differences (measured:
    # ~1e-7, against ~2e-10 with the FP64 forward)
    import torch
    steps = 20
    c = small_case(steps)
    g_fd, log = ora.fd_gradient(c, steps, c.objective, BID, eps=1e-5, threads=8)
    pid_cap = int(c.next_pid) + 4096
    recs = oracle_records(torch, sens, log, pid_cap)
    desc = sph.make_objective(c.objective, BID)
    errs = []
    for prec in (sph.SPH_FP64, sph.SPH_FP32_MIXED):
        sim = sph.Simulation(c, precision=prec)
        start = sim.save()
        for k in range(2):
            gJ = [1.0, 0.0] if k == 0 else [0.0, 1.0]
            g = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, gJ, K=7)
            errs.append(rel_max(g, g_fd[:, k]))
    print(f"fp64 {errs[0]:.2e} {errs[1]:.2e}  fp32-forward {errs[2]:.2e} {errs[3]:.2e}", flush=True)
    assert max(errs) <= 1e-4


def test_adjoint_matches_gpu_finite_differences_longer_channel(sph, sens):
    import torch
    steps = 12
    c = small_case(steps, length=2.0, dp=1 / 40)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    desc = sph.make_objective(c.objective, BID)
    J0, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    a0 = np.array([b for b in c.buffers if b.id == BID][0].coef)
    g = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, [1.0, 0.5], K=5)
    eps = 1e-5
    for m in (0, 1, 6):
        Jp = []
        for sgn in (1, -1):
            a = a0.copy()
            a[m] += sgn * eps
            J, _ = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, recs, coef=a)
            Jp.append(J[0] + 0.5 * J[1])
        fd = (Jp[0] - Jp[1]) / (2 * eps)
        assert abs(g[m] - fd) <= 1e-4 * np.abs(g).max(), (m, g[m], fd)


@pytest.mark.parametrize("field", ["x", "v", "rho", "drho"])
@pytest.mark.parametrize("steps", [1, 3])
def test_state_cotangent_dot_product(sph, sens, field, steps):
    # <lambda_start, delta> against central differences of the rollout along a
    # random perturbation delta of one field of the real particles' start state
    import torch
    c = small_case(steps)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    desc = sph.make_objective(c.objective, BID)
    _, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    sim.restore(start)
    J, out, ckpts = sens.rollout(sim, steps, desc, pid_cap, replay=recs, checkpoint_every=2)
    gJ = torch.tensor([1.0, 3.0], dtype=torch.float64)
    _, lam = sens.adjoint(sim, desc, out, ckpts, pid_cap, gJ, steps, 2,
                          return_state_cotangent=True)
    lam = lam.cpu().numpy()
    n = start["n"]
    tag = start["tag"].cpu().numpy()[:n].view(np.uint32)
    pid = start["pid"].cpu().numpy()[:n].view(np.uint32)
    real = (tag & 3) <= 1
    rng = np.random.default_rng(7)
    rows = {"x": [0, 1], "v": [3, 4], "rho": [6], "drho": [7]}[field]
    scale = {"x": c.params["dp"] * 1e-2, "v": 0.1, "rho": 1e-3, "drho": 0.1}[field]
    delta = np.zeros((len(rows), n))
    delta[:, real] = rng.uniform(-1, 1, (len(rows), int(real.sum()))) * scale
    pred = sum(float(np.dot(lam[r][pid], delta[q])) for q, r in enumerate(rows))

    def run(sgn, eps):
        snap = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in start.items()}
        key = {"x": "x", "v": "v", "rho": "rho", "drho": "drho"}[field]
        d = torch.as_tensor(delta, device="cuda")
        if key in ("x", "v"):
            snap[key][: len(rows), :n] += sgn * eps * d
        else:
            snap[key][:n] += sgn * eps * d[0]
        sim.restore(snap)
        Jr, _, _ = sens.rollout(sim, steps, desc, pid_cap, replay=recs)
        Jr = (Jr / steps).cpu().numpy()
        return Jr[0] + 3.0 * Jr[1]
    eps = 1e-4
    fd = (run(1, eps) - run(-1, eps)) / (2 * eps)
    print(f"{field} steps={steps}: adjoint {pred:.12e} fd {fd:.12e}", flush=True)
    assert abs(pred - fd) <= 1e-5 * max(abs(fd), 1e-12) + 1e-12


def test_checkpointing_does_not_change_the_gradient(sph, sens):
    steps = 9
    c = small_case(steps)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    desc = sph.make_objective(c.objective, BID)
    _, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    g1 = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, [1.0, 1.0], K=steps)
    g2 = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, [1.0, 1.0], K=2)
    assert np.array_equal(g1, g2)


def test_autograd_function(sph, sens):
    import torch
    steps = 8
    c = small_case(steps)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    start = sim.save()
    a = torch.tensor(np.array([b for b in c.buffers if b.id == BID][0].coef),
                     dtype=torch.float64, requires_grad=True)
    J = sens.inlet_sensitivity(a, sim, c.objective, BID, steps, checkpoint_every=3)
    (J[0] + 2.0 * J[1]).backward()
    g = a.grad.numpy().copy()
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    # against the recorded-event adjoint called directly
    sim.restore(start)
    desc = sph.make_objective(c.objective, BID)
    pid_cap = sens.default_pid_cap(sim, steps)
    _, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    g2 = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, [1.0, 2.0], K=3)
    assert np.allclose(g, g2, rtol=1e-12, atol=1e-14 * np.abs(g2).max())


def test_adjoint_argument_errors(sph, sens):
    import torch
    c = small_case(4)
    simt = sph.Simulation(cases.make_jet(dp=0.25), precision=sph.SPH_FP64)   # k-epsilon
    assert sph.sph_adjoint_workspace_size(simt.ctx, 4) == 0
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    nb = sph.sph_adjoint_workspace_size(sim.ctx, 4)
    assert nb > 0
    pre = sim.save()
    desc = sph.make_objective(c.objective, BID)
    pid_cap = int(c.next_pid) + 64
    dec = torch.zeros(pid_cap, dtype=torch.int32, device="cuda")
    mem = torch.zeros(pid_cap, dtype=torch.uint8, device="cuda")
    lam = torch.zeros(8, pid_cap, dtype=torch.float64, device="cuda")
    grad = torch.zeros(16, dtype=torch.float64, device="cuda")
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) & ~255
    step, t, npid = sim.clock()
    good = dict(dt_adv=1e-3, n_ac=4, pid_cap=pid_cap)

    def ctl(**kw):
        d = dict(good, **kw)
        return sph.sph_adjoint_ctrl(step, t, npid, d["dt_adv"], d["n_ac"], 0, dec.data_ptr(),
                                    mem.data_ptr(), d["pid_cap"], 1.0, 0.0)
    with pytest.raises(sph.SphError) as e:   # sub-steps beyond the workspace
        sph.sph_adjoint_step(sim.ctx, sim.parts_of(pre), pre["n"], desc, ctl(n_ac=9),
                             lam.data_ptr(), grad.data_ptr(), wp, nb)
    assert e.value.status == sph.SPH_E_ARG
    with pytest.raises(sph.SphError) as e:   # particle ids beyond pid_cap
        sph.sph_adjoint_step(sim.ctx, sim.parts_of(pre), pre["n"], desc, ctl(pid_cap=4),
                             lam.data_ptr(), grad.data_ptr(), wp, nb)
    assert e.value.status == sph.SPH_E_ARG
    with pytest.raises(sph.SphError) as e:   # turbulent context
        sph.sph_adjoint_step(simt.ctx, sim.parts_of(pre), pre["n"], desc, ctl(),
                             lam.data_ptr(), grad.data_ptr(), wp, nb)
    assert e.value.status == sph.SPH_E_ARG
    # a valid call runs
    sph.sph_adjoint_step(sim.ctx, sim.parts_of(pre), pre["n"], desc, ctl(),
                         lam.data_ptr(), grad.data_ptr(), wp, nb)


def test_forward_reverse_split_equals_the_replaying_step(sph, sens):
    # sph_adjoint_forward on every step of a segment, then sph_adjoint_reverse
    # on the kept workspaces, against sph_adjoint_step replaying each step from
    # its saved start state: the same gradient and state cotangent, bit for bit
    import torch
    steps, K = 6, 3
    c = small_case(steps)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    desc = sph.make_objective(c.objective, BID)
    _, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    sim.restore(start)
    J, out, ckpts = sens.rollout(sim, steps, desc, pid_cap, replay=recs, checkpoint_every=K)
    gJ = torch.tensor([1.0, 0.5], dtype=torch.float64)
    g1, lam1 = sens.adjoint(sim, desc, out, ckpts, pid_cap, gJ, steps, K,
                            return_state_cotangent=True)
    # the replaying form, step by step from saved start states
    sim.restore(start)
    pres = []
    for r in out:
        pres.append(sim.save())
        sim.build_cells()
        sim.correction()
        sim.step(r.dt_adv, r.n_ac)
        sim.buffer_update_ex(forced=r.dec, pid_cap=pid_cap)
    nb = sph.sph_adjoint_workspace_size(sim.ctx, max(r.n_ac for r in out))
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) & ~255
    lam2 = torch.zeros(8, pid_cap, dtype=torch.float64, device="cuda")
    g2 = torch.zeros(16, dtype=torch.float64, device="cuda")
    for n in reversed(range(steps)):
        r, pre = out[n], pres[n]
        ctl = sph.sph_adjoint_ctrl(r.step, r.t, r.next_pid, r.dt_adv, r.n_ac, 0, r.dec.data_ptr(),
                                   r.member.data_ptr(), pid_cap, 1.0 / steps, 0.5 / steps)
        sph.sph_adjoint_step(sim.ctx, sim.parts_of(pre), pre["n"], desc, ctl, lam2.data_ptr(),
                             g2.data_ptr(), wp, nb)
    assert np.abs(g1.cpu().numpy()).max() > 0
    assert np.array_equal(g1.cpu().numpy(), g2[:16].cpu().numpy())
    assert torch.equal(lam1, lam2)


def test_forward_reverse_argument_errors(sph, sens):
    import torch
    c = small_case(4)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    nb = sph.sph_adjoint_workspace_size(sim.ctx, 4)
    desc = sph.make_objective(c.objective, BID)
    pid_cap = int(c.next_pid) + 64
    dec = torch.zeros(pid_cap, dtype=torch.int32, device="cuda")
    mem = torch.zeros(pid_cap, dtype=torch.uint8, device="cuda")
    lam = torch.zeros(8, pid_cap, dtype=torch.float64, device="cuda")
    grad = torch.zeros(16, dtype=torch.float64, device="cuda")
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) & ~255
    step, t, npid = sim.clock()

    def ctl(next_pid=npid):
        return sph.sph_adjoint_ctrl(step, t, next_pid, 1e-3, 4, 0, dec.data_ptr(), mem.data_ptr(),
                                    pid_cap, 1.0, 0.0)
    with pytest.raises(sph.SphError) as e:   # not the recorded step's start state
        sph.sph_adjoint_forward(sim.ctx, ctl(next_pid=npid + 1), wp, nb)
    assert e.value.status == sph.SPH_E_STATE
    with pytest.raises(sph.SphError) as e:   # workspace too small
        sph.sph_adjoint_forward(sim.ctx, ctl(), wp, nb - 256)
    assert e.value.status == sph.SPH_E_ARG
    n_step = sph.sph_adjoint_forward(sim.ctx, ctl(), wp, nb)
    assert n_step == c.n
    with pytest.raises(sph.SphError) as e:   # slot count beyond the capacity
        sph.sph_adjoint_reverse(sim.ctx, desc, ctl(), 1 << 40, lam.data_ptr(), grad.data_ptr(),
                                wp, nb)
    assert e.value.status == sph.SPH_E_ARG
    sph.sph_adjoint_reverse(sim.ctx, desc, ctl(), n_step, lam.data_ptr(), grad.data_ptr(), wp, nb)


def test_adjoint_full_size_against_gpu_finite_differences(sph, sens):
    # the adjoint channel at its full size (20H x H, dp = H/80, ~130k
    # particles), a shortened rollout; two sampled coefficients
    steps = 10
    c = cases.make_adjoint_channel(steps=steps)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 8192
    start = sim.save()
    desc = sph.make_objective(c.objective, BID)
    _, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    g = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, [0.0, 1.0], K=5)
    a0 = np.array([b for b in c.buffers if b.id == BID][0].coef)
    eps = 1e-5
    for m in (0, 3):
        Jp = []
        for sgn in (1, -1):
            a = a0.copy()
            a[m] += sgn * eps
            J, _ = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, recs, coef=a)
            Jp.append(J[1])
        fd = (Jp[0] - Jp[1]) / (2 * eps)
        assert abs(g[m] - fd) <= 1e-4 * np.abs(g).max(), (m, g[m], fd)


def test_adjoint_3d_matches_oracle_finite_differences(sph, sens, ora):
    # the 3D duct (sine inlet on the transverse coordinate y, four walls)
    import torch
    steps = 8
    c = cases.make_duct3d(steps=steps)
    cf = [0, 1, 4]
    g_fd, log = ora.fd_gradient(c, steps, c.objective, BID, eps=1e-5, threads=8, coefs=cf)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    recs = oracle_records(torch, sens, log, pid_cap)
    desc = sph.make_objective(c.objective, BID)
    J, _ = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, recs)
    J_o, _, _ = ora.rollout(c, steps, c.objective, replay=log, threads=8)
    assert np.abs(J - J_o).max() <= 1e-10 * np.abs(J_o).max()
    for k in range(2):
        gJ = [1.0, 0.0] if k == 0 else [0.0, 1.0]
        g = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, gJ, K=3)
        err = rel_max(g[cf], g_fd[cf, k])
        print(f"3D objective {k}: max rel err {err:.3e}", flush=True)
        assert err <= 1e-4


@pytest.mark.parametrize("field", ["x", "v", "rho"])
def test_state_cotangent_dot_product_3d(sph, sens, field):
    import torch
    steps = 2
    c = cases.make_duct3d(steps=steps)
    sim = sph.Simulation(c, precision=sph.SPH_FP64)
    pid_cap = int(c.next_pid) + 4096
    start = sim.save()
    desc = sph.make_objective(c.objective, BID)
    _, recs = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, None)
    sim.restore(start)
    J, out, ckpts = sens.rollout(sim, steps, desc, pid_cap, replay=recs, checkpoint_every=1)
    _, lam = sens.adjoint(sim, desc, out, ckpts, pid_cap, torch.tensor([1.0, 2.0],
                          dtype=torch.float64), steps, 1, return_state_cotangent=True)
    lam = lam.cpu().numpy()
    n = start["n"]
    tag = start["tag"].cpu().numpy()[:n].view(np.uint32)
    pid = start["pid"].cpu().numpy()[:n].view(np.uint32)
    real = (tag & 3) <= 1
    rng = np.random.default_rng(11)
    rows = {"x": [0, 1, 2], "v": [3, 4, 5], "rho": [6]}[field]
    scale = {"x": c.params["dp"] * 1e-2, "v": 0.1, "rho": 1e-3}[field]
    delta = np.zeros((len(rows), n))
    delta[:, real] = rng.uniform(-1, 1, (len(rows), int(real.sum()))) * scale
    pred = sum(float(np.dot(lam[r][pid], delta[q])) for q, r in enumerate(rows))

    def run(sgn, eps):
        snap = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in start.items()}
        d = torch.as_tensor(delta, device="cuda")
        if field in ("x", "v"):
            snap[field][:, :n] += sgn * eps * d
        else:
            snap[field][:n] += sgn * eps * d[0]
        sim.restore(snap)
        Jr, _, _ = sens.rollout(sim, steps, desc, pid_cap, replay=recs)
        Jr = (Jr / steps).cpu().numpy()
        return Jr[0] + 2.0 * Jr[1]
    eps = 1e-4
    fd = (run(1, eps) - run(-1, eps)) / (2 * eps)
    print(f"3D {field}: adjoint {pred:.12e} fd {fd:.12e}", flush=True)
    assert abs(pred - fd) <= 1e-5 * max(abs(fd), 1e-12) + 1e-12


@pytest.mark.parametrize("pname,prec", [("fp64", 0), ("fp32", 1)])
def test_adjoint_configured_run_against_oracle_finite_differences(sph, sens, ora, pname, prec):
    # the configured sensitivity run: the adjoint channel at full size (20H x H,
    # dp = H/80, ~138k particles), 100 steps, checkpoints every 10; the GPU
    # replays the oracle's own events and its adjoint gradient is compared with
    # the oracle's central differences of the same frozen-event map, stored by
    # tests/golden/make_adjoint_fd.py (three coefficients, both objectives).
    # The FP32-mixed forward gives the FP64 scheme's gradient at its FP32
    # trajectory, within the same 1e-4.
    import json
    import torch
    path = os.path.join(os.path.dirname(__file__), "golden", "adjoint_channel_fd.json")
    ref = json.load(open(path))
    steps = ref["steps"]
    c = cases.make_adjoint_channel(steps=steps)
    assert c.n == ref["particles"]
    J_o, log, _ = ora.rollout(c, steps, c.objective, threads=THREADS)
    assert np.abs(J_o - np.array(ref["J_mean"])).max() <= 1e-12 * np.abs(J_o).max()
    sim = sph.Simulation(c, precision=prec)
    pid_cap = int(c.next_pid) + 8192
    start = sim.save()
    recs = oracle_records(torch, sens, log, pid_cap)
    desc = sph.make_objective(c.objective, BID)
    J, _ = gpu_rollout(sph, sens, sim, start, desc, pid_cap, steps, recs)
    assert np.abs(J - J_o).max() <= (1e-10 if prec == 0 else 1e-5) * np.abs(J_o).max()
    cf = [int(m) for m in ref["coefs"]]
    g = {}
    for k in range(2):
        gJ = [1.0, 0.0] if k == 0 else [0.0, 1.0]
        g[k] = gpu_gradient(sph, sens, sim, start, desc, pid_cap, steps, recs, gJ, K=10)[cf]
    fd_tau = np.array([ref["grad"][str(m)][1] for m in cf])
    err = rel_max(g[1], fd_tau)
    print(f"configured adjoint run {pname}: wall shear gradient {g[1]}, oracle {fd_tau}, "
          f"max rel err {err:.3e}; outlet flux gradient {g[0]}", flush=True)
    assert err <= 1e-4
    # in 100 steps (t = 0.4) no disturbance of the inlet reaches the outlet
    # slab 20H downstream: the oracle's central differences of the slab flux
    # are exactly zero, and the adjoint's are negligible beside the shear's
    fd_q = np.array([ref["grad"][str(m)][0] for m in cf])
    assert np.all(fd_q == 0.0)
    assert np.abs(g[0]).max() <= 1e-9 * np.abs(fd_tau).max()
