"""Inlet-profile sensitivity: recorded rollouts and the adjoint through
``torch.autograd.Function`` (argument marshalling and call sequencing only;
every step, objective and adjoint step runs in libsphx.so).

Forward: ``steps`` advection steps (cell build, correction, step, objective,
buffer update) with the time steps, buffer decisions and slab membership of
every step recorded by particle id, and a device checkpoint of the full state
every ``checkpoint_every`` steps.  Backward: segment by segment in reverse,
restore the checkpoint, recompute the segment with ``sph_adjoint_forward``
(replaying the record, one workspace per step holding its sub-step states),
then call ``sph_adjoint_reverse`` on the workspaces in reverse, carrying the
state cotangent (by particle id) and accumulating the gradient with respect
to the control buffer's sine coefficients.
"""
from __future__ import annotations

from dataclasses import dataclass

from .sph import (make_objective, sph_adjoint_ctrl, sph_adjoint_forward,
                  sph_adjoint_reverse, sph_adjoint_workspace_size)


@dataclass
class StepRecord:
    step: int
    t: float
    next_pid: int
    dt_adv: float
    n_ac: int
    dec: object      # device int32 [pid_cap]: decisions by particle id
    member: object   # device uint8 [pid_cap]: slab membership by particle id


def default_pid_cap(sim, steps, headroom=None):
    _, _, next_pid = sim.clock()
    if headroom is None:
        headroom = max(4096, 512 * steps)
    return int(next_pid + headroom)


def rollout(sim, steps, desc, pid_cap, replay=None, checkpoint_every=0, J=None):
    """Runs `steps` steps from the current state; returns (J_sum, records,
    checkpoints).  `replay` (records of an earlier run) freezes the time
    steps, buffer decisions and slab membership."""
    torch = sim.torch
    dev = sim.device
    if J is None:
        J = torch.zeros(2, dtype=torch.float64, device=dev)
    records, ckpts = [], {}
    for n in range(steps):
        if checkpoint_every and n % checkpoint_every == 0:
            ckpts[n] = sim.save()
        step, t, next_pid = sim.clock()
        sim.build_cells()
        sim.correction()
        if replay is None:
            info = sim.step()
            dt_adv, n_ac = info.dt_adv, info.n_ac
            member = torch.zeros(pid_cap, dtype=torch.uint8, device=dev)
            dec = torch.zeros(pid_cap, dtype=torch.int32, device=dev)
            sim.objective(desc, J, member_out=member, pid_cap=pid_cap)
            sim.buffer_update_ex(log=dec, pid_cap=pid_cap)
        else:
            r = replay[n]
            sim.step(r.dt_adv, r.n_ac)
            dt_adv, n_ac, member, dec = r.dt_adv, r.n_ac, r.member, r.dec
            sim.objective(desc, J, member_in=member, pid_cap=pid_cap)
            sim.buffer_update_ex(forced=dec, pid_cap=pid_cap)
        records.append(StepRecord(step, t, next_pid, float(dt_adv), int(n_ac), dec, member))
    return J, records, ckpts


def adjoint(sim, desc, records, ckpts, pid_cap, gJ, steps, checkpoint_every, n_coef=16,
            return_state_cotangent=False, timings=None):
    """Reverse sweep: returns d(gJ . mean J)/da (device FP64 [n_coef]) and, on
    request, the cotangent of the start state (device FP64 [8][pid_cap], rows
    x0 x1 x2 v0 v1 v2 rho drho, by particle id).  `timings` (a dict) receives
    the wall time of the segment recomputations and of the adjoint steps."""
    import time
    torch = sim.torch
    dev = sim.device
    lam = torch.zeros(8, pid_cap, dtype=torch.float64, device=dev)
    grad = torch.zeros(16, dtype=torch.float64, device=dev)
    max_nac = max(r.n_ac for r in records)
    nbytes = sph_adjoint_workspace_size(sim.ctx, max_nac)
    if nbytes == 0:
        raise RuntimeError("the adjoint needs a laminar context")
    K = checkpoint_every if checkpoint_every > 0 else steps
    stride = (nbytes + 255) & ~255
    ws = torch.empty(stride * min(K, steps) + 256, dtype=torch.uint8, device=dev)
    ws_base = (ws.data_ptr() + 255) & ~255
    g = gJ.detach().to("cpu", torch.float64).numpy()
    wq, wt = float(g[0]) / steps, float(g[1]) / steps
    starts = list(range(0, steps, K))
    t_re = t_adj = 0.0
    for s0 in reversed(starts):
        s1 = min(s0 + K, steps)
        t0 = time.perf_counter()
        sim.restore(ckpts[s0])
        ctls, nsteps = {}, {}
        for n in range(s0, s1):
            r = records[n]
            ctls[n] = sph_adjoint_ctrl(r.step, r.t, r.next_pid, r.dt_adv, r.n_ac, 0,
                                       r.dec.data_ptr(), r.member.data_ptr(), pid_cap, wq, wt)
            nsteps[n] = sph_adjoint_forward(sim.ctx, ctls[n], ws_base + (n - s0) * stride, nbytes)
        sim.stream.synchronize()
        t1 = time.perf_counter()
        t_re += t1 - t0
        for n in reversed(range(s0, s1)):
            sph_adjoint_reverse(sim.ctx, desc, ctls[n], nsteps[n], lam.data_ptr(),
                                grad.data_ptr(), ws_base + (n - s0) * stride, nbytes)
        t_adj += time.perf_counter() - t1
    if timings is not None:
        timings["recompute_s"] = t_re
        timings["adjoint_s"] = t_adj
    if return_state_cotangent:
        return grad[:n_coef], lam
    return grad[:n_coef]


class InletSensitivity:
    """d mean_steps [J_Q, J_tau] / d a through ``torch.autograd``.

    apply(coef, sim, objective_dict, buffer_id, steps, checkpoint_every)
    runs the forward rollout from the simulation's current state with the
    control buffer's coefficients set to `coef` and returns the step-averaged
    [J_Q, J_tau]; backward runs the adjoint.  The simulation must be a
    laminar context; it is left at the end of the rollout after forward and
    at an earlier state after backward.
    """

    @staticmethod
    def function():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, coef, sim, objective, buffer_id, steps, checkpoint_every=10):
                if sim.turbulence:
                    raise RuntimeError("the adjoint needs a laminar context")
                sim.set_profile_coef(buffer_id, coef.detach().cpu().numpy())
                desc = make_objective(objective, buffer_id)
                pid_cap = default_pid_cap(sim, steps)
                J, recs, ckpts = rollout(sim, steps, desc, pid_cap,
                                         checkpoint_every=checkpoint_every)
                ctx.sim, ctx.desc, ctx.recs, ctx.ckpts = sim, desc, recs, ckpts
                ctx.pid_cap, ctx.steps, ctx.K = pid_cap, steps, checkpoint_every
                ctx.n_coef = int(coef.numel())
                ctx.coef_meta = (coef.dtype, coef.device)
                return J / steps

            @staticmethod
            def backward(ctx, gJ):
                g = adjoint(ctx.sim, ctx.desc, ctx.recs, ctx.ckpts, ctx.pid_cap, gJ, ctx.steps,
                            ctx.K, ctx.n_coef)
                dtype, device = ctx.coef_meta
                return g.to(device=device, dtype=dtype), None, None, None, None, None

        return _F


def inlet_sensitivity(coef, sim, objective, buffer_id, steps, checkpoint_every=10):
    """Step-averaged [J_Q, J_tau] as a differentiable function of `coef`."""
    return InletSensitivity.function().apply(coef, sim, objective, buffer_id, steps,
                                             checkpoint_every)
