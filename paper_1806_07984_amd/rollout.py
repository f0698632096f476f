"""Differentiable rollout of the ADER-DG step (torch.autograd.Function).

The forward pass advances the state n steps with a FROZEN time-step
schedule (the dt of every step of the unperturbed run, from adg_step's
history); the backward pass runs the library's hand-written adjoint
(adg_step_adjoint) step by step in reverse.  Only every k-th state is kept
(checkpointing); each segment is recomputed forward before its adjoint steps,
by default as recorded steps (adg_step_record) whose tapes the adjoint steps
read (adg_step_adjoint_tape), so no predictor runs twice.  The last segment is
recorded by the forward pass itself, since its tapes are the first the
backward pass needs.
The point-sample misfit of the density, J = 1/2 sum_s (rho_h(x_s) - rho*_s)^2,
is a second Function whose backward scatters through adg_sample_adjoint.
"""
import torch


def dt_schedule(mesh, u0, n_steps):
    """dt of every step of the unperturbed forward run (step-major, one value
    per instance and step)."""
    u = u0.detach().clone()
    ws = mesh.empty_workspace()
    hist = torch.zeros(n_steps * mesh.n_instances, dtype=torch.float64, device=u.device)
    mesh.step(u, n_steps, ws, hist)
    mesh.status()
    return hist


class _Buffers:
    def __init__(self, mesh):
        self.ustar = mesh.empty_u()
        self.traces = mesh.empty_traces()
        self.fside = mesh.empty_fside()


def advance_fixed(mesh, u, dt_sched, n0, n1, bufs):
    """Advance u in place from step n0 to step n1 with the frozen schedule."""
    ni = mesh.n_instances
    for n in range(n0, n1):
        dt = dt_sched[n * ni:(n + 1) * ni]
        mesh.predictor(u, dt, bufs.ustar, bufs.traces)
        mesh.riemann(bufs.traces, bufs.fside)
        mesh.corrector(bufs.ustar, bufs.fside, dt, u)


class Rollout(torch.autograd.Function):
    """u_n = step^n(u_0) at the frozen schedule; checkpoint every k steps."""

    @staticmethod
    def forward(ctx, u0, mesh, dt_sched, n_steps, k, record=True):
        u = u0.detach().clone()
        ckpts = []
        ws = mesh.empty_adjoint_workspace()
        ni = mesh.n_instances
        # with recording, the last segment keeps its tapes and states for the
        # backward pass, which starts there
        tapes = [mesh.empty_tape() for _ in range(min(k, n_steps))] if record and n_steps > 0 else None
        last = ((n_steps - 1) // k) * k if n_steps > 0 else 0
        states = []
        for s0 in range(0, n_steps, k):
            ckpts.append(u.clone())
            for n in range(s0, min(s0 + k, n_steps)):
                dt = dt_sched[n * ni:(n + 1) * ni]
                if tapes is not None and s0 == last:
                    states.append(u.clone())
                    mesh.step_record(states[-1], dt, u, tapes[n - s0], ws)
                else:
                    # one step at the frozen dt (adg_step_record without a tape)
                    mesh.step_record(u, dt, u, None, ws)
        ctx.mesh, ctx.k, ctx.n_steps, ctx.record = mesh, k, n_steps, record
        ctx.tapes, ctx.last_states = tapes, states
        ctx.save_for_backward(dt_sched, *ckpts)
        return u

    @staticmethod
    def backward(ctx, ubar_out):
        dt_sched, *ckpts = ctx.saved_tensors
        mesh, k, n_steps = ctx.mesh, ctx.k, ctx.n_steps
        ni = mesh.n_instances
        bufs = _Buffers(mesh)
        ws = mesh.empty_adjoint_workspace()
        ubar = ubar_out.detach().contiguous().clone()
        nxt = torch.empty_like(ubar)
        # recorded segments: each forward predictor of the segment runs once
        # and keeps what its adjoint step reads (k tapes); otherwise the
        # adjoint step runs the predictor again from the recomputed state
        tapes = ctx.tapes
        for si in reversed(range(len(ckpts))):
            s0, s1 = si * k, min(si * k + k, n_steps)
            states = [ckpts[si]]
            if tapes is not None:
                if si == len(ckpts) - 1:
                    # recorded by the forward pass
                    states, ctx.last_states = ctx.last_states, None
                else:
                    for n in range(s0, s1):
                        nxt_state = torch.empty_like(states[-1]) if n < s1 - 1 else None
                        mesh.step_record(states[-1], dt_sched[n * ni:(n + 1) * ni], nxt_state, tapes[n - s0], ws)
                        if nxt_state is not None:
                            states.append(nxt_state)
                for n in reversed(range(s0, s1)):
                    mesh.step_adjoint_tape(states[n - s0], dt_sched[n * ni:(n + 1) * ni], tapes[n - s0], ubar, nxt,
                                           ws)
                    ubar, nxt = nxt, ubar
                continue
            for n in range(s0, s1 - 1):
                u = states[-1].clone()
                advance_fixed(mesh, u, dt_sched, n, n + 1, bufs)
                states.append(u)
            for n in reversed(range(s0, s1)):
                mesh.step_adjoint(states[n - s0], dt_sched[n * ni:(n + 1) * ni], ubar, nxt, ws)
                ubar, nxt = nxt, ubar
        ctx.tapes = None
        return ubar, None, None, None, None, None


class SampledMisfit(torch.autograd.Function):
    """J = 1/2 sum_s (rho_h(x_s) - target_s)^2 on a single-instance uniform mesh."""

    @staticmethod
    def forward(ctx, u, mesh, pts, target):
        vals = torch.empty(pts.shape[0], dtype=torch.float64, device=u.device)
        mesh.sample(u.detach().contiguous(), pts, vals)
        r = vals - target
        ctx.mesh = mesh
        ctx.save_for_backward(pts, r)
        return 0.5 * (r * r).sum()

    @staticmethod
    def backward(ctx, jbar):
        pts, r = ctx.saved_tensors
        mesh = ctx.mesh
        ubar = torch.zeros(mesh.info["u_elems"], dtype=torch.float64, device=r.device)
        wbar = (r * jbar).contiguous()
        mesh.sample_adjoint(pts, wbar, ubar)
        return ubar, None, None, None


def loss_and_grad(mesh, u0, pts, target, n_steps, k=5, dt_sched=None, record=True):
    """J(u0) after n_steps (frozen schedule) and dJ/du0 through the adjoint;
    record: recompute each segment with recorded steps (k tapes of
    adjoint_tape_bytes) instead of running every predictor twice."""
    if dt_sched is None:
        dt_sched = dt_schedule(mesh, u0, n_steps)
    u0 = u0.detach().clone().requires_grad_(True)
    uT = Rollout.apply(u0, mesh, dt_sched, n_steps, k, record)
    J = SampledMisfit.apply(uT, mesh, pts, target)
    J.backward()
    return J.detach(), u0.grad.detach(), dt_sched


def record_switches(mesh, u0, dt_sched, n_steps):
    """Rusanov switch tapes (one per step) of the unperturbed run."""
    tapes = torch.zeros((n_steps, mesh.info["n_conforming_faces"]), dtype=torch.int16, device=u0.device)
    u = u0.detach().clone()
    bufs = _Buffers(mesh)
    for n in range(n_steps):
        mesh.set_switch_tape(tapes[n], 1)
        advance_fixed(mesh, u, dt_sched, n, n + 1, bufs)
    mesh.set_switch_tape(None, 0)
    return tapes


def loss_fixed(mesh, u0, pts, target, dt_sched, n_steps, tapes=None):
    """J at the frozen schedule without recording a graph (for finite
    differences); with tapes, the Rusanov switches are replayed as well."""
    u = u0.detach().clone()
    bufs = _Buffers(mesh)
    if tapes is None:
        advance_fixed(mesh, u, dt_sched, 0, n_steps, bufs)
    else:
        for n in range(n_steps):
            mesh.set_switch_tape(tapes[n], 2)
            advance_fixed(mesh, u, dt_sched, n, n + 1, bufs)
        mesh.set_switch_tape(None, 0)
    vals = torch.empty(pts.shape[0], dtype=torch.float64, device=u.device)
    mesh.sample(u, pts, vals)
    r = vals - target
    return 0.5 * float((r * r).sum())
