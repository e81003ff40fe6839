"""Receiver misfit and its gradient with respect to the per-cell sound speed.

J(c) = 1/2 dt sum_{n=1}^{Nt} sum_r (p_h(x_r, t^n) - d_r^n)^2, where p_h is the
pressure of the ADER-DG solution (linear acoustics, per-cell c, point source)
read at the receivers after each step.  The gradient is the discrete adjoint
of the whole time loop: the library's adjoint step (transpose of the step in
Q, plus the material derivative) swept backwards, with the receiver residuals
injected at each step.  States are checkpointed every `checkpoint` steps in
the forward run and each segment is recomputed once in the backward sweep; the
recomputation also keeps each step's forward face data, which the adjoint step
needs, instead of having it recomputed from the stored state.  With the
solver's predictor and volume kernels set to a lower format, the forward steps
and the adjoint steps both run their contractions in it.
"""
import torch

from .aderdg import Solver


class ReceiverMisfit(torch.autograd.Function):
    """J = ReceiverMisfit.apply(c, solver, Q0, dt, nsteps, data, checkpoint, t0).

    c: per-cell sound speed (CUDA float64, one per cell); solver: an acoustic
    Solver with its source and receivers already set; Q0: initial state (CUDA
    float64); data: [nsteps, nrec] CUDA float64 observed traces."""

    @staticmethod
    def forward(ctx, c, solver, Q0, dt, nsteps, data, checkpoint=20, t0=0.0):
        if not isinstance(solver, Solver):
            raise TypeError("solver must be an aderdg.Solver")
        # the library takes FP64 per-cell values; a lower-precision c is widened here
        c = c.detach().to(torch.float64).contiguous()
        solver.set_material(c)
        solver.set_state(Q0)
        solver.time = t0
        ckpts = {0: Q0.detach().clone()}
        traces = torch.empty((nsteps, solver.nrec), dtype=torch.float64, device=Q0.device)
        for k in range(nsteps):
            solver.step(dt, 1)
            solver.read_receivers(out=traces[k])
            if (k + 1) % checkpoint == 0 and k + 1 < nsteps:
                ckpts[k + 1] = solver.get_state(out=torch.empty_like(Q0))
        J = 0.5 * dt * torch.sum((traces - data) ** 2)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.checkpoint, ctx.t0 = solver, dt, nsteps, checkpoint, t0
        ctx.ckpts, ctx.traces, ctx.data = ckpts, traces, data
        ctx.c = c
        return J

    @staticmethod
    def backward(ctx, gJ):
        solver, dt, nsteps, K, t0 = ctx.solver, ctx.dt, ctx.nsteps, ctx.checkpoint, ctx.t0
        solver.set_material(ctx.c)
        Q0 = ctx.ckpts[0]
        lam = torch.zeros_like(Q0)
        grad = torch.zeros(solver.ncell, dtype=torch.float64, device=Q0.device)
        resid = (ctx.traces - ctx.data) * dt
        nseg = (nsteps + K - 1) // K
        for m in range(nseg - 1, -1, -1):
            start, end = m * K, min((m + 1) * K, nsteps)
            # recompute the states start .. end-1 of this segment and the face data of
            # the steps start+1 .. end
            states, faces = [ctx.ckpts[start]], []
            solver.set_state(ctx.ckpts[start])
            solver.time = t0 + start * dt
            nbytes = solver.face_bytes()
            for k in range(start, end):
                solver.step(dt, 1)
                faces.append(solver.copy_faces(torch.empty(nbytes, dtype=torch.uint8, device=Q0.device)))
                if k < end - 1:
                    states.append(solver.get_state(out=torch.empty_like(Q0)))
            for k in range(end, start, -1):
                # misfit at t^k (state after step k), then the adjoint of step k
                solver.receivers_adjoint(resid[k - 1].contiguous(), lam)
                solver.step_adjoint(dt, t0 + (k - 1) * dt, states[k - 1 - start], lam, grad,
                                    fwd_faces=faces[k - 1 - start])
            del states, faces
        ctx.adjoint_Q0 = lam
        return gJ * grad, None, None, None, None, None, None, None


def misfit(c, solver, Q0, dt, nsteps, data, checkpoint=20, t0=0.0):
    return ReceiverMisfit.apply(c, solver, Q0, dt, nsteps, data, checkpoint, t0)


def record(solver, c, Q0, dt, nsteps, t0=0.0):
    """Forward run returning the receiver traces [nsteps, nrec] (synthetic data)."""
    solver.set_material(c)
    solver.set_state(Q0)
    solver.time = t0
    traces = torch.empty((nsteps, solver.nrec), dtype=torch.float64, device=Q0.device)
    for k in range(nsteps):
        solver.step(dt, 1)
        solver.read_receivers(out=traces[k])
    return traces
