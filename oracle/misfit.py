"""Receiver-misfit objective and its gradient on the CPU oracle (test infrastructure).

J(c) = 1/2 dt sum_{n=1}^{Nt} sum_r (p_h(x_r, t^n) - d_r^n)^2 for the acoustic
step with per-cell sound speed c; the gradient comes from the oracle's
reverse-mode step adjoint, sweeping the stored states backwards.
"""
import numpy as np


def forward(o, Q0, c, dt, nsteps, rec, data=None, t0=0.0):
    """Run nsteps; returns (J, receiver traces [nsteps][nrec], states[0..nsteps])."""
    o.set_material(c)
    o.set_state(Q0)
    states = [np.array(Q0, copy=True)]
    traces = []
    J = 0.0
    for k in range(nsteps):
        o.step(t0 + k * dt, dt)
        Q = o.get_state()
        states.append(Q)
        p = o.sample_points(rec, 0)
        traces.append(p)
        if data is not None:
            J += 0.5 * dt * float(np.sum((p - data[k]) ** 2))
    return J, np.array(traces), states


def gradient(o, Q0, c, dt, nsteps, rec, data, t0=0.0):
    """(J, dJ/dc, dJ/dQ0) by the adjoint sweep."""
    J, traces, states = forward(o, Q0, c, dt, nsteps, rec, data, t0)
    weights = [o.point_weights(x) for x in rec]
    lam = np.zeros(o.shape)
    grad = np.zeros(o.ncell)
    for k in range(nsteps, 0, -1):
        resid = traces[k - 1] - data[k - 1]
        for r, (cell, w) in enumerate(weights):
            lam[cell, 0, :] += dt * resid[r] * w
        lam, grad = o.adjoint_step(states[k - 1], t0 + (k - 1) * dt, dt, lam, grad)
    return J, grad, lam
