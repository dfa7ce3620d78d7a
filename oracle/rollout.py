"""Oracle kick-drift-kick rollouts (FP64, CPU).  TEST INFRASTRUCTURE ONLY.

`rollout` and `rollout_grad` follow the leapfrog definition step by step with
the oracle's tree walk and adjoint:

    v_half = v + dt/2 a(x),  x' = x + dt v_half,  v' = v_half + dt/2 a(x'),

and the transposed step in reverse order for L = sum(wx . x_final).
`frozen_replay` records every force evaluation's tree and interaction lists
and replays the rollout in PyTorch with those lists frozen, so autograd gives
the gradient of the same frozen-decision function by an independent route.
"""
from __future__ import annotations

import numpy as np
import torch

from . import oracle as O
from . import pm as PM
from .frozen import frozen_loss


def _mass_array(mass, n):
    return np.broadcast_to(np.asarray(mass, np.float64), (n,)).copy()


def accel(x, mass, eps, params, box=1.0, n_mesh=None):
    """Short-range tree force, plus the PM long-range force on an n_mesh^3 mesh
    (same r_s and G) when n_mesh is given: the whole TreePM force."""
    t = O.Tree(x, mass, eps, box)
    a, _ = O.walk(t, params)
    if n_mesh:
        a = a + PM.pm_accel(x, _mass_array(mass, len(x)), box, n_mesh, params["r_s"], params.get("G", 1.0))
    return a, t


def rollout(x0, v0, mass, eps, params, n_steps, dt, box=1.0, n_mesh=None):
    x = np.array(x0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    a, _ = accel(x, mass, eps, params, box, n_mesh)
    for _ in range(n_steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a, _ = accel(x, mass, eps, params, box, n_mesh)
        v = v + 0.5 * dt * a
    return x, v


def _adjoint(t, x, mass, params, w, box, n_mesh):
    g, _ = O.adjoint(t, params, w)
    if n_mesh:
        g = g + PM.pm_adjoint(x, _mass_array(mass, len(x)), box, n_mesh, params["r_s"], w, params.get("G", 1.0))[0]
    return g


def rollout_grad(x0, v0, mass, eps, params, n_steps, dt, wx, box=1.0, n_mesh=None):
    """dL/dx0, dL/dv0 of L = sum(wx . x_final) with the decisions of every force
    evaluation frozen (the oracle's adjoint at each evaluation, plus the PM
    adjoint when n_mesh is given)."""
    xs, vs = [np.array(x0, dtype=np.float64)], [np.array(v0, dtype=np.float64)]
    for _ in range(n_steps):
        x, v = rollout(xs[-1], vs[-1], mass, eps, params, 1, dt, box, n_mesh)
        xs.append(x)
        vs.append(v)
    xb = np.array(wx, dtype=np.float64)
    vb = np.zeros_like(xb)
    for k in reversed(range(n_steps)):
        a0, t0 = accel(xs[k], mass, eps, params, box, n_mesh)
        vh = vs[k] + 0.5 * dt * a0
        x1 = xs[k] + dt * vh
        _, t1 = accel(x1, mass, eps, params, box, n_mesh)
        xb = xb + _adjoint(t1, x1, mass, params, 0.5 * dt * vb, box, n_mesh)
        vb = vb + dt * xb
        xb = xb + _adjoint(t0, xs[k], mass, params, 0.5 * dt * vb, box, n_mesh)
    return xb, vb


def frozen_replay(x0, v0, mass, eps, params, n_steps, dt, box=1.0, n_mesh=None):
    """Returns f(x0_t, v0_t) -> x_final (torch), replaying the rollout with each
    force evaluation's tree topology and interaction lists recorded from the
    unperturbed run (and, with n_mesh, the PM force in PyTorch)."""
    recs = []
    x = np.array(x0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)

    def record(xx):
        t = O.Tree(xx, mass, eps, box)
        starts, ent = O.interaction_lists(t, params)
        a, _ = accel(xx, mass, eps, params, box, n_mesh)
        recs.append((t, starts, ent))
        return a

    a = record(x)
    for _ in range(n_steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = record(x)
        v = v + 0.5 * dt * a
    m_t = torch.as_tensor(np.broadcast_to(np.asarray(mass, np.float64), (x.shape[0],)).copy())
    tg = np.arange(x.shape[0])

    def acc_of(k, xt):
        t, starts, ent = recs[k]
        xw = xt - box * torch.floor(xt / box).detach()
        _, acc = frozen_loss(t, starts, ent, tg, xw, m_t, params, np.zeros((x.shape[0], 3)))
        if n_mesh:
            acc = acc + PM.pm_accel_torch(xt, m_t, box, n_mesh, params["r_s"], params.get("G", 1.0))
        return acc

    def f(x0_t, v0_t):
        xt, vt = x0_t, v0_t
        a_t = acc_of(0, xt)
        for k in range(n_steps):
            vt = vt + 0.5 * dt * a_t
            xt = xt + dt * vt
            a_t = acc_of(k + 1, xt)
            vt = vt + 0.5 * dt * a_t
        return xt, vt

    return f
