"""Oracle kick-drift-kick rollouts (FP64, CPU).  TEST INFRASTRUCTURE ONLY.

`rollout` and `rollout_grad` follow the leapfrog definition step by step with
the oracle's tree walk and adjoint:

    v_half = v + dt/2 a(x),  x' = x + dt v_half,  v' = v_half + dt/2 a(x'),

and the transposed step in reverse order for L = sum(wx . x_final).
`frozen_replay` records every force evaluation's tree and interaction lists
and replays the rollout in PyTorch with those lists frozen, so autograd gives
the gradient of the same frozen-decision function by an independent route.

`rebuild_every = k` reuses trees between rebuilds (paper App. A: the tree
nodes drift with their particles between rebuilds): force evaluation e (0 at
the start, then one per step) builds the tree when e is a multiple of k, and
otherwise drifts the tree of the last build by x_e - x_b (Tree.drift).
"""
from __future__ import annotations

import numpy as np
import torch

from . import oracle as O
from . import pm as PM
from .frozen import frozen_loss


def _mass_array(mass, n):
    return np.broadcast_to(np.asarray(mass, np.float64), (n,)).copy()


def accel(x, mass, eps, params, box=1.0, n_mesh=None, base=None):
    """Short-range tree force, plus the PM long-range force on an n_mesh^3 mesh
    (same r_s and G) when n_mesh is given: the whole TreePM force.  With `base`
    the tree is built at base and drifted to x."""
    t = O.Tree(x, mass, eps, box) if base is None else O.Tree(base, mass, eps, box).drift(x - base)
    a, _ = O.walk(t, params)
    if n_mesh:
        a = a + PM.pm_accel(x, _mass_array(mass, len(x)), box, n_mesh, params["r_s"], params.get("G", 1.0))
    return a, t


def _base_of(e, xs, rebuild_every):
    """Positions of the build that force evaluation e drifts, or None (a build)."""
    return None if e % rebuild_every == 0 else xs[e - e % rebuild_every]


def trajectory(x0, v0, mass, eps, params, n_steps, dt, box=1.0, n_mesh=None, rebuild_every=1):
    """The states (x_e, v_e), e = 0 .. n_steps, of the rollout."""
    xs, vs = [np.array(x0, dtype=np.float64)], [np.array(v0, dtype=np.float64)]
    a, _ = accel(xs[0], mass, eps, params, box, n_mesh)
    for e in range(1, n_steps + 1):
        v = vs[-1] + 0.5 * dt * a
        x = xs[-1] + dt * v
        xs.append(x)
        a, _ = accel(x, mass, eps, params, box, n_mesh, _base_of(e, xs, rebuild_every))
        vs.append(v + 0.5 * dt * a)
    return xs, vs


def rollout(x0, v0, mass, eps, params, n_steps, dt, box=1.0, n_mesh=None, rebuild_every=1):
    xs, vs = trajectory(x0, v0, mass, eps, params, n_steps, dt, box, n_mesh, rebuild_every)
    return xs[-1], vs[-1]


def _adjoint(t, x, mass, params, w, box, n_mesh):
    g, _ = O.adjoint(t, params, w)
    if n_mesh:
        g = g + PM.pm_adjoint(x, _mass_array(mass, len(x)), box, n_mesh, params["r_s"], w, params.get("G", 1.0))[0]
    return g


def rollout_grad(x0, v0, mass, eps, params, n_steps, dt, wx, box=1.0, n_mesh=None, rebuild_every=1):
    """dL/dx0, dL/dv0 of L = sum(wx . x_final) with the decisions of every force
    evaluation frozen (the oracle's adjoint at each evaluation, plus the PM
    adjoint when n_mesh is given)."""
    xs, vs = trajectory(x0, v0, mass, eps, params, n_steps, dt, box, n_mesh, rebuild_every)
    xb = np.array(wx, dtype=np.float64)
    vb = np.zeros_like(xb)
    for k in reversed(range(n_steps)):
        a0, t0 = accel(xs[k], mass, eps, params, box, n_mesh, _base_of(k, xs, rebuild_every))
        vh = vs[k] + 0.5 * dt * a0
        x1 = xs[k] + dt * vh
        _, t1 = accel(x1, mass, eps, params, box, n_mesh, _base_of(k + 1, xs, rebuild_every))
        xb = xb + _adjoint(t1, x1, mass, params, 0.5 * dt * vb, box, n_mesh)
        vb = vb + dt * xb
        xb = xb + _adjoint(t0, xs[k], mass, params, 0.5 * dt * vb, box, n_mesh)
    return xb, vb


def frozen_replay(x0, v0, mass, eps, params, n_steps, dt, box=1.0, n_mesh=None, rebuild_every=1):
    """Returns f(x0_t, v0_t) -> x_final (torch), replaying the rollout with each
    force evaluation's tree topology and interaction lists recorded from the
    unperturbed run (and, with n_mesh, the PM force in PyTorch).  A drifted
    evaluation places the particles at the built (wrapped) positions plus
    x - x_base, as the drifted tree does."""
    recs = []
    x = np.array(x0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    built = {}

    def record(xx, e):
        if e % rebuild_every == 0:
            t = O.Tree(xx, mass, eps, box)
            built["x"], built["xw"] = xx.copy(), t.xw.copy()
            drift = None
        else:
            t = O.Tree(built["x"], mass, eps, box).drift(xx - built["x"])
            drift = (torch.as_tensor(built["x"]), torch.as_tensor(built["xw"]))
        starts, ent = O.interaction_lists(t, params)
        a, _ = accel(xx, mass, eps, params, box, n_mesh, None if drift is None else built["x"])
        recs.append((t, starts, ent, drift))
        return a

    a = record(x, 0)
    for e in range(1, n_steps + 1):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = record(x, e)
        v = v + 0.5 * dt * a
    m_t = torch.as_tensor(np.broadcast_to(np.asarray(mass, np.float64), (x.shape[0],)).copy())
    tg = np.arange(x.shape[0])

    def acc_of(k, xt):
        t, starts, ent, drift = recs[k]
        if drift is None:
            xw = xt - box * torch.floor(xt / box).detach()
        else:
            xb, xwb = drift
            xw = xwb + (xt - xb)
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
