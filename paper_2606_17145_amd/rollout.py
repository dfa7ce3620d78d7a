"""Kick-drift-kick leapfrog rollouts of the short-range force, differentiated
with checkpointing and recomputation of the tree.

One step (state x, v; the state is kept unwrapped, only the tree wraps):

    v_half = v + dt/2 a(x)
    x'     = x + dt v_half        (tree rebuilt at x')
    v'     = v_half + dt/2 a(x')

The backward pass walks the steps in reverse.  For step k it restores the
checkpoint (x_k, v_k), rebuilds the trees at x_k and x_k' and re-runs the two
forward walks (so the adjoint walks see the forward's decisions), then applies
the transposed step:

    x'bar += A'(x')^T (dt/2 v'bar),  v_half bar = v'bar + dt x'bar,
    x bar  = x'bar + A'(x)^T (dt/2 v_half bar),  v bar = v_half bar.

With a PM handle (`pm`), a(x) is the whole TreePM force: the short-range tree
force plus the PM long-range force of the same r_s and G, and each adjoint
adds pm_accel_adjoint's position gradient.

Tree reuse (`rebuild_every = k`; paper App. A: between rebuilds the tree nodes
drift with their particles): force evaluation e (0 at the start, then one per
step) builds the tree when e is a multiple of k and otherwise drifts the last
build's tree to x_e (tree_drift by x_e - x_b, topology kept, moments and node
cubes refolded).  The backward pass recomputes a drifted evaluation's tree as
the build at the checkpoint x_b followed by the same drift.

Every arithmetic step runs in the HIP library: the forces and their adjoints
(shortrange_accel / shortrange_accel_adjoint, pm_accel / pm_accel_adjoint) and
the elementwise updates (sr_axpy).  This module only sequences the calls and
holds the checkpoints.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from . import Tree, shortrange_accel, shortrange_accel_adjoint


def _axpy(y: torch.Tensor, x: torch.Tensor, a: float):
    """y += a x on the device (sr_axpy)."""
    codes = {torch.float64: 0, torch.float32: 1}
    assert y.is_contiguous() and x.is_contiguous() and y.numel() == x.numel()
    with torch.cuda.device(y.device):
        _lib.check(_lib.lib().sr_axpy(_lib.ptr(y), codes[y.dtype], _lib.ptr(x), codes[x.dtype], float(a),
                                      y.numel(), _lib.stream_handle()))


def _accel(tree: Tree, x, mass, eps, params, box, pm=None, base=None, built=False):
    """a(x) on `tree`: rebuilt at x, or (base given) drifted from its build at base
    (`built`: the tree already holds that build)."""
    if base is None:
        tree.build(x, mass, eps=eps, box=box)
    else:
        if not built:
            tree.build(base, mass, eps=eps, box=box)
        disp = x.clone()
        _axpy(disp, base, -1.0)
        tree.drift(disp)
    a, _ = shortrange_accel(tree, params, counts=False)
    if pm is not None:
        _axpy(a, pm.accel(x, mass, box=box, r_s=params["r_s"], G=params.get("G", 1.0)), 1.0)
    return a


def _adjoint(tree: Tree, x, mass, params, w, box, pm=None):
    # on the lists of the tree's last forward walk (its recomputation in this step)
    g, _ = shortrange_accel_adjoint(tree, params, w, list_token=tree.list_token)
    if pm is not None:
        gp, _ = pm.accel_adjoint(x, mass, w, box=box, r_s=params["r_s"], G=params.get("G", 1.0))
        _axpy(g, gp, 1.0)
    return g


def kdk_rollout(pos, vel, mass, eps, params: dict, n_steps: int, dt: float, box: float = 1.0,
                checkpoints: bool = False, pm=None, rebuild_every: int = 1):
    """Forward rollout.  Returns (x, v) after n_steps, plus the list of (x_k, v_k)
    checkpoints when `checkpoints` is set.  a(x_{k+1}) of one step's closing kick
    is the next step's opening kick, so n_steps + 1 force evaluations are made.
    `pm`: a PM handle to add the long-range force (TreePM).  `rebuild_every`:
    rebuild the tree at every k-th evaluation and drift it in between."""
    if rebuild_every < 1:
        raise ValueError("rebuild_every must be >= 1")
    x = pos.detach().to(torch.float64).contiguous().clone()
    v = vel.detach().to(torch.float64).contiguous().clone()
    tree = Tree()
    saved = []
    base = None
    a = _accel(tree, x, mass, eps, params, box, pm)
    if rebuild_every > 1:
        base = x.clone()
    for e in range(1, n_steps + 1):
        if checkpoints:
            saved.append((x.clone(), v.clone()))
        _axpy(v, a, 0.5 * dt)
        _axpy(x, v, dt)
        if e % rebuild_every == 0:
            a = _accel(tree, x, mass, eps, params, box, pm)
            base = x.clone()
        else:
            a = _accel(tree, x, mass, eps, params, box, pm, base=base, built=True)
        _axpy(v, a, 0.5 * dt)
    return (x, v, saved) if checkpoints else (x, v)


def kdk_rollout_grad(pos, vel, mass, eps, params: dict, n_steps: int, dt: float, wx, wv=None,
                     box: float = 1.0, pm=None, rebuild_every: int = 1):
    """Gradient of L = sum(wx . x_final) + sum(wv . v_final) with respect to the
    initial positions and velocities.  Returns (dL/dx0, dL/dv0, x_final, v_final)."""
    x_fin, v_fin, saved = kdk_rollout(pos, vel, mass, eps, params, n_steps, dt, box, checkpoints=True, pm=pm,
                                      rebuild_every=rebuild_every)

    def base_of(e):
        # positions of the build that evaluation e drifts (a checkpoint), or None
        return None if e % rebuild_every == 0 else saved[e - e % rebuild_every][0]

    dev = x_fin.device
    wdt = torch.float32 if params.get("precision", "fp64") == "fp32" else torch.float64
    xb = wx.detach().to(torch.float64).contiguous().clone()
    vb = (torch.zeros_like(xb) if wv is None else wv.detach().to(torch.float64).contiguous().clone())
    t0, t1 = Tree(), Tree()
    w = torch.empty(xb.shape, dtype=wdt, device=dev)
    for k in reversed(range(n_steps)):
        x0, v0 = saved[k]
        # recompute step k: trees and forward walks at x0 and x1
        a0 = _accel(t0, x0, mass, eps, params, box, pm, base=base_of(k))
        x1 = x0.clone()
        vh = v0.clone()
        _axpy(vh, a0, 0.5 * dt)
        _axpy(x1, vh, dt)
        _accel(t1, x1, mass, eps, params, box, base=base_of(k + 1))  # the walk's lists at x1 (the PM needs none)
        # closing kick: v' = v_half + dt/2 a(x1)
        w.zero_()
        _axpy(w, vb, 0.5 * dt)
        _axpy(xb, _adjoint(t1, x1, mass, params, w, box, pm), 1.0)     # x1 bar
        _axpy(vb, xb, dt)                       # v_half bar = v' bar + dt x1 bar
        # opening kick: v_half = v + dt/2 a(x0)
        w.zero_()
        _axpy(w, vb, 0.5 * dt)
        _axpy(xb, _adjoint(t0, x0, mass, params, w, box, pm), 1.0)     # x0 bar = x1 bar + A'(x0)^T w
    return xb, vb, x_fin, v_fin
