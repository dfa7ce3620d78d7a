"""Autograd re-evaluation of the oracle's frozen interaction lists (PyTorch, CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Given the interaction lists the oracle's walk
recorded (which node or particle each target took as a source), this module
re-evaluates L = sum_t w_t . a_t as a differentiable function of the particle
positions and masses -- node masses and centres of mass recomputed from their
member particles -- so that torch.autograd yields a gradient by a route that
shares nothing with the hand-written adjoint of ``oracle.c``.  This is how the
adjoint is pinned: decisions and topology frozen, everything else traced.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .oracle import H_PER_EPS


def _g_short(u):
    return torch.special.erfc(u) + (2.0 / math.sqrt(math.pi)) * u * torch.exp(-u * u)


def _spline_S(r, h):
    q = r / h
    qs = torch.clamp(q, min=0.5)          # keeps the outer branch finite where unused
    rs = torch.clamp(r, min=1e-300)
    inner = (32.0 / 3.0 + q * q * (32.0 * q - 192.0 / 5.0)) / h ** 3
    outer = (64.0 / 3.0 - 48.0 * qs + 192.0 / 5.0 * qs * qs - 32.0 / 3.0 * qs ** 3
             - 1.0 / (15.0 * qs ** 3)) / h ** 3
    far = 1.0 / torch.where(q >= 1.0, rs, h) ** 3
    return torch.where(q < 0.5, inner, torch.where(q < 1.0, outer, far))


def pair_accel(d, M, h, G, r_s):
    r2 = (d * d).sum(-1)
    r = torch.sqrt(torch.clamp(r2, min=1e-300))
    K = G * _spline_S(r, h) * _g_short(r / (2.0 * r_s))
    return (M * K)[:, None] * d


def frozen_loss(tree, starts, entries, targets, xw, mass, params, w):
    """L(xw, mass) with the lists (starts, entries) of the oracle tree `tree`.

    xw (n, 3) and mass (n,) are torch float64 tensors (wrapped positions); w is
    the (n_t, 3) cotangent.  Returns (L, acc) with acc the (n_t, 3) accelerations.
    """
    n = tree.n
    box = tree.box
    m_nodes = tree.n_nodes
    hs = torch.as_tensor(H_PER_EPS * tree.eps)
    # node moments from explicit (node, member) pairs
    rows = np.repeat(np.arange(m_nodes), tree.count[:m_nodes])
    cols = np.concatenate([tree.perm[f:f + c] for f, c in zip(tree.first[:m_nodes],
                                                              tree.count[:m_nodes])]) \
        if m_nodes else np.zeros(0, np.int64)
    rows_t = torch.as_tensor(rows)
    cols_t = torch.as_tensor(cols)
    Mn = torch.zeros(max(m_nodes, 1), dtype=torch.float64).index_add(0, rows_t, mass[cols_t])
    Sn = torch.zeros((max(m_nodes, 1), 3), dtype=torch.float64).index_add(
        0, rows_t, mass[cols_t][:, None] * xw[cols_t])
    com = Sn / Mn[:, None]
    # interaction pairs
    targets = np.asarray(targets, np.int64)
    n_per = np.diff(starts)
    tslot = np.repeat(np.arange(targets.shape[0]), n_per)
    tidx = targets[tslot]
    ent = np.asarray(entries, np.int64)
    is_node = ent >= 0
    node_id = np.where(is_node, ent, 0)
    part_id = np.where(is_node, 0, -ent - 1)
    isn = torch.as_tensor(is_node)
    src = torch.where(isn[:, None], com[torch.as_tensor(node_id)], xw[torch.as_tensor(part_id)])
    Ms = torch.where(isn, Mn[torch.as_tensor(node_id)], mass[torch.as_tensor(part_id)])
    hsrc = np.where(is_node, tree.hmax[node_id], H_PER_EPS * tree.eps[part_id])
    h = torch.as_tensor(np.maximum(H_PER_EPS * tree.eps[tidx], hsrc))
    d = src - xw[torch.as_tensor(tidx)]
    d = torch.where(d > 0.5 * box, d - box, torch.where(d < -0.5 * box, d + box, d))
    F = pair_accel(d, Ms, h, params.get("G", 1.0), params["r_s"])
    acc = torch.zeros((targets.shape[0], 3), dtype=torch.float64).index_add(
        0, torch.as_tensor(tslot), F)
    L = (torch.as_tensor(w) * acc).sum()
    del hs, n
    return L, acc


def frozen_gradient(tree, params, w, targets=None, a_old=None):
    """dL/dx, dL/dm by autograd through the frozen lists of the oracle's walk."""
    from . import oracle as O
    tg = np.arange(tree.n) if targets is None else np.asarray(targets, np.int64)
    starts, entries = O.interaction_lists(tree, params, tg, a_old)
    xw = torch.tensor(tree.xw, dtype=torch.float64, requires_grad=True)
    m = torch.tensor(tree.mass, dtype=torch.float64, requires_grad=True)
    L, acc = frozen_loss(tree, starts, entries, tg, xw, m, params, w)
    L.backward()
    return xw.grad.numpy(), m.grad.numpy(), acc.detach().numpy()


def direct_pair_gradient(pos, mass, eps, params, w, box=1.0):
    """Exact short-range sum over all pairs within r_cut, and its autograd gradient.

    A dense O(N^2) pair search in torch (no tree at all); suitable for N of a few
    thousand.  Returns (acc, dL/dx, dL/dm).
    """
    pos = np.asarray(pos, np.float64)
    u = pos / box
    u = u - np.floor(u)
    u[u >= 1.0] = 0.0
    xw_np = u * box
    n = xw_np.shape[0]
    xw = torch.tensor(xw_np, requires_grad=True)
    m = torch.tensor(np.broadcast_to(np.asarray(mass, np.float64), (n,)).copy(), requires_grad=True)
    hs = torch.as_tensor(H_PER_EPS * np.broadcast_to(np.asarray(eps, np.float64), (n,)))
    with torch.no_grad():
        dd = xw[None, :, :] - xw[:, None, :]
        dd = torch.where(dd > 0.5 * box, dd - box, torch.where(dd < -0.5 * box, dd + box, dd))
        r2 = (dd * dd).sum(-1)
        mask = r2 < params["r_cut"] ** 2
        mask.fill_diagonal_(False)
        ii, jj = torch.nonzero(mask, as_tuple=True)
    d = xw[jj] - xw[ii]
    d = torch.where(d > 0.5 * box, d - box, torch.where(d < -0.5 * box, d + box, d))
    F = pair_accel(d, m[jj], torch.maximum(hs[ii], hs[jj]), params.get("G", 1.0), params["r_s"])
    acc = torch.zeros((n, 3), dtype=torch.float64).index_add(0, ii, F)
    L = (torch.as_tensor(np.asarray(w, np.float64)) * acc).sum()
    L.backward()
    return acc.detach().numpy(), xw.grad.numpy(), m.grad.numpy()
