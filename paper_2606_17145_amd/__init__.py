"""Short-range TreePM gravity on AMD Instinct MI355X.

The short-range half of a Gadget-style TreePM solver -- Morton-key octree
build, FP64 node moments, group-wise Barnes-Hut walk with the erfc-split,
spline-softened, minimum-image pair force -- as hand-written HIP kernels for
gfx950 behind a C ABI (``include/srgrav.h``).  This package is the thin torch
binding: tensors in, tensors out, every step on the device.

    tree = tree_build(pos, mass, eps=eps, box=1.0)
    acc, counts = shortrange_accel(tree, params)              # params: dict
    dLdx, dLdm = shortrange_accel_adjoint(tree, params, w,    # L = sum w . acc, on the
                                          list_token=tree.list_token)  # forward's lists
    acc = ShortRangeAccel.apply(pos, mass, eps, params)       # differentiable

``params`` keys: G, r_s, r_cut, theta, criterion ("bh" | "relative"), alpha,
precision ("fp64" | "fp32" | "fp32_acc64").
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import SrgravError  # noqa: F401

__all__ = ["Tree", "tree_build", "shortrange_accel", "shortrange_accel_noalloc", "shortrange_accel_adjoint", "ShortRangeAccel",
           "kdk_rollout", "SrgravError", "PM", "PMAccel", "pm_accel", "pm_accel_adjoint", "sph_density"]


def _dev_f64(x, n=None, name="tensor"):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    x = x.detach().to(torch.float64).contiguous()
    return x


class Tree:
    """An sr_tree handle: the device-resident tree of one particle set."""

    def __init__(self):
        self._h = C.c_void_p(None)
        self.n = 0
        self.box = 1.0
        self.device = None
        self.list_token = 0      # token of the interaction lists of the last shortrange_accel

    def __del__(self):
        try:
            if self._h:
                _lib.lib().tree_free(self._h)
                self._h = C.c_void_p(None)
        except Exception:
            pass

    def build(self, pos, mass, eps=None, eps_scalar=None, box=1.0):
        pos = _dev_f64(pos, name="pos")
        n = pos.shape[0]
        if pos.shape != (n, 3):
            raise ValueError("pos must have shape (N, 3)")
        mass = torch.as_tensor(mass, dtype=torch.float64, device=pos.device)
        mass = mass.expand(n).contiguous() if mass.dim() == 0 else mass.contiguous()
        eps_t = None
        if eps is not None and (not isinstance(eps, (int, float))):
            eps_t = torch.as_tensor(eps, dtype=torch.float64, device=pos.device)
            eps_t = eps_t.expand(n).contiguous() if eps_t.dim() == 0 else eps_t.contiguous()
        else:
            eps_scalar = float(eps if eps is not None else eps_scalar)
        with torch.cuda.device(pos.device):
            _lib.check(_lib.lib().tree_build(_lib.ptr(pos), _lib.ptr(mass), _lib.ptr(eps_t),
                                             float(eps_scalar or 0.0), n, float(box), 1,
                                             _lib.stream_handle(), C.byref(self._h)))
        self.n, self.box, self.device = n, float(box), pos.device
        self.list_token = 0      # a rebuild replaces the lists
        return self

    def drift(self, disp):
        """Move the particles to their built positions plus `disp` ((N, 3), input
        order) and refold moments and node cubes on the same topology (tree_drift)."""
        d = _dev_f64(disp, name="disp")
        if d.shape != (self.n, 3):
            raise ValueError(f"disp must have shape ({self.n}, 3)")
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().tree_drift(self._h, _lib.ptr(d), _lib.stream_handle()))
        self.list_token = 0      # a drift voids the lists' token
        return self

    def node_count(self) -> int:
        m = C.c_int64(0)
        _lib.check(_lib.lib().tree_node_count(self._h, C.byref(m)))
        return int(m.value)

    def walk_stats(self) -> dict:
        """Work statistics of the last walk on this handle."""
        s = (C.c_int64 * 4)()
        _lib.check(_lib.lib().tree_walk_stats(self._h, s))
        return dict(node_tests=int(s[0]), chunks=int(s[1]), units=int(s[2]), targets=int(s[3]))

    def export(self) -> dict:
        """Copies of the sorted keys, permutation and node arrays (device tensors)."""
        n, m = self.n, self.node_count()
        dev = self.device
        i32 = dict(dtype=torch.int32, device=dev)
        out = dict(key_hi=torch.empty(n, dtype=torch.int64, device=dev),
                   key_lo=torch.empty(n, dtype=torch.int64, device=dev),
                   perm=torch.empty(n, **i32), level=torch.empty(m, **i32),
                   first=torch.empty(m, **i32), count=torch.empty(m, **i32),
                   parent=torch.empty(m, **i32), skip=torch.empty(m, **i32),
                   corner=torch.empty((m, 3), **i32),
                   M=torch.empty(m, dtype=torch.float64, device=dev),
                   com=torch.empty((m, 3), dtype=torch.float64, device=dev),
                   M32=torch.empty(m, dtype=torch.float32, device=dev),
                   comX=torch.empty((m, 3), **i32),
                   side=torch.empty(m, dtype=torch.float64, device=dev))
        ex = _lib.SrTreeExport(*[_lib.ptr(out[k]) if out[k].numel() else None for k in
                                 ("key_hi", "key_lo", "perm", "level", "first", "count", "parent",
                                  "skip", "corner", "M", "com", "M32", "comX", "side")])
        with torch.cuda.device(dev):
            _lib.check(_lib.lib().tree_export(self._h, C.byref(ex), _lib.stream_handle()))
        return out


def tree_build(pos, mass, eps=None, box=1.0, tree: Tree | None = None) -> Tree:
    """Build (or rebuild in place) the tree of the particles (pos: (N, 3) CUDA tensor)."""
    t = tree if tree is not None else Tree()
    return t.build(pos, mass, eps=eps, box=box)


def _targets(tree: Tree, active):
    if active is None:
        return None, tree.n
    a = torch.as_tensor(active, device=tree.device).to(torch.int32).contiguous()
    if a.numel() == 0:
        # an empty subset still needs a non-NULL pointer (NULL means all particles)
        return torch.zeros(1, dtype=torch.int32, device=tree.device), 0
    return a, a.shape[0]


def shortrange_accel(tree: Tree, params: dict, active=None, a_old=None, counts: bool = True):
    """Short-range accelerations of all particles, or of `active` (input indices)."""
    prec = params.get("precision", "fp64")
    act, n_t = _targets(tree, active)
    dt = torch.float32 if prec == "fp32" else torch.float64
    acc = torch.empty((n_t, 3), dtype=dt, device=tree.device)
    cnt = torch.empty((n_t, 2), dtype=torch.int32, device=tree.device) if counts else None
    ao = None if a_old is None else _dev_f64(torch.as_tensor(a_old, device=tree.device), name="a_old")
    p = _lib.make_params(params)
    tok = C.c_int64(0)
    with torch.cuda.device(tree.device):
        _lib.check(_lib.lib().shortrange_accel(tree._h, C.byref(p), _lib.ptr(act), n_t, _lib.ptr(ao),
                                               _lib.ptr(acc), _lib.ptr(cnt), C.byref(tok),
                                               _lib.stream_handle()))
    tree.list_token = int(tok.value)
    return acc, cnt


def shortrange_accel_noalloc(tree: Tree, params: dict, active=None, a_old=None, out=None, counts=None):
    """shortrange_accel through the allocation-free entry point: the library's lists
    live in its fixed per-GPU buffer.  `out` / `counts`: optional preallocated
    outputs ((n_t, 3) and (n_t, 2) int32); missing ones are allocated here by torch."""
    prec = params.get("precision", "fp64")
    act, n_t = _targets(tree, active)
    dt = torch.float32 if prec == "fp32" else torch.float64
    acc = out if out is not None else torch.empty((n_t, 3), dtype=dt, device=tree.device)
    if acc.shape != (n_t, 3) or acc.dtype != dt or not acc.is_contiguous():
        raise ValueError(f"out must be a contiguous ({n_t}, 3) {dt} tensor")
    if counts is not None and (counts.shape != (n_t, 2) or counts.dtype != torch.int32
                               or not counts.is_contiguous()):
        raise ValueError(f"counts must be a contiguous ({n_t}, 2) int32 tensor")
    ao = None if a_old is None else _dev_f64(torch.as_tensor(a_old, device=tree.device), name="a_old")
    p = _lib.make_params(params)
    with torch.cuda.device(tree.device):
        _lib.check(_lib.lib().shortrange_accel_noalloc(tree._h, C.byref(p), _lib.ptr(act), n_t,
                                                       _lib.ptr(ao), _lib.ptr(acc), _lib.ptr(counts),
                                                       _lib.stream_handle()))
    tree.list_token = 0      # no token names these lists; the handle's earlier token is void
    return acc, counts


def shortrange_accel_adjoint(tree: Tree, params: dict, w, active=None, a_old=None, list_token: int = 0):
    """dL/dx (N, 3) and dL/dm (N) of L = sum_t w_t . a_t, decisions as in the forward.

    list_token: 0 repeats the forward's walk for `active` / `a_old`; a token from
    shortrange_accel (``tree.list_token`` right after it) differentiates that call on
    its own lists and targets (`active` then only sets the length of `w`)."""
    prec = params.get("precision", "fp64")
    act, n_t = _targets(tree, active)
    dt = torch.float32 if prec == "fp32" else torch.float64
    w = torch.as_tensor(w, device=tree.device).to(dt).contiguous()
    if w.shape != (n_t, 3):
        raise ValueError(f"w must have shape ({n_t}, 3)")
    dx = torch.empty((tree.n, 3), dtype=torch.float64, device=tree.device)
    dm = torch.empty(tree.n, dtype=torch.float64, device=tree.device)
    ao = None if a_old is None else _dev_f64(torch.as_tensor(a_old, device=tree.device), name="a_old")
    p = _lib.make_params(params)
    with torch.cuda.device(tree.device):
        _lib.check(_lib.lib().shortrange_accel_adjoint(tree._h, C.byref(p), _lib.ptr(act), n_t,
                                                       _lib.ptr(ao), _lib.ptr(w), _lib.ptr(dx),
                                                       _lib.ptr(dm), int(list_token), _lib.stream_handle()))
    if list_token == 0:
        tree.list_token = 0      # the repeated walk replaced the handle's lists
    return dx, dm


class ShortRangeAccel(torch.autograd.Function):
    """Differentiable short-range acceleration a(pos, mass).

    ShortRangeAccel.apply(pos, mass, eps, params[, box, active, a_old]) returns
    the accelerations of the targets (all particles, or `active`).  The backward
    runs the adjoint on the tree and interaction lists of the forward (kept on the
    context, named by their list token), so topology, opening decisions and
    cutoff membership are those of the forward pass.  The gradient flows to `pos`
    and, when it is a tensor, to `mass` (a 0-dimensional mass gets the sum).
    """

    @staticmethod
    def forward(ctx, pos, mass, eps, params, box=1.0, active=None, a_old=None):
        tree = tree_build(pos, mass, eps=eps, box=box)
        acc, _ = shortrange_accel(tree, params, active=active, a_old=a_old, counts=False)
        ctx.tree, ctx.params, ctx.active, ctx.a_old = tree, params, active, a_old
        ctx.token = tree.list_token
        ctx.pos_dtype = pos.dtype
        ctx.mass_kind = (mass.dtype, mass.dim()) if isinstance(mass, torch.Tensor) else None
        return acc

    @staticmethod
    def backward(ctx, grad):
        dx, dm = shortrange_accel_adjoint(ctx.tree, ctx.params, grad.contiguous(), active=ctx.active,
                                          a_old=ctx.a_old, list_token=ctx.token)
        if ctx.mass_kind is None:
            gm = None
        else:
            mdt, mdim = ctx.mass_kind
            gm = (dm if mdim > 0 else dm.sum()).to(mdt)
        return dx.to(ctx.pos_dtype), gm, None, None, None, None, None


class PM:
    """An sr_pm handle: mesh workspace and FFT plans of one n_mesh^3 periodic mesh."""

    def __init__(self, n_mesh: int):
        self._h = C.c_void_p(None)
        self.n_mesh = int(n_mesh)
        _lib.check(_lib.lib().pm_create(self.n_mesh, C.byref(self._h)))
        self.device = torch.device("cuda", torch.cuda.current_device())

    def __del__(self):
        try:
            if self._h:
                _lib.lib().pm_free(self._h)
                self._h = C.c_void_p(None)
        except Exception:
            pass

    def accel(self, pos, mass, *, box: float, r_s: float, G: float = 1.0):
        """Long-range (PM) accelerations (N, 3) float64 of all particles, input order."""
        pos = _dev_f64(pos, name="pos")
        n = pos.shape[0]
        if pos.shape != (n, 3):
            raise ValueError("pos must have shape (N, 3)")
        mass = torch.as_tensor(mass, dtype=torch.float64, device=pos.device)
        mass = mass.expand(n).contiguous() if mass.dim() == 0 else mass.contiguous()
        acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        with torch.cuda.device(pos.device):
            _lib.check(_lib.lib().pm_accel(self._h, _lib.ptr(pos), _lib.ptr(mass), n, float(box), float(r_s),
                                           float(G), _lib.ptr(acc), _lib.stream_handle()))
        return acc

    def accel_adjoint(self, pos, mass, w, *, box: float, r_s: float, G: float = 1.0):
        """(dL/dpos (N, 3), dL/dmass (N,)) float64 of L = sum(w * accel(pos, mass))."""
        pos = _dev_f64(pos, name="pos")
        n = pos.shape[0]
        if pos.shape != (n, 3):
            raise ValueError("pos must have shape (N, 3)")
        mass = torch.as_tensor(mass, dtype=torch.float64, device=pos.device)
        mass = mass.expand(n).contiguous() if mass.dim() == 0 else mass.contiguous()
        w = _dev_f64(w, name="w")
        if w.shape != (n, 3):
            raise ValueError("w must have shape (N, 3)")
        dpos = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        dmass = torch.empty(n, dtype=torch.float64, device=pos.device)
        with torch.cuda.device(pos.device):
            _lib.check(_lib.lib().pm_accel_adjoint(self._h, _lib.ptr(pos), _lib.ptr(mass), n, float(box), float(r_s),
                                                   float(G), _lib.ptr(w), _lib.ptr(dpos), _lib.ptr(dmass),
                                                   _lib.stream_handle()))
        return dpos, dmass


def _pm_handle(pm, n_mesh):
    h = pm if pm is not None else PM(n_mesh)
    if h.n_mesh != n_mesh:
        raise ValueError(f"pm handle has n_mesh {h.n_mesh}, not {n_mesh}")
    return h


def pm_accel_adjoint(pos, mass, w, *, box: float, n_mesh: int, r_s: float, G: float = 1.0, pm: PM | None = None):
    """(dL/dpos (N, 3), dL/dmass (N,)) of L = sum(w * pm_accel(pos, mass, ...))."""
    return _pm_handle(pm, n_mesh).accel_adjoint(pos, mass, w, box=box, r_s=r_s, G=G)


class PMAccel(torch.autograd.Function):
    """Differentiable PM accelerations: PMAccel.apply(pos, mass, pm, box, r_s[, G])."""

    @staticmethod
    def forward(ctx, pos, mass, pm, box, r_s, G=1.0):
        ctx.save_for_backward(pos, mass)
        ctx.args = (pm, float(box), float(r_s), float(G))
        ctx.dtypes = (pos.dtype, mass.dtype)
        return pm.accel(pos, mass, box=box, r_s=r_s, G=G)

    @staticmethod
    def backward(ctx, grad):
        pos, mass = ctx.saved_tensors
        pm, box, r_s, G = ctx.args
        dx, dm = pm.accel_adjoint(pos, mass, grad, box=box, r_s=r_s, G=G)
        dm = dm if mass.dim() > 0 else dm.sum()
        return dx.to(ctx.dtypes[0]), dm.to(ctx.dtypes[1]), None, None, None, None


def pm_accel(pos, mass, *, box: float, n_mesh: int, r_s: float, G: float = 1.0, pm: PM | None = None):
    """Long-range (PM) accelerations on an n_mesh^3 mesh (pass `pm` to reuse its plans)."""
    return _pm_handle(pm, n_mesh).accel(pos, mass, box=box, r_s=r_s, G=G)


def sph_density(tree: Tree, n_ngb: float = 64.0):
    """SPH smoothing lengths and densities (cubic spline; h the root of
    (4 pi/3) h^3 rho / m = n_ngb) of the particles of a built tree.
    Returns (h (N,), rho (N,), unconverged count), input order."""
    if not tree._h:
        raise ValueError("tree is not built")
    h = torch.empty(tree.n, dtype=torch.float64, device=tree.device)
    rho = torch.empty(tree.n, dtype=torch.float64, device=tree.device)
    bad = C.c_int64(0)
    with torch.cuda.device(tree.device):
        _lib.check(_lib.lib().sph_density(tree._h, float(n_ngb), _lib.ptr(h), _lib.ptr(rho), C.byref(bad),
                                          _lib.stream_handle()))
    return h, rho, int(bad.value)


def kdk_rollout(*args, **kwargs):
    from .rollout import kdk_rollout as _k
    return _k(*args, **kwargs)
