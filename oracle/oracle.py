"""Python face of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it to produce expected values.  It imports nothing
from the GPU package and the GPU package never imports it.

Every function takes and returns numpy arrays in input order.  Parameters are
given as a plain dict with keys G, r_s, r_cut, theta, criterion ("bh" or
"relative") and alpha.
"""
from __future__ import annotations

import copy
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

# Spline support per unit Plummer-equivalent softening (Springel, Yoshida & White 2001).
H_PER_EPS = 2.8


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", LIB_PATH + ".tmp",
               os.path.join(HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def use_native_build() -> str:
    """Compile oracle.c with -O3 -march=native for the machine this runs on and route
    every later call through that build (the same source and arithmetic: contraction
    and fast-math stay off).  Used to time the oracle on the host it runs on."""
    global _lib
    path = os.path.join(HERE, "liboracle_native.so")
    cmd = ["gcc", "-std=c99", "-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", path + ".tmp", os.path.join(HERE, "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    L = C.CDLL(path)
    _declare(L)
    _lib = L
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64 = C.c_int64
D = C.c_double


class CTree(C.Structure):
    _fields_ = [("n", I64), ("box", D), ("xw", P), ("mass", P), ("hsml", P), ("X", P),
                ("perm", P), ("pparent", P), ("n_nodes", I64), ("level", P), ("first", P),
                ("count", P), ("parent", P), ("skip", P), ("corner", P), ("child_start", P),
                ("child", P), ("M", P), ("com", P), ("hmax", P), ("hmin", P), ("half", P)]


class CParams(C.Structure):
    _fields_ = [("G", D), ("r_s", D), ("r_cut", D), ("criterion", C.c_int32), ("theta", D),
                ("alpha", D)]


def _declare(L):
    L.or_wrap_quantize.argtypes = [I64, P, D, P, P]
    L.or_morton.argtypes = [I64, P, P, P]
    L.or_sort.argtypes = [I64, P, P, P]
    L.or_build_topology.argtypes = [I64, P, P, P] + [P] * 9
    L.or_build_topology.restype = I64
    L.or_moments.argtypes = [C.POINTER(CTree)] + [P] * 7
    L.or_extents.argtypes = [C.POINTER(CTree), P]
    L.or_walk.argtypes = [C.POINTER(CTree), C.POINTER(CParams), I64, P, P, P, P]
    L.or_direct.argtypes = [I64, P, P, P, D, C.POINTER(CParams), I64, P, P, P]
    L.or_adjoint.argtypes = [C.POINTER(CTree), C.POINTER(CParams), I64, P, P, P, P, P, P, P]
    L.or_gradient_of.argtypes = [C.POINTER(CTree), C.POINTER(CParams), I64, P, P, P, I64, P, P, P]
    L.or_fd_gradient_of.argtypes = [C.POINTER(CTree), C.POINTER(CParams), P, I64, P, P, P, I64,
                                    P, D, D, P, P]
    L.or_interaction_lists.argtypes = [C.POINTER(CTree), C.POINTER(CParams), I64, P, P, I64, P, P]
    L.or_interaction_lists.restype = I64
    for name in ("or_g_short", "or_dg_short"):
        getattr(L, name).argtypes = [D]
        getattr(L, name).restype = D
    for name in ("or_spline_S", "or_spline_dS"):
        getattr(L, name).argtypes = [D, D]
        getattr(L, name).restype = D
    L.or_num_threads.restype = C.c_int


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def params_struct(p: dict) -> CParams:
    crit = {"bh": 0, "relative": 1}[p.get("criterion", "bh")]
    return CParams(float(p.get("G", 1.0)), float(p["r_s"]), float(p["r_cut"]), crit,
                   float(p.get("theta", 0.5)), float(p.get("alpha", 0.0)))


# --- elementary steps ------------------------------------------------------------

def wrap_quantize(pos, box=1.0):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    X = np.empty((n, 3), np.uint32)
    xw = np.empty((n, 3), np.float64)
    lib().or_wrap_quantize(n, _p(pos), float(box), _p(X), _p(xw))
    return X, xw


def morton(X):
    X = np.ascontiguousarray(X, dtype=np.uint32)
    n = X.shape[0]
    hi = np.empty(n, np.uint64)
    lo = np.empty(n, np.uint64)
    lib().or_morton(n, _p(X), _p(hi), _p(lo))
    return hi, lo


def sort_keys(hi, lo):
    n = hi.shape[0]
    perm = np.empty(n, np.int64)
    lib().or_sort(n, _p(np.ascontiguousarray(hi)), _p(np.ascontiguousarray(lo)), _p(perm))
    return perm


class Tree:
    """The oracle's tree: keys, sort, compressed pre-order octree and moments."""

    def __init__(self, pos, mass, eps, box=1.0):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        n = pos.shape[0]
        self.n = n
        self.box = float(box)
        self.mass = np.ascontiguousarray(np.broadcast_to(np.asarray(mass, np.float64), (n,)))
        self.eps = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float64), (n,)))
        self.hsml = H_PER_EPS * self.eps
        self.X, self.xw = wrap_quantize(pos, box)
        self.hi, self.lo = morton(self.X)
        self.perm = sort_keys(self.hi, self.lo)
        hs, ls = self.hi[self.perm].copy(), self.lo[self.perm].copy()
        Xs = np.ascontiguousarray(self.X[self.perm])
        cap = max(n - 1, 1)
        self.level = np.zeros(cap, np.int32)
        self.first = np.zeros(cap, np.int64)
        self.count = np.zeros(cap, np.int64)
        self.parent = np.zeros(cap, np.int64)
        self.skip = np.zeros(cap, np.int64)
        self.corner = np.zeros((cap, 3), np.uint32)
        self.child_start = np.zeros(cap + 1, np.int64)
        self.child = np.zeros(max(2 * n - 2, 1), np.int64)
        self.pparent = np.zeros(n, np.int64)
        m = lib().or_build_topology(n, _p(hs), _p(ls), _p(Xs), _p(self.level), _p(self.first),
                                    _p(self.count), _p(self.parent), _p(self.skip),
                                    _p(self.corner), _p(self.child_start), _p(self.child),
                                    _p(self.pparent))
        self.n_nodes = int(m)
        mm = max(m, 1)
        self.M = np.zeros(mm)
        self.S = np.zeros((mm, 3))
        self.com = np.zeros((mm, 3))
        self.M32 = np.zeros(mm, np.float32)
        self.comX = np.zeros((mm, 3), np.uint32)
        self.hmax = np.zeros(mm)
        self.hmin = np.zeros(mm)
        self.half = None         # set by drift(): node half-sides of a drifted tree
        self.ct = self._struct()
        lib().or_moments(C.byref(self.ct), _p(self.M), _p(self.S), _p(self.com), _p(self.M32),
                         _p(self.comX), _p(self.hmax), _p(self.hmin))

    def _struct(self) -> CTree:
        return CTree(self.n, self.box, _p(self.xw), _p(self.mass), _p(self.hsml), _p(self.X),
                     _p(self.perm), _p(self.pparent), self.n_nodes, _p(self.level),
                     _p(self.first), _p(self.count), _p(self.parent), _p(self.skip),
                     _p(self.corner), _p(self.child_start), _p(self.child), _p(self.M),
                     _p(self.com), _p(self.hmax), _p(self.hmin),
                     None if self.half is None else _p(self.half))

    def drift(self, disp):
        """The tree after its particles moved by `disp` (N x 3, input order) from where
        it was built: the same nodes and node order, the particles at the built
        (wrapped) positions plus disp (not wrapped again; their integer coordinates
        are those of the moved positions), the moments refolded in the build's order,
        and each node's cube grown to hold its particles (or_extents)."""
        disp = np.ascontiguousarray(disp, dtype=np.float64)
        assert disp.shape == (self.n, 3)
        d = copy.copy(self)
        base = self.xw if self.half is None else self.xw0
        d.xw0 = base
        d.xw = np.ascontiguousarray(base + disp)
        d.X, _ = wrap_quantize(d.xw, self.box)
        mm = max(self.n_nodes, 1)
        d.M = np.zeros(mm)
        d.S = np.zeros((mm, 3))
        d.com = np.zeros((mm, 3))
        d.M32 = np.zeros(mm, np.float32)
        d.comX = np.zeros((mm, 3), np.uint32)
        d.hmax = np.zeros(mm)
        d.hmin = np.zeros(mm)
        d.half = np.zeros(mm)
        d.ct = d._struct()
        lib().or_moments(C.byref(d.ct), _p(d.M), _p(d.S), _p(d.com), _p(d.M32), _p(d.comX),
                         _p(d.hmax), _p(d.hmin))
        if self.n_nodes > 0:
            lib().or_extents(C.byref(d.ct), _p(d.half))
        return d

    # node arrays trimmed to the node count
    def nodes(self) -> dict:
        m = self.n_nodes
        out = dict(level=self.level[:m], first=self.first[:m], count=self.count[:m],
                   parent=self.parent[:m], skip=self.skip[:m], corner=self.corner[:m],
                   M=self.M[:m], com=self.com[:m], M32=self.M32[:m], comX=self.comX[:m],
                   hmax=self.hmax[:m], hmin=self.hmin[:m])
        if self.half is not None:
            out["half"] = self.half[:m]
        return out

    def children(self, nd: int):
        """Children of node nd in digit order: ('node', k) or ('particle', sorted s)."""
        out = []
        for c in range(self.child_start[nd], self.child_start[nd + 1]):
            ch = int(self.child[c])
            out.append(("node", ch) if ch >= 0 else ("particle", -ch - 1))
        return out


def _targets(tree: Tree, targets):
    if targets is None:
        return np.arange(tree.n, dtype=np.int64)
    return np.ascontiguousarray(targets, dtype=np.int64)


def _aold(a_old):
    return None if a_old is None else np.ascontiguousarray(a_old, dtype=np.float64)


def walk(tree: Tree, params: dict, targets=None, a_old=None):
    """Accelerations (n_t, 3) and counts (n_t, 2) = (particle-particle, particle-node)."""
    tgt = _targets(tree, targets)
    acc = np.zeros((tgt.shape[0], 3))
    counts = np.zeros((tgt.shape[0], 2), np.int64)
    ao = _aold(a_old)
    ps = params_struct(params)
    lib().or_walk(C.byref(tree.ct), C.byref(ps), tgt.shape[0], _p(tgt),
                  None if ao is None else _p(ao), _p(acc), _p(counts))
    return acc, counts


def direct(pos, mass, eps, params: dict, box=1.0, targets=None):
    """Exact short-range sum over every pair within r_cut (the theta = 0 reference)."""
    X, xw = wrap_quantize(pos, box)
    n = xw.shape[0]
    mass = np.ascontiguousarray(np.broadcast_to(np.asarray(mass, np.float64), (n,)))
    hs = H_PER_EPS * np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float64), (n,)))
    tgt = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, np.int64)
    acc = np.zeros((tgt.shape[0], 3))
    counts = np.zeros(tgt.shape[0], np.int64)
    ps = params_struct(params)
    lib().or_direct(n, _p(xw), _p(mass), _p(hs), float(box), C.byref(ps), tgt.shape[0], _p(tgt),
                    _p(acc), _p(counts))
    return acc, counts


def adjoint(tree: Tree, params: dict, w, targets=None, a_old=None):
    """dL/dx (n, 3) and dL/dm (n) of L = sum_t w_t . a_t, decisions frozen."""
    tgt = _targets(tree, targets)
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert w.shape == (tgt.shape[0], 3)
    dx = np.zeros((tree.n, 3))
    dm = np.zeros(tree.n)
    mm = max(tree.n_nodes, 1)
    xbn = np.zeros((mm, 3))
    mbn = np.zeros(mm)
    ao = _aold(a_old)
    ps = params_struct(params)
    lib().or_adjoint(C.byref(tree.ct), C.byref(ps), tgt.shape[0], _p(tgt),
                     None if ao is None else _p(ao), _p(w), _p(dx), _p(dm), _p(xbn), _p(mbn))
    return dx, dm


def gradient_of(tree: Tree, params: dict, w, js, targets=None, a_old=None):
    """dL/dx_j and dL/dm_j for the particles js, each computed on its own."""
    tgt = _targets(tree, targets)
    w = np.ascontiguousarray(w, dtype=np.float64)
    js = np.ascontiguousarray(js, dtype=np.int64)
    gx = np.zeros((js.shape[0], 3))
    gm = np.zeros(js.shape[0])
    ao = _aold(a_old)
    ps = params_struct(params)
    lib().or_gradient_of(C.byref(tree.ct), C.byref(ps), tgt.shape[0], _p(tgt),
                         None if ao is None else _p(ao), _p(w), js.shape[0], _p(js), _p(gx), _p(gm))
    return gx, gm


def fd_gradient_of(tree: Tree, params: dict, w, js, hx=1e-6, hm_rel=1e-6, targets=None, a_old=None):
    """Central differences of the frozen-decision L for the particles js."""
    tgt = _targets(tree, targets)
    w = np.ascontiguousarray(w, dtype=np.float64)
    js = np.ascontiguousarray(js, dtype=np.int64)
    gx = np.zeros((js.shape[0], 3))
    gm = np.zeros(js.shape[0])
    ao = _aold(a_old)
    ps = params_struct(params)
    lib().or_fd_gradient_of(C.byref(tree.ct), C.byref(ps), _p(tree.S), tgt.shape[0], _p(tgt),
                            None if ao is None else _p(ao), _p(w), js.shape[0], _p(js),
                            float(hx), float(hm_rel), _p(gx), _p(gm))
    return gx, gm


def interaction_lists(tree: Tree, params: dict, targets=None, a_old=None):
    """Frozen interaction lists (CSR): entry >= 0 node index, < 0 particle -(j+1)."""
    tgt = _targets(tree, targets)
    start = np.zeros(tgt.shape[0] + 1, np.int64)
    ao = _aold(a_old)
    ps = params_struct(params)
    total = lib().or_interaction_lists(C.byref(tree.ct), C.byref(ps), tgt.shape[0], _p(tgt),
                                       None if ao is None else _p(ao), 0, _p(start), None)
    entries = np.zeros(max(total, 1), np.int64)
    lib().or_interaction_lists(C.byref(tree.ct), C.byref(ps), tgt.shape[0], _p(tgt),
                               None if ao is None else _p(ao), total, _p(start), _p(entries))
    return start, entries[:total]


def g_short(u: float) -> float:
    return lib().or_g_short(float(u))


def dg_short(u: float) -> float:
    return lib().or_dg_short(float(u))


def spline_S(r: float, h: float) -> float:
    return lib().or_spline_S(float(r), float(h))


def spline_dS(r: float, h: float) -> float:
    return lib().or_spline_dS(float(r), float(h))


def num_threads() -> int:
    return lib().or_num_threads()


def force_sum_norm(acc_ref: np.ndarray) -> np.ndarray:
    return np.linalg.norm(acc_ref, axis=1)
