"""Pins of the oracle's unequal-softening reading, independent of the oracle.

With particles of different softening lengths the walk also opens a node whose
particles do not share one support h while the target lies within the largest
of them (r_COM^2 < h_max^2 and h_min != h_max), so that a pair inside a support
is never replaced by a node moment (the unequal-softening option of Gadget,
which the paper's code descends from; paper Sec. 2 walks the tree per active
particle).  These tests fix that reading from outside the oracle:

* h_max and h_min of every node are recomputed with numpy from the node's
  particle range of the sorted order;
* on a compact clump (nothing pruned), every node a target accepts fails every
  opening test and every ancestor of an interaction passes one, all evaluated
  here in numpy geometry;
* hand-built three-particle trees with exact binary geometry put the target
  between h_min and h_max (the node must be opened), exactly at h_max (strict
  comparison: accepted), and inside h of a node of equal softenings (accepted).
"""
import numpy as np
import pytest

H_PER_EPS = 2.8


def _params(r_s, theta=0.5):
    return dict(G=1.0, r_s=r_s, r_cut=4.5 * r_s, theta=theta, criterion="bh", alpha=0.0)


def _node_h_range(t):
    """Largest and smallest support over each node's particles (numpy, sorted ranges)."""
    m = t.n_nodes
    h_sorted = H_PER_EPS * t.eps[t.perm]
    hx = np.array([h_sorted[t.first[k]:t.first[k] + t.count[k]].max() for k in range(m)])
    hn = np.array([h_sorted[t.first[k]:t.first[k] + t.count[k]].min() for k in range(m)])
    return hx, hn


def _mi(d, L=1.0):
    return np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))


def _opening(t, nd, xi, theta, hx, hn, L=1.0):
    """(guard, bh, mixed) opening tests of node nd for a target at xi, in numpy."""
    lev = int(t.level[nd])
    l = L * 2.0 ** -lev
    c = L * (t.corner[nd].astype(np.float64) / 2.0 ** 32 + 2.0 ** -(lev + 1))
    dc = _mi(c - xi, L)
    guard = bool(np.all(np.abs(dc) < 0.6 * l))
    d = _mi(t.com[nd] - xi, L)
    r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    bh = bool(l * l > (theta * theta) * r2)
    mixed = bool(hn[nd] != hx[nd] and r2 < hx[nd] * hx[nd])
    return guard, bh, mixed


def test_node_h_range_matches_numpy(oracle):
    rng = np.random.default_rng(31)
    n = 900
    pos = 0.5 + 0.01 * rng.standard_normal((n, 3))
    eps = np.where(rng.random(n) < 0.25, 1 / 1200, 1 / 300)
    t = oracle.Tree(pos, 1.0 / n, eps)
    hx, hn = _node_h_range(t)
    assert np.array_equal(t.hmax[:t.n_nodes], hx)
    assert np.array_equal(t.hmin[:t.n_nodes], hn)
    assert np.any(hx != hn) and np.any(hx == hn)


def test_clump_decisions_follow_the_mixed_rule(oracle):
    # 1/4 of the particles with a quarter of the softening; every pair lies within
    # r_cut, so no subtree is pruned and the visited nodes are exactly the accepted
    # ones and the ancestors of every interaction
    rng = np.random.default_rng(32)
    n = 700
    pos = 0.5 + 0.01 * rng.standard_normal((n, 3))
    eps = np.where(rng.random(n) < 0.25, 1 / 1200, 1 / 300)
    p = _params(r_s=0.05)
    t = oracle.Tree(pos, 1.0 / n, eps)
    hx, hn = _node_h_range(t)
    starts, ent = oracle.interaction_lists(t, p)
    invperm = np.empty(n, np.int64)
    invperm[t.perm] = np.arange(n)
    opened_by_mixed_only = 0
    accepted_nodes = 0
    for i in range(0, n, 7):
        xi = t.xw[i]
        cover = np.zeros(n, np.int64)
        ancestors = set()
        for e in ent[starts[i]:starts[i + 1]]:
            if e >= 0:
                g, b, mx = _opening(t, e, xi, p["theta"], hx, hn)
                assert not (g or b or mx), (i, e)
                accepted_nodes += 1
                cover[t.perm[t.first[e]:t.first[e] + t.count[e]]] += 1
                a = t.parent[e]
            else:
                cover[-e - 1] += 1
                a = t.pparent[invperm[-e - 1]]
            while a >= 0 and a not in ancestors:
                ancestors.add(int(a))
                a = t.parent[a]
        for a in ancestors:
            g, b, mx = _opening(t, a, xi, p["theta"], hx, hn)
            assert g or b or mx, (i, a)
            opened_by_mixed_only += int(mx and not (g or b))
        assert cover[i] == 0 and np.all(np.delete(cover, i) == 1)
    # the sample exercises both outcomes of the mixed rule
    assert opened_by_mixed_only > 50 and accepted_nodes > 50


def _eps_for_support(h):
    """A softening whose support 2.8 eps rounds to exactly h in FP64."""
    e = h / H_PER_EPS
    for _ in range(64):
        got = H_PER_EPS * e
        if got == h:
            return e
        e = np.nextafter(e, np.inf) if got < h else np.nextafter(e, -np.inf)
    raise AssertionError("no softening maps to the support")


def _three_body(oracle, r, h_big, h_small, pair_eps=None):
    """Target (input 0) at distance r along -x from the COM (1/2, 1/2, c) of a close
    pair (inputs 1, 2: one of support h_big, one of h_small unless given)."""
    e_big, e_small = _eps_for_support(h_big), _eps_for_support(h_small)
    c, delta = 0.5 + 2.0 ** -6 + 2.0 ** -20, 2.0 ** -23
    pos = np.array([[0.5 - r, 0.5, c], [0.5, 0.5, c + delta], [0.5, 0.5, c - delta]])
    eps = np.array([e_small, e_big, e_small]) if pair_eps is None else np.array([e_small, *pair_eps])
    t = oracle.Tree(pos, np.full(3, 0.25), eps)
    # the pair forms one node whose COM is exact, and the geometry is exact; the node
    # is small enough that Barnes-Hut alone accepts it (l^2 <= theta^2 r^2)
    assert t.n_nodes == 2
    pair = [k for k in range(2) if t.count[k] == 2][0]
    assert (2.0 ** -int(t.level[pair])) ** 2 <= 0.25 * r * r / 64
    assert np.array_equal(t.com[pair], [0.5, 0.5, c]) and t.xw[0, 0] == 0.5 - r
    return t, pair


def _entries_of_target(oracle, t, p):
    starts, ent = oracle.interaction_lists(t, p, targets=np.array([0]))
    return sorted(int(e) for e in ent[starts[0]:starts[1]])


def test_hand_node_inside_h_max_is_opened(oracle):
    # h_min < r < h_max: Barnes-Hut accepts the tiny node, the mixed rule opens it;
    # a rule on the target's own support (h_min here) or on h_min would accept it
    h_big, h_small, r = 2.0 ** -4, 2.0 ** -7, 2.0 ** -5
    t, pair = _three_body(oracle, r, h_big, h_small)
    p = _params(r_s=0.04)
    assert _entries_of_target(oracle, t, p) == [-3, -2]
    acc, cnt = oracle.walk(t, p, targets=np.array([0]))
    assert cnt.tolist() == [[2, 0]]


def test_hand_node_at_h_max_is_accepted(oracle):
    # r exactly h_max: r^2 == h_max^2 in FP64 and the comparison is strict, so the node
    # is accepted as one moment
    h_big, h_small = 2.0 ** -4, 2.0 ** -7
    t, pair = _three_body(oracle, h_big, h_big, h_small)
    p = _params(r_s=0.04)
    assert _entries_of_target(oracle, t, p) == [pair]
    acc, cnt = oracle.walk(t, p, targets=np.array([0]))
    assert cnt.tolist() == [[0, 1]]
    # just inside h_max the node is opened
    t2, _ = _three_body(oracle, h_big - 2.0 ** -20, h_big, h_small)
    assert _entries_of_target(oracle, t2, p) == [-3, -2]


def test_hand_equal_softening_node_is_accepted(oracle):
    # both particles of the node share one support: the mixed rule does not apply
    # even with the target well inside h, and Barnes-Hut accepts the node
    h_big, h_small, r = 2.0 ** -4, 2.0 ** -7, 2.0 ** -5
    e_big = _eps_for_support(h_big)
    t, pair = _three_body(oracle, r, h_big, h_small, pair_eps=(e_big, e_big))
    p = _params(r_s=0.04)
    assert _entries_of_target(oracle, t, p) == [pair]
    # the pair is applied with h = max(h_target, h_max): the softened force of the
    # node's mass at the COM
    acc, _ = oracle.walk(t, p, targets=np.array([0]))
    assert acc[0, 0] == pytest.approx(0.5 * oracle.spline_S(r, h_big) * oracle.g_short(r / 0.08) * r,
                                      rel=1e-14)
