"""Pins of the oracle's drifted tree (CPU): a tree reused after its particles
moved, with its topology kept, its moments refolded and each node's cube grown
to hold its particles (paper App. A: between rebuilds the nodes drift with
their particles).

* zero displacement gives back the built tree bit for bit (every node array,
  half-sides equal to half the cell sides, identical walk);
* the refolded centres of mass are the mass-weighted means of the moved
  members (math.fsum), the masses unchanged;
* every node's half-side is the smallest cube half-width about its cell centre
  that holds its moved members and is at least half the cell side (containment
  plus attainment, which fix the maximum);
* with theta = 0 the walk of a drifted tree is the exact direct sum at the moved
  positions (the prune of the grown cubes drops no pair within r_cut, even for
  particles that left their cells);
* on a compact clump every target's sources partition the other particles;
* a hand case with exact binary coordinates where the grown cube changes the
  decision: the node is opened (two particle interactions) where the cell's own
  side would accept it beyond r_cut (none).
"""
import math

import numpy as np
import pytest

from paper_2606_17145_amd import workloads as WL


def params(r_s=1.25 / 28, theta=0.5, **kw):
    return dict(G=1.0, r_s=r_s, r_cut=4.5 * r_s, theta=theta, criterion="bh", alpha=0.0, **kw)


def cell(t, nd):
    lev = int(t.level[nd])
    side = math.ldexp(t.box, -lev)
    c = t.box * (np.ldexp(t.corner[nd].astype(np.float64), -32) + math.ldexp(1.0, -lev - 1))
    return c, side


@pytest.mark.parametrize("case", ["clustered", "duplicates", "mixed"])
def test_zero_drift_is_the_built_tree(oracle, case):
    rng = np.random.default_rng(21)
    n = 2500
    pos = WL.clustered_positions(rng, n, 6)
    eps = np.full(n, 1 / 420)
    if case == "duplicates":
        pos[100:140] = pos[100]
    if case == "mixed":
        eps[::4] /= 4
    t = oracle.Tree(pos, 1.0 / n, eps)
    d = t.drift(np.zeros((n, 3)))
    nt, nd = t.nodes(), d.nodes()
    for k in nt:
        assert np.array_equal(nt[k], nd[k]), k
    assert np.array_equal(nd["half"], 0.5 * np.ldexp(1.0, -nt["level"].astype(np.int64)))
    assert np.array_equal(d.X, t.X) and np.array_equal(d.xw, t.xw)
    p = params()
    a0, c0 = oracle.walk(t, p)
    a1, c1 = oracle.walk(d, p)
    assert np.array_equal(c0, c1) and np.array_equal(a0, a1)


def drifted_case(oracle, n=2000, seed=22, sigma=0.01):
    rng = np.random.default_rng(seed)
    pos = WL.clustered_positions(rng, n, 5)
    t = oracle.Tree(pos, rng.uniform(0.5, 1.5, n) / n, 1 / 420)
    disp = sigma * rng.standard_normal((n, 3))
    return t, t.drift(disp), disp


def test_drifted_moments_are_member_means(oracle):
    t, d, disp = drifted_case(oracle)
    nd = d.nodes()
    assert np.array_equal(nd["M"], t.nodes()["M"])
    assert np.array_equal(d.xw, t.xw + disp)
    for k in range(0, d.n_nodes, 7):
        mem = d.perm[d.first[k]:d.first[k] + d.count[k]]
        m = d.mass[mem]
        for ax in range(3):
            ref = math.fsum(m * d.xw[mem, ax]) / math.fsum(m)
            assert abs(nd["com"][k, ax] - ref) <= 1e-13 * max(abs(ref), 1.0)


def test_half_sides_hold_their_members_tightly(oracle):
    t, d, _ = drifted_case(oracle)
    grown = 0
    for k in range(d.n_nodes):
        c, side = cell(d, k)
        mem = d.perm[d.first[k]:d.first[k] + d.count[k]]
        off = np.abs(d.xw[mem] - c)
        h = d.half[k]
        assert h >= 0.5 * side
        assert np.all(off <= h)
        if h > 0.5 * side:
            grown += 1
            assert np.any(off == h)
    assert grown > d.n_nodes // 10   # the displacements move many particles out of their cells


@pytest.mark.parametrize("sigma", [0.003, 0.02])
def test_theta_zero_walk_of_drifted_tree_is_direct_sum(oracle, sigma):
    t, d, _ = drifted_case(oracle, n=2500, seed=23, sigma=sigma)
    p = params()
    acc0, cnt0 = oracle.walk(d, dict(p, theta=0.0))
    accd, cntd = oracle.direct(d.xw, d.mass, d.eps, p)
    assert np.array_equal(cnt0[:, 0], cntd) and np.all(cnt0[:, 1] == 0)
    scale = np.linalg.norm(accd, axis=1)
    assert np.all(np.linalg.norm(acc0 - accd, axis=1) <= 1e-13 * np.maximum(scale, 1e-6 * np.median(scale)))


def test_drifted_walk_partitions_mass(oracle):
    rng = np.random.default_rng(24)
    n = 600
    pos = 0.5 + 0.01 * rng.standard_normal((n, 3))
    t = oracle.Tree(pos, 1.0 / n, 1e-4)
    d = t.drift(0.004 * rng.standard_normal((n, 3)))
    p = params(r_s=0.05)
    starts, ent = oracle.interaction_lists(d, p)
    for i in range(0, n, 11):
        cover = np.zeros(n, np.int64)
        for e in ent[starts[i]:starts[i + 1]]:
            if e >= 0:
                cover[d.perm[d.first[e]:d.first[e] + d.count[e]]] += 1
            else:
                cover[-e - 1] += 1
        assert cover[i] == 0 and np.all(np.delete(cover, i) == 1)


def test_hand_case_grown_cube_opens_the_node(oracle):
    # A = (1/8, 1/8, 1/8) and B = (3/8, 1/8, 1/8) share the level-1 cell [0, 1/2)^3
    # (centre 1/4, side 1/2); C = (7/8, 7/8, 7/8) is a child of the root.  B moves
    # by +1/4 in x to (5/8, 1/8, 1/8): the node's half-side becomes 3/8 and its
    # centre of mass (3/8, 1/8, 1/8).  Seen from C the cell centre is 3/8 away on
    # every axis (minimum image), inside the enlarged cube of the grown side
    # (0.6 * 3/4 = 9/20), so the node is opened for any theta and C meets A and B
    # one by one (each at r^2 = 3/16 < r_cut^2).  With the cell's own side the
    # guard would not fire (3/8 > 0.6 * 1/2) and for theta^2 >= 2/3 the node would
    # be accepted at r^2 = 3/8 > r_cut^2: no interaction at all.
    pos = np.array([[0.125, 0.125, 0.125], [0.375, 0.125, 0.125], [0.875, 0.875, 0.875]])
    t = oracle.Tree(pos, 1.0, 1e-6)
    assert t.n_nodes == 2 and int(t.level[1]) == 1
    disp = np.zeros((3, 3))
    disp[1, 0] = 0.25
    d = t.drift(disp)
    assert d.half[1] == 0.375 and d.half[0] == 0.5
    assert np.array_equal(d.com[1], [0.375, 0.125, 0.125])
    p = dict(G=1.0, r_s=0.1, r_cut=0.45, criterion="bh", alpha=0.0)
    for th in (0.5, 0.9, 1.0, 1.5, 3.0):
        _, cnt = oracle.walk(d, dict(p, theta=th), targets=np.array([2]))
        assert cnt.tolist() == [[2, 0]], th
    # the built tree (B still in its cell) accepts the node for theta^2 >= 2/3
    _, cnt = oracle.walk(t, dict(p, theta=1.0), targets=np.array([2]))
    assert cnt.tolist() == [[0, 0]]
