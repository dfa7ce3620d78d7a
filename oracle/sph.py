"""FP64 oracle of the SPH density with an iterated smoothing length.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to produce expected values.
It imports nothing from the GPU package and the GPU package never imports it.

The paper's density module iterates each particle's smoothing length until its
kernel sphere holds a fixed number of neighbours (Sec. 2); it names no kernel
or criterion.  This follows Gadget-2's SPH density (Springel 2005):

* the cubic-spline kernel with support h,
  W(r, h) = 8 / (pi h^3) w(r / h),
  w(q) = 1 - 6 q^2 + 6 q^3 (q <= 1/2),  2 (1 - q)^3 (1/2 < q <= 1),  0 beyond;
* the density rho_i(h) = sum_j m_j W(|x_j - x_i|, h) over all particles j,
  the particle itself included, with minimum-image separations;
* the mass-weighted neighbour number N_i(h) = (4 pi / 3) h^3 rho_i(h) / m_i
  = (32 / 3) sum_j (m_j / m_i) w(r_ij / h).

Gadget stops its iteration once N_i lies within a tolerance band around the
desired number T, so its h depends on the path taken.  Here h_i is the root of
N_i(h) = T, which is unique: N_i(h) is constant (32/3, the particle alone)
below the nearest neighbour and strictly increasing once any neighbour lies
within h.  The root is found by bisection to the last bit, and rho_i is taken
at that h.  The distances of each particle's nearest neighbours come from
scipy's periodic k-d tree (a library step); the list is lengthened until the
bracket's upper end holds the root.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def w(q):
    """The cubic spline's shape w(q), q = r / h."""
    q = np.asarray(q, dtype=np.float64)
    inner = 1.0 - 6.0 * q * q + 6.0 * q * q * q
    outer = 2.0 * (1.0 - q) ** 3
    return np.where(q <= 0.5, inner, np.where(q <= 1.0, outer, 0.0))


def kernel(r, h):
    """W(r, h) = 8 / (pi h^3) w(r / h)."""
    return 8.0 / (np.pi * h ** 3) * w(np.asarray(r) / h)


def neighbour_number(dist, mass_ratio, h):
    """N(h) = (32 / 3) sum_j (m_j / m_i) w(r_j / h) over the rows of `dist`
    (one row per particle, the particle itself at distance 0)."""
    h = np.asarray(h, dtype=np.float64)[..., None]
    return 32.0 / 3.0 * (mass_ratio * w(dist / h)).sum(axis=-1)


def wrap(pos, box):
    """Positions mapped into [0, L)."""
    u = np.asarray(pos, dtype=np.float64) / box
    u = u - np.floor(u)
    u[u >= 1.0] = 0.0
    return u * box


def density(pos, mass, box: float, n_ngb: float = 64.0, targets=None, k0: int = 128):
    """(h, rho) of the particles `targets` (default all), input order.

    h is the root of N(h) = n_ngb by bisection; rho = rho(h).  Requires
    n_ngb > 32/3 and a root below L/4 (raises otherwise)."""
    x = wrap(pos, box)
    n = len(x)
    mass = np.broadcast_to(np.asarray(mass, dtype=np.float64), (n,))
    tg = np.arange(n) if targets is None else np.asarray(targets)
    if not n_ngb > 32.0 / 3.0:
        raise ValueError("n_ngb must exceed 32/3 (the particle alone)")
    tree = cKDTree(x, boxsize=box)
    h = np.empty(len(tg))
    rho = np.empty(len(tg))
    todo = np.arange(len(tg))
    k = min(k0, n)
    while todo.size:
        dist, idx = tree.query(x[tg[todo]], k=k)
        dist = dist.reshape(len(todo), k)
        idx = idx.reshape(len(todo), k)
        ratio = mass[idx] / mass[tg[todo]][:, None]
        hi = dist[:, -1].copy()
        ok = neighbour_number(dist, ratio, hi) >= n_ngb
        if k < n and not ok.all():
            # the k nearest do not reach the root for some: lengthen their lists
            done = todo[ok]
            sel = ok
        else:
            done = todo
            sel = np.ones(len(todo), dtype=bool)
        if done.size:
            d, r, top = dist[sel], ratio[sel], hi[sel]
            if not (neighbour_number(d, r, top) >= n_ngb).all():
                raise ValueError("fewer particles than the neighbour number needs")
            lo = np.zeros(len(done))
            up = top
            for _ in range(80):
                mid = 0.5 * (lo + up)
                below = neighbour_number(d, r, mid) < n_ngb
                lo = np.where(below, mid, lo)
                up = np.where(below, up, mid)
            if (up > box / 4).any():
                raise ValueError("the neighbour number is not reached within L/4")
            h[done] = up
            m_j = r * mass[tg[done]][:, None]
            rho[done] = (m_j * kernel(d, up[:, None])).sum(axis=1)
        todo = todo[~sel]
        k = min(2 * k, n)
    return h, rho
