"""Pins of the SPH density oracle against facts that do not come from the
oracle itself: the kernel's normalisation (quadrature) and smoothness at its
knots, a closed-form root for a particle with equidistant neighbours, a pure
Python brute-force bisection on a small periodic set, the symmetry of a lattice
and the scaling of h and rho with lengths and masses."""
import math

import numpy as np
from scipy import integrate

from oracle import sph


def test_kernel_is_normalised_and_smooth():
    for h in (0.3, 1.0, 2.5):
        val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * float(sph.kernel(r, h)), 0, h, points=[h / 2])
        assert abs(val - 1.0) < 1e-12
    # value and slope continuous at q = 1/2; value and slope zero at q = 1
    e = 1e-7
    assert abs(float(sph.w(0.5 - e)) - float(sph.w(0.5 + e))) < 1e-6
    s_in = (float(sph.w(0.5)) - float(sph.w(0.5 - e))) / e
    s_out = (float(sph.w(0.5 + e)) - float(sph.w(0.5))) / e
    assert abs(s_in - s_out) < 1e-5 and abs(s_in + 1.5) < 1e-5       # w'(1/2) = -3/2
    assert float(sph.w(1.0)) == 0.0 and abs(float(sph.w(1.0 - e))) < 1e-18
    assert float(sph.w(0.0)) == 1.0 and float(sph.w(0.25)) == 1 - 6 / 16 + 6 / 64


def test_equidistant_neighbours_have_a_closed_form_root():
    # K equal masses at distance r0 from a centre, nothing else within reach:
    # (32/3)(1 + K w(r0/h)) = T, and with c = (3T/32 - 1)/K <= w(1/2) = 1/4 the
    # outer piece gives 2 (1 - q)^3 = c
    rng = np.random.default_rng(4)
    K, T, r0, box = 40, 64.0, 0.01, 1.0
    u = rng.standard_normal((K, 3))
    ring = 0.5 + r0 * u / np.linalg.norm(u, axis=1, keepdims=True)
    far = rng.uniform(0.0, 1.0, (400, 3))
    far = far[np.linalg.norm(far - 0.5, axis=1) > 0.2]
    pos = np.vstack([[0.5, 0.5, 0.5], ring, far])
    mass = np.ones(len(pos))
    h, rho = sph.density(pos, mass, box, T, targets=[0])
    c = (3 * T / 32 - 1) / K
    q = 1 - (c / 2) ** (1 / 3)
    assert abs(h[0] - r0 / q) <= 1e-12 * h[0]
    w_ring = 2 * (1 - q) ** 3
    assert abs(rho[0] - 8 / (math.pi * h[0] ** 3) * (1 + K * w_ring)) <= 1e-12 * rho[0]


def _brute(pos, mass, box, T, i):
    d = pos - pos[i]
    d -= box * np.round(d / box)
    r = [math.sqrt(x * x + y * y + z * z) for x, y, z in d]

    def N(h):
        return 32 / 3 * sum(mass[j] / mass[i] * float(sph.w(r[j] / h)) for j in range(len(r)))

    lo, hi = 0.0, box / 4
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if N(mid) < T:
            lo = mid
        else:
            hi = mid
    return hi, sum(mass[j] * float(sph.kernel(r[j], hi)) for j in range(len(r)))


def test_matches_brute_force_on_a_small_periodic_set():
    rng = np.random.default_rng(5)
    pos = rng.uniform(-1.0, 2.0, (1000, 3))         # unwrapped: the oracle wraps
    mass = rng.uniform(0.5, 1.5, 1000)
    tg = [0, 17, 123, 999]
    h, rho = sph.density(pos, mass, 1.0, 32.0, targets=tg, k0=16)
    for a, i in enumerate(tg):
        hb, rb = _brute(pos, mass, 1.0, 32.0, i)
        assert abs(h[a] - hb) <= 1e-13 * hb and abs(rho[a] - rb) <= 1e-12 * rb


def test_lattice_symmetry_and_scaling():
    # every particle of a periodic cubic lattice sees the same neighbourhood
    g = (np.arange(12) + 0.5) / 12
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    h, rho = sph.density(lat, np.ones(len(lat)), 1.0, 64.0, targets=[0, 500, 1727])
    assert np.ptp(h) <= 1e-13 * h[0] and np.ptp(rho) <= 1e-12 * rho[0]
    # dimensional analysis: lengths times s -> h times s, rho over s^3; masses
    # times c -> h unchanged, rho times c
    rng = np.random.default_rng(6)
    pos = rng.random((2000, 3))
    mass = rng.uniform(0.5, 1.5, 2000)
    tg = np.arange(0, 2000, 97)
    h1, r1 = sph.density(pos, mass, 1.0, 48.0, targets=tg)
    h2, r2 = sph.density(pos * 4.0, mass * 3.0, 4.0, 48.0, targets=tg)
    assert np.abs(h2 / h1 - 4.0).max() <= 1e-12 and np.abs(r2 / r1 - 3.0 / 64.0).max() <= 1e-12 * 3 / 64
