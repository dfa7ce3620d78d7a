"""Pins of the PM (long-range) oracle against facts that do not come from the
oracle itself: mass conservation of the assignment, the exactly vanishing force
of a mesh-aligned lattice, momentum conservation (the assignment and the
interpolation share their weights and the spectral gradient is antisymmetric),
and the analytic long-range pair force G m [erf(u) - 2u/sqrt(pi) e^{-u^2}] / r^2,
u = r / 2 r_s, that the exp(-k^2 r_s^2) filter stands for."""
import numpy as np

from oracle import pm


def test_assignment_conserves_mass_and_lands_on_mesh_points():
    rng = np.random.default_rng(1)
    n_mesh, box = 16, 2.0
    pos = rng.uniform(-3.0, 5.0, (300, 3))
    mass = rng.uniform(0.5, 2.0, 300)
    rho = pm.cic_assign(pos, mass, box, n_mesh)
    h3 = (box / n_mesh) ** 3
    assert abs(rho.sum() * h3 - mass.sum()) <= 1e-12 * mass.sum()
    # a particle on a mesh point puts all its mass on that point
    rho1 = pm.cic_assign(np.array([[3 * box / n_mesh, 5 * box / n_mesh, 0.0]]), np.array([2.0]), box, n_mesh)
    assert rho1[3, 5, 0] * h3 == 2.0 and np.count_nonzero(rho1) == 1


def test_mesh_aligned_lattice_has_no_force():
    n_mesh = 16
    g = (np.arange(n_mesh) + 0.0) / n_mesh
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    mass = np.full(len(pos), 1.0 / len(pos))
    acc = pm.pm_accel(pos, mass, 1.0, n_mesh, r_s=1.25 / n_mesh)
    scale = 1.0 / len(pos) / (1.0 / n_mesh) ** 2       # G m / h^2
    assert np.abs(acc).max() <= 1e-10 * scale


def test_momentum_is_conserved():
    rng = np.random.default_rng(2)
    pos = rng.random((500, 3))
    mass = rng.uniform(0.1, 1.0, 500)
    acc = pm.pm_accel(pos, mass, 1.0, 32, r_s=1.25 / 32)
    p = (mass[:, None] * acc).sum(axis=0)
    assert np.abs(p).max() <= 1e-12 * (mass[:, None] * np.abs(acc)).sum()


def _pair_errors(n_mesh, d_cells, r_s_cells=1.25, trials=6):
    rng = np.random.default_rng(3)
    r_s = r_s_cells / n_mesh
    errs = []
    for _ in range(trials):
        c = rng.random(3)
        u = rng.standard_normal(3)
        d = d_cells / n_mesh * u / np.linalg.norm(u)
        acc = pm.pm_accel(np.array([c, c + d]), np.array([1.0, 1e-9]), 1.0, n_mesh, r_s)
        ref = pm.long_range_pair(d[None], 1.0, r_s)[0]
        errs.append(np.linalg.norm(acc[1] - ref) / np.linalg.norm(ref))
    return np.array(errs)


def test_pair_force_follows_the_long_range_kernel():
    # eight cells apart: mesh and periodic-image effects stay near 1%; a wrong sign,
    # normalisation or filter width is off by far more
    assert _pair_errors(128, 8).max() <= 0.02
    # three cells apart the CIC window matters: dividing it out twice (assignment and
    # interpolation) leaves ~1%, once ~5%, not at all ~8%
    assert _pair_errors(128, 3).mean() <= 0.025
