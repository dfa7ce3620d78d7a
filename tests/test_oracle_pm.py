"""Pins of the PM (long-range) oracle against facts that do not come from the
oracle itself: mass conservation of the assignment, the exactly vanishing force
of a mesh-aligned lattice, momentum conservation (the assignment and the
interpolation share their weights and the spectral gradient is antisymmetric),
and the analytic long-range pair force G m [erf(u) - 2u/sqrt(pi) e^{-u^2}] / r^2,
u = r / 2 r_s, that the exp(-k^2 r_s^2) filter stands for.  The adjoint is pinned
to the forward by brute force: L = sum w . a is linear in the masses, and
quadratic in each coordinate inside a mesh cell, so unit masses and central
differences give its gradient to rounding."""
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


def test_mesh_derivative_is_fourth_order():
    # a smooth periodic potential with a known gradient: halving h cuts the error
    # of the mesh force by 2^4 (a second-order rule, a wrong weight or a sign slip
    # gives 4 or no convergence at all)
    def err(n):
        x = np.arange(n) / n
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        t = 2.0 * np.pi
        phi = np.sin(t * X) * np.cos(2 * t * Y) + 0.5 * np.sin(3 * t * Z)
        exact = -np.stack([t * np.cos(t * X) * np.cos(2 * t * Y),
                           -2 * t * np.sin(t * X) * np.sin(2 * t * Y),
                           1.5 * t * np.cos(3 * t * Z) * np.ones_like(X)])
        return np.abs(pm.mesh_force(phi, 1.0) - exact).max()
    e32, e64, e128 = err(32), err(64), err(128)
    assert 15.0 < e32 / e64 < 16.5 and 15.5 < e64 / e128 < 16.5


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
    # interpolation) leaves ~1.7%, once ~5%, not at all ~9%
    assert _pair_errors(128, 3).mean() <= 0.025


def _adjoint_case(seed=5, n=6, n_mesh=8, box=1.0):
    rng = np.random.default_rng(seed)
    h = box / n_mesh
    # cell fractions in [0.1, 0.9]: a small step never crosses a mesh plane;
    # whole-box shifts check the periodic wrap
    cells = rng.integers(0, n_mesh, (n, 3))
    pos = (cells + rng.uniform(0.1, 0.9, (n, 3))) * h + box * rng.integers(-1, 2, (n, 3))
    mass = rng.uniform(0.5, 2.0, n)
    w = rng.standard_normal((n, 3))
    return pos, mass, w, box, n_mesh, 1.25 * h


def _loss(pos, mass, w, box, n_mesh, r_s):
    return float((w * pm.pm_accel(pos, mass, box, n_mesh, r_s)).sum())


def test_adjoint_mass_gradient_is_the_response_to_unit_masses():
    pos, mass, w, box, n_mesh, r_s = _adjoint_case()
    _, dm = pm.pm_adjoint(pos, mass, box, n_mesh, r_s, w)
    brute = np.array([_loss(pos, np.eye(len(mass))[j], w, box, n_mesh, r_s) for j in range(len(mass))])
    assert np.abs(dm - brute).max() <= 1e-10 * np.abs(brute).max()


def test_adjoint_position_gradient_matches_central_differences():
    pos, mass, w, box, n_mesh, r_s = _adjoint_case()
    dx, _ = pm.pm_adjoint(pos, mass, box, n_mesh, r_s, w)
    step = 1e-6 * box / n_mesh
    fd = np.zeros_like(pos)
    for j in range(len(pos)):
        for e in range(3):
            p1, p0 = pos.copy(), pos.copy()
            p1[j, e] += step
            p0[j, e] -= step
            fd[j, e] = (_loss(p1, mass, w, box, n_mesh, r_s) - _loss(p0, mass, w, box, n_mesh, r_s)) / (2 * step)
    assert np.abs(dx - fd).max() <= 1e-6 * np.abs(fd).max()
    # both terms matter: the target term alone (particle j's own weights) misses
    # its pull on the others by far more than the tolerance
    force = pm.mesh_force(pm.potential_mesh(pos, mass, box, n_mesh, r_s), box)
    target_only = sum(w[:, d][:, None] * pm.cic_gradient_interpolate(force[d], pos, box) for d in range(3))
    assert np.abs(target_only - fd).max() > 1e-2 * np.abs(fd).max()
