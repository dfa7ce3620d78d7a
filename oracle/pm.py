"""FP64 oracle of the particle-mesh (PM) long-range force of the TreePM split.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to produce expected values.
It imports nothing from the GPU package and the GPU package never imports it.

The paper computes the long-range half of the TreePM force on the CPU with
FFTW (Sec. 3.1) and defines no scheme of its own; this follows Gadget-2's
periodic PM (Springel 2005, its TreePM section), written out plainly:

1. periodic cloud-in-cell (CIC) assignment of the masses to an N^3 mesh whose
   points sit at (i, j, k) L / N, giving the density rho = mass per cell / h^3;
2. rho_hat = DFT(rho);
3. phi_hat(k) = -4 pi G rho_hat(k) exp(-k^2 r_s^2) / k^2, phi_hat(0) = 0, divided
   by the CIC window twice (assignment and interpolation): prod_d sinc(pi n_d / N)^4
   with n_d the signed integer wavenumber and sinc(x) = sin(x) / x;
4. phi = inverse DFT (normalised by 1/N^3) on the mesh;
5. the force field F = -grad phi on the mesh by the fourth-order central
   difference along each axis:
   F_d(i) = [8 (phi(i - e_d) - phi(i + e_d)) - (phi(i - 2 e_d) - phi(i + 2 e_d))] / (12 h);
6. CIC interpolation of F_d back to the particles with the assignment weights.

The exp(-k^2 r_s^2) filter is the Fourier transform of the long-range part
G m erf(r / 2 r_s) / r of the potential, the complement of the short-range
erfc(r / 2 r_s) / r that the tree walk applies.
"""
from __future__ import annotations

import numpy as np


def wrap_unit(pos: np.ndarray, box: float) -> np.ndarray:
    """u = x / L - floor(x / L) in [0, 1); a rounding to 1 maps to 0."""
    u = pos / box
    u = u - np.floor(u)
    u[u >= 1.0] = 0.0
    return u


def cic_weights(pos: np.ndarray, box: float, n_mesh: int):
    """Per particle and axis: the lower mesh index and the weight of the upper one."""
    s = wrap_unit(np.asarray(pos, dtype=np.float64), box) * n_mesh
    i0 = np.floor(s).astype(np.int64)
    f = s - i0
    i0 %= n_mesh
    return i0, f


def cic_assign(pos: np.ndarray, mass: np.ndarray, box: float, n_mesh: int) -> np.ndarray:
    """Density on the mesh: each particle's mass spread over the 8 surrounding mesh
    points with weights prod_d (1 - f_d or f_d), divided by the cell volume."""
    i0, f = cic_weights(pos, box, n_mesh)
    rho = np.zeros((n_mesh, n_mesh, n_mesh))
    h3 = (box / n_mesh) ** 3
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = (i0[:, 0] + cx) % n_mesh
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + cy) % n_mesh
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + cz) % n_mesh
                np.add.at(rho, (ix, iy, iz), mass * (wx * wy * wz) / h3)
    return rho


def cic_interpolate(field: np.ndarray, pos: np.ndarray, box: float) -> np.ndarray:
    """Value of a mesh field at the particles with the assignment weights."""
    n_mesh = field.shape[0]
    i0, f = cic_weights(pos, box, n_mesh)
    out = np.zeros(len(i0))
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = (i0[:, 0] + cx) % n_mesh
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + cy) % n_mesh
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + cz) % n_mesh
                out += (wx * wy * wz) * field[ix, iy, iz]
    return out


def wavenumbers(n_mesh: int):
    """Signed integer wavenumbers of the full axes and of the halved last axis."""
    n = np.arange(n_mesh)
    full = np.where(n <= n_mesh // 2, n, n - n_mesh)
    half = np.arange(n_mesh // 2 + 1)
    return full, half


def potential_spectrum(rho_hat: np.ndarray, box: float, r_s: float, G: float) -> np.ndarray:
    """phi_hat = -4 pi G rho_hat exp(-k^2 r_s^2) / k^2 / W_CIC(k)^2, phi_hat(0) = 0."""
    n_mesh = rho_hat.shape[0]
    full, half = wavenumbers(n_mesh)
    nx, ny, nz = np.meshgrid(full, full, half, indexing="ij")
    two_pi_l = 2.0 * np.pi / box
    k2 = (two_pi_l * nx) ** 2 + (two_pi_l * ny) ** 2 + (two_pi_l * nz) ** 2

    def sinc(n):
        x = np.pi * n / n_mesh
        return np.where(n == 0, 1.0, np.sin(x) / np.where(n == 0, 1.0, x))

    w = sinc(nx) * sinc(ny) * sinc(nz)          # one CIC window is w^2
    with np.errstate(divide="ignore", invalid="ignore"):
        green = -4.0 * np.pi * G * np.exp(-k2 * r_s * r_s) / k2 / (w ** 4)
    green[0, 0, 0] = 0.0
    return rho_hat * green


def potential_mesh(pos: np.ndarray, mass: np.ndarray, box: float, n_mesh: int, r_s: float,
                   G: float = 1.0) -> np.ndarray:
    """The long-range potential phi on the mesh (steps 1-4)."""
    rho = cic_assign(pos, mass, box, n_mesh)
    phi_hat = potential_spectrum(np.fft.rfftn(rho), box, r_s, G)
    return np.fft.irfftn(phi_hat, s=(n_mesh, n_mesh, n_mesh), axes=(0, 1, 2))


def mesh_force(phi: np.ndarray, box: float) -> np.ndarray:
    """-grad phi (3, N, N, N) by the periodic fourth-order central difference (step 5).
    np.roll(phi, s, axis=d)[i] is phi(i - s e_d)."""
    h = box / phi.shape[0]
    out = np.empty((3,) + phi.shape)
    for d in range(3):
        out[d] = (8.0 * (np.roll(phi, 1, d) - np.roll(phi, -1, d))
                  - (np.roll(phi, 2, d) - np.roll(phi, -2, d))) / (12.0 * h)
    return out


def pm_accel(pos: np.ndarray, mass: np.ndarray, box: float, n_mesh: int, r_s: float,
             G: float = 1.0) -> np.ndarray:
    """Long-range (PM) accelerations (N, 3) of all particles, in input order."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    force = mesh_force(potential_mesh(pos, mass, box, n_mesh, r_s, G), box)
    acc = np.zeros((len(pos), 3))
    for d in range(3):
        acc[:, d] = cic_interpolate(force[d], pos, box)
    return acc


def cic_gradient_interpolate(field: np.ndarray, pos: np.ndarray, box: float) -> np.ndarray:
    """(N, 3): d/dx_e of the interpolated field value at each particle with the mesh
    field held fixed.  The weight of axis e is 1 - f_e or f_e with df_e/dx_e = N / L,
    so its derivative is -N / L or +N / L (the derivative inside a cell)."""
    n_mesh = field.shape[0]
    i0, f = cic_weights(pos, box, n_mesh)
    inv_h = n_mesh / box
    out = np.zeros((len(i0), 3))
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        dx = inv_h if cx else -inv_h
        ix = (i0[:, 0] + cx) % n_mesh
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            dy = inv_h if cy else -inv_h
            iy = (i0[:, 1] + cy) % n_mesh
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                dz = inv_h if cz else -inv_h
                iz = (i0[:, 2] + cz) % n_mesh
                v = field[ix, iy, iz]
                out[:, 0] += dx * wy * wz * v
                out[:, 1] += wx * dy * wz * v
                out[:, 2] += wx * wy * dz * v
    return out


def pm_adjoint(pos: np.ndarray, mass: np.ndarray, box: float, n_mesh: int, r_s: float, w: np.ndarray,
               G: float = 1.0):
    """Gradient of L = sum_i w_i . a_i (a the PM accelerations) with respect to the
    positions (N, 3) and the masses (N,), taking the forward steps in reverse:

    With W_i(c) the CIC weight of particle i at mesh point c, rho = sum_j m_j W_j / h^3,
    phi = K rho (K the filtered Green's convolution of steps 2-4, a symmetric
    operator), F_d = D_d phi (D_d the difference rule of step 5, an odd operator:
    its transpose is -D_d) and a_i,d = sum_c W_i(c) F_d(c):

      omega_d(c) = sum_i w_i,d W_i(c)                    (the weights assigned to the mesh)
      psi        = K^T sum_d D_d^T omega_d = -K sum_d D_d omega_d
      dL/dm_j    = sum_c W_j(c) psi(c) / h^3
      dL/dx_j    = sum_d w_j,d sum_c grad W_j(c) F_d(c) + m_j / h^3 sum_c grad W_j(c) psi(c)

    The second term of dL/dx_j is particle j as a source, the first as a target.
    The CIC weights are piecewise linear, so this is the derivative inside the mesh
    cells (a position exactly on a mesh plane takes the one-sided value of the
    cell that holds it)."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    h3 = (box / n_mesh) ** 3
    force = mesh_force(potential_mesh(pos, mass, box, n_mesh, r_s, G), box)
    chi = np.zeros((n_mesh, n_mesh, n_mesh))
    for d in range(3):
        omega = cic_assign(pos, w[:, d], box, n_mesh) * h3          # without the 1/h^3 of a density
        chi -= mesh_force(omega, box)[d]
    psi = np.fft.irfftn(potential_spectrum(np.fft.rfftn(chi), box, r_s, G),
                        s=(n_mesh, n_mesh, n_mesh), axes=(0, 1, 2))
    dmass = cic_interpolate(psi, pos, box) / h3
    dpos = mass[:, None] * cic_gradient_interpolate(psi, pos, box) / h3
    for d in range(3):
        dpos += w[:, d][:, None] * cic_gradient_interpolate(force[d], pos, box)
    return dpos, dmass


def pm_accel_torch(x, mass, box: float, n_mesh: int, r_s: float, G: float = 1.0):
    """The same PM accelerations in PyTorch FP64 (CPU), differentiable in x and mass
    by autograd: an independent route to the gradient that pm_adjoint composes by
    hand.  Inside a mesh cell the CIC weights are linear in x, and the cell index is
    held fixed (floor carries no gradient)."""
    import torch
    x = torch.as_tensor(x, dtype=torch.float64)
    mass = torch.as_tensor(mass, dtype=torch.float64)
    n = n_mesh
    h = box / n
    u = x / box
    u = u - torch.floor(u).detach()
    s = u * n
    lo = torch.floor(s).detach()
    f = s - lo
    i0 = lo.long() % n
    green = torch.as_tensor(potential_spectrum(np.ones((n, n, n // 2 + 1), dtype=np.complex128), box, r_s, G))
    corners = []
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                wgt = ((f[:, 0] if cx else 1 - f[:, 0]) * (f[:, 1] if cy else 1 - f[:, 1])
                       * (f[:, 2] if cz else 1 - f[:, 2]))
                flat = (((i0[:, 0] + cx) % n) * n + (i0[:, 1] + cy) % n) * n + (i0[:, 2] + cz) % n
                corners.append((wgt, flat))
    rho = torch.zeros(n ** 3, dtype=torch.float64)
    for wgt, flat in corners:
        rho = rho.index_add(0, flat, mass * wgt / h ** 3)
    phi = torch.fft.irfftn(torch.fft.rfftn(rho.view(n, n, n)) * green, s=(n, n, n), dim=(0, 1, 2))
    acc = []
    for d in range(3):
        F = (8.0 * (torch.roll(phi, 1, d) - torch.roll(phi, -1, d))
             - (torch.roll(phi, 2, d) - torch.roll(phi, -2, d))) / (12.0 * h)
        Ff = F.reshape(-1)
        acc.append(sum(wgt * Ff[flat] for wgt, flat in corners))
    return torch.stack(acc, dim=1)


def long_range_pair(d: np.ndarray, m: float, r_s: float, G: float = 1.0) -> np.ndarray:
    """Acceleration of a test particle at separation vector d (N, 3) from a point mass m
    under the long-range part of the split alone, in infinite space (no images):
    a = -G m d / r^3 [erf(u) - 2u/sqrt(pi) exp(-u^2)], u = r / 2 r_s, pointing to the mass."""
    from math import erf, exp, pi, sqrt
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    out = np.zeros_like(d)
    for i, v in enumerate(d):
        r = float(np.linalg.norm(v))
        u = r / (2.0 * r_s)
        f = erf(u) - 2.0 * u / sqrt(pi) * exp(-u * u)
        out[i] = -G * m * v / r ** 3 * f
    return out
