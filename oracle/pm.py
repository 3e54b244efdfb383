"""FP64 CPU oracle for the long-range particle-mesh (PM) force.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code
with the HIP library and never imports it.

The steps follow sec. 3.1 (PM-Tree-PP method) in the paper's order, in
plain numpy, one step per function:

1. cloud-in-cell (CIC) assignment of the particle masses to a periodic
   mesh of n_mesh^3 points, spacing Delta = L / n_mesh (sec. 3.1 names CIC);
2. the Poisson equation (Eq. eq:poisson, nabla^2 phi = 4 pi G rho) solved in
   Fourier space with the 3-point difference Green function of sec. 3.1,
   g_k = pi G Delta^2 / (sin^2(pi l/N) + sin^2(pi m/N) + sin^2(pi n/N)),
   phi_k = -g_k rho_k, the k = 0 mode set to zero (periodic box);
3. the long-range part kept by the k-space Gaussian filter
   exp(-k^2 r_s^2), k^2 = (2 pi / L)^2 (l^2 + m^2 + n^2) with signed
   wave numbers: the complement of the short-range factor of Eq. equ:split
   (sec. 3.1 writes the filter in real space; the equation fixes it);
4. an inverse FFT to the mesh potential;
5. the mesh acceleration -grad phi by a 4-point central difference (the
   paper does not name the stencil; this is the Gadget-2 one it follows);
6. the acceleration of each particle interpolated linearly (CIC weights)
   from the mesh (sec. 3.1: "linearly interpolated").
"""
from __future__ import annotations

import numpy as np


def _cic_weights(pos: np.ndarray, L: float, n_mesh: int):
    """Mesh index of the lower corner and the linear weights per axis.
    Mesh point p sits at p * Delta; a particle at x shares its mass between
    floor(x / Delta) and the next point."""
    d = L / n_mesh
    w = np.mod(np.asarray(pos, dtype=np.float64), L) / d          # [3, n] in mesh units
    i0 = np.floor(w).astype(np.int64)
    f = w - i0                                                    # weight of the upper point
    i0 = np.mod(i0, n_mesh)
    return i0, f


def cic_deposit(pos: np.ndarray, mass: np.ndarray, L: float, n_mesh: int) -> np.ndarray:
    """Step 1: density rho (mass / Delta^3) on the mesh, [n_mesh]^3, x first."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    i0, f = _cic_weights(pos, L, n_mesh)
    rho = np.zeros((n_mesh, n_mesh, n_mesh))
    for cx in (0, 1):
        wx = f[0] if cx else 1.0 - f[0]
        ix = (i0[0] + cx) % n_mesh
        for cy in (0, 1):
            wy = f[1] if cy else 1.0 - f[1]
            iy = (i0[1] + cy) % n_mesh
            for cz in (0, 1):
                wz = f[2] if cz else 1.0 - f[2]
                iz = (i0[2] + cz) % n_mesh
                np.add.at(rho, (ix, iy, iz), mass * wx * wy * wz)
    return rho / (L / n_mesh) ** 3


def pm_potential(rho: np.ndarray, L: float, G: float, rs: float | None) -> np.ndarray:
    """Steps 2-4: the long-range potential on the mesh (rs=None: no filter,
    the whole mesh potential)."""
    n = rho.shape[0]
    d = L / n
    rk = np.fft.rfftn(rho)
    l = np.fft.fftfreq(n, 1.0 / n)                    # signed wave numbers
    lz = np.fft.rfftfreq(n, 1.0 / n)
    sx = np.sin(np.pi * l / n) ** 2
    sz = np.sin(np.pi * lz / n) ** 2
    S = sx[:, None, None] + sx[None, :, None] + sz[None, None, :]
    S[0, 0, 0] = 1.0
    gk = np.pi * G * d * d / S
    gk[0, 0, 0] = 0.0
    phik = -gk * rk
    if rs is not None:
        k2 = (2.0 * np.pi / L) ** 2 * (l[:, None, None] ** 2 + l[None, :, None] ** 2
                                        + lz[None, None, :] ** 2)
        phik = phik * np.exp(-k2 * rs * rs)
    return np.fft.irfftn(phik, s=rho.shape, axes=(0, 1, 2))


def mesh_accel(phi: np.ndarray, L: float) -> np.ndarray:
    """Step 5: -grad phi on the mesh by the 4-point central difference,
    [3][n_mesh]^3."""
    d = L / phi.shape[0]
    out = np.empty((3,) + phi.shape)
    for ax in range(3):
        p1 = np.roll(phi, -1, axis=ax)
        m1 = np.roll(phi, 1, axis=ax)
        p2 = np.roll(phi, -2, axis=ax)
        m2 = np.roll(phi, 2, axis=ax)
        out[ax] = -(8.0 * (p1 - m1) - (p2 - m2)) / (12.0 * d)
    return out


def cic_interp(mesh3: np.ndarray, pos: np.ndarray, L: float) -> np.ndarray:
    """Step 6: the mesh field at the particles with the CIC weights, [3][n]."""
    n_mesh = mesh3.shape[1]
    pos = np.asarray(pos, dtype=np.float64)
    i0, f = _cic_weights(pos, L, n_mesh)
    out = np.zeros((3, pos.shape[1]))
    for cx in (0, 1):
        wx = f[0] if cx else 1.0 - f[0]
        ix = (i0[0] + cx) % n_mesh
        for cy in (0, 1):
            wy = f[1] if cy else 1.0 - f[1]
            iy = (i0[1] + cy) % n_mesh
            for cz in (0, 1):
                wz = f[2] if cz else 1.0 - f[2]
                iz = (i0[2] + cz) % n_mesh
                w = wx * wy * wz
                for ax in range(3):
                    out[ax] += w * mesh3[ax][ix, iy, iz]
    return out


def pm_accel(pos: np.ndarray, mass: np.ndarray, params, n_mesh: int) -> np.ndarray:
    """Long-range acceleration of every particle, [3][n] FP64 (steps 1-6)."""
    rho = cic_deposit(pos, mass, params.L, n_mesh)
    phi = pm_potential(rho, params.L, params.G, params.rs)
    return cic_interp(mesh_accel(phi, params.L), pos, params.L)
