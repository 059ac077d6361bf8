"""FP64 CPU oracle of the forward model and its adjoint.

TEST INFRASTRUCTURE ONLY (as the rest of this package): only tests, the
smoke check and the benchmark's CPU leg may call it; the product path never
does, and nothing here is shared with the GPU path.

The forward model is the free-space wave equation of Section 2 (the initial
value problem whose solution at the sensor plane the reconstruction of
eq. exact inverts) written on the same Fourier lattice as the
reconstruction: an image f on the grid x_a = (a - Nx/2)X/Nx,
y_b = (b - Ny/2)Y/Ny, z_e = e Z/Nz has the Fourier coefficients

  D(K) = dV * sum_r f(r) exp(-i K.r),   dV = (X/Nx)(Y/Ny)(Z/Nz),

and the pressure it launches (zero initial velocity) is the standing-wave
sum p(r, t) = 1/V sum_K D(K) exp(i K.r) cos(c|K| t), V = XYZ. Sampling it
at the sensors (z = 0) at t_n = n dt gives

  (A f)[m, n] = 1/V sum_K D(K) exp(i(Kx x_m + Ky y_m)) cos(c|K| t_n),

with K over the lattice of the reconstruction minus the three Nyquist
planes (j = -Nx/2, k = -Ny/2, l = -Nz/2), so that the sum is real.

The adjoint for the Euclidean inner products sum_{m,n} g g' and
sum_r f f' (no quadrature weights on either side) is

  (A* g)(r) = 1/V sum_K F*(K) exp(i K.r),
  F*(K)     = dV sum_n cos(c|K| t_n) sum_m g[m,n] exp(-i(Kx x_m + Ky y_m)),

i.e. the reconstruction's stages with unit data weights, the weight W
replaced by the constant dV and exp(-i omega t) replaced by cos(c|K| t)
(the average of the two signs of Kz), including the l = 0 plane.

The derivative of each trace with respect to its own sensor position,
d(A f)[m, n]/dx_m, is the same sum with i*Kx in front of each term (i*Ky
for y_m).

Readings (also listed in the design notes): Euclidean inner products; the
lattice and its Nyquist planes as in the reconstruction; depth periodic
with period Z, so a source at depth z also arrives from z - Z (callers pad
the depth so that these arrivals fall after the last sample).
"""
from __future__ import annotations

import numpy as np

from .reference import inverse, lattice, stage_lateral

__all__ = ["image_spectrum", "forward", "adjoint", "power_norm_sq", "landweber"]


def _nyquist_zero(F):
    """Zero the planes j = -Nx/2, k = -Ny/2, l = -Nz/2 (index 0 of each
    natural-order axis)."""
    F = F.copy()
    F[0, :, :] = 0.0
    F[:, 0, :] = 0.0
    F[:, :, 0] = 0.0
    return F


def image_spectrum(f, extent):
    """D(K) = dV sum_r f(r) exp(-i K.r) in natural order, Nyquist planes zero.

    With x_a = (a - Nx/2)dx the x phase is exp(-2 pi i j a/Nx) (-1)^j (and
    likewise in y); z_e = e dz has no offset. numpy's fftn (a library DFT)
    evaluates the sums in FFT order; fftshift puts j = -Nx/2 first.
    """
    f = np.asarray(f, dtype=np.float64)
    nx, ny, nz = f.shape
    X, Y, Z = extent
    dV = (X / nx) * (Y / ny) * (Z / nz)
    j = np.arange(-(nx // 2), nx - nx // 2)
    k = np.arange(-(ny // 2), ny - ny // 2)
    sign = ((-1.0) ** j)[:, None, None] * ((-1.0) ** k)[None, :, None]
    D = np.fft.fftshift(np.fft.fftn(f), axes=(0, 1, 2)) * sign * dV
    return _nyquist_zero(D)


def forward(f, xy, nt, dt, c, extent, deriv=None, n_index=None):
    """(A f)[m, n] (module docstring); deriv = "x" or "y" gives the
    derivative of each trace with respect to its sensor's x or y. With
    n_index only the samples t_n = n dt for those n, as columns in that
    order (each output is its own sum, so a sample of them equals the same
    entries of the full result).

    Per lateral mode column: P[k, n] = sum_l D[j,k,l] cos(c|K| t_n); then the
    sensor sum exp(i Kx x_m) sum_k exp(i Ky y_m) P[k, n] as matrix products.
    """
    f = np.asarray(f, dtype=np.float64)
    xy = np.asarray(xy, dtype=np.float64)
    nx, ny, nz = f.shape
    X, Y, Z = extent
    V = X * Y * Z
    D = image_spectrum(f, extent)
    kx, ky, kz = lattice(nx, X), lattice(ny, Y), lattice(nz, Z)
    t = (np.arange(nt) if n_index is None else np.asarray(n_index)) * dt
    ey = np.exp(1j * np.outer(xy[:, 1], ky))                 # [M, ny]
    if deriv == "y":
        ey = ey * (1j * ky)[None, :]
    g = np.zeros((xy.shape[0], len(t)))
    for j in range(nx):
        kabs = np.sqrt(kx[j] ** 2 + ky[:, None] ** 2 + kz[None, :] ** 2)      # [ny, nz]
        cosk = np.cos(c * kabs[:, :, None] * t[None, None, :])                # [ny, nz, nt]
        P = np.einsum("kl,kln->kn", D[j], cosk)                               # [ny, nt]
        ex = np.exp(1j * kx[j] * xy[:, 0])                                    # [M]
        if deriv == "x":
            ex = ex * (1j * kx[j])
        g += (ex[:, None] * (ey @ P)).real
    return g / V


def adjoint(g, xy, dt, c, shape, extent):
    """(A* g)(r) on the output grid (module docstring)."""
    g = np.asarray(g, dtype=np.float64)
    nx, ny, nz = shape
    X, Y, Z = extent
    dV = (X / nx) * (Y / ny) * (Z / nz)
    nt = g.shape[1]
    # sum_m g[m,n] exp(-i(Kx x_m + Ky y_m)): stage L with unit weights
    G0 = stage_lateral(xy, np.ones(len(g)), g, 1.0, nx, ny, X, Y)          # [nx, ny, nt]
    kx, ky, kz = lattice(nx, X), lattice(ny, Y), lattice(nz, Z)
    t = np.arange(nt) * dt
    F = np.empty((nx, ny, nz), dtype=np.complex128)
    for j in range(nx):
        kabs = np.sqrt(kx[j] ** 2 + ky[:, None] ** 2 + kz[None, :] ** 2)      # [ny, nz]
        cosk = np.cos(c * kabs[:, :, None] * t[None, None, :])                # [ny, nz, nt]
        F[j] = dV * np.einsum("kn,kln->kl", G0[j], cosk)
    return inverse(_nyquist_zero(F), X, Y, Z)


def power_norm_sq(apply_normal, x0, iters):
    """Power iteration for the largest eigenvalue of the normal operator
    A*A (= ||A||^2), from the start vector x0: x <- A*A x / ||A*A x||; the
    estimate is the Rayleigh quotient <x, A*A x> of the last iterate."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = apply_normal(x)
        lam = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
    return lam


def landweber(g, xy, dt, c, shape, extent, iters, tau):
    """Landweber iteration f_{k+1} = f_k + tau A*(g - A f_k) from f_0 = 0.
    Returns the iterates' residual norms ||g - A f_k|| (k = 0..iters) and the
    last iterate."""
    nt = g.shape[1]
    f = np.zeros(shape)
    res = []
    for _ in range(iters):
        r = g - forward(f, xy, nt, dt, c, extent)
        res.append(float(np.linalg.norm(r)))
        f = f + tau * adjoint(r, xy, dt, c, shape, extent)
    res.append(float(np.linalg.norm(g - forward(f, xy, nt, dt, c, extent))))
    return f, res
