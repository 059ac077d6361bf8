"""FP64 CPU oracle for planar photoacoustic reconstruction.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call this package; the product
path never does. It shares no code with the GPU path: it evaluates the
discretised Fourier inversion formula directly, as a plain non-uniform DFT,
with no windows, no oversampling and no interpolation.

Definition followed (Section 2, eq. exact and eq. disc_rec, with the grids
of eq. eval_equi and the frequency interval G_Ky; physical units):

  lattice   Kx_j = 2*pi*j/X, Ky_k = 2*pi*k/Y, Kz_l = 2*pi*l/Z,
            j in [-Nx/2, Nx/2), k in [-Ny/2, Ny/2), l in [-Nz/2, Nz/2)
  |K|       = sqrt(Kx^2 + Ky^2 + Kz^2)
  omega(K)  = c * sign(Kz) * |K|        (kappa of eq. exact, in time units)
  W(K)      = 2*c*|Kz|/|K|              (2 K_y / kappa of eq. exact with the
                                         transform taken in t), W = 0 on l = 0
  stage L   G[j,k,n] = sum_m h_m*dt*g[m,n]*exp(-i(Kx_j x_m + Ky_k y_m))
            (eq. NUDFT2 with physical phases, the inner sum of eq. disc_rec)
  stage T   S[j,k,l] = sum_n G[j,k,n]*exp(-i*omega(K)*t_n), t_n = n*dt
            (eq. NUDFT1, the outer sum of eq. disc_rec)
  weight    F[j,k,l] = W(K)*S[j,k,l], zeroed on the planes j = -Nx/2,
            k = -Ny/2 and l = -Nz/2
  inverse   f[a,b,e] = 1/(X*Y*Z) * sum_K F(K) exp(+i(Kx x_a + Ky y_b + Kz z_e))
            with x_a = (a - Nx/2)X/Nx, y_b = (b - Ny/2)Y/Ny, z_e = e*Z/Nz
            (the equispaced inverse transform, step 3 of the NEDNER list in
            Section 3); the real part is taken.

Readings where the paper is garbled or silent (all also listed in the design
notes): physical wavenumbers instead of index units (the kappa of Section 2
assumes equal steps); W := 0 on the whole l = 0 plane (the 0/0 at l = 0);
the three Nyquist planes are zeroed so the spectrum is Hermitian and the
image exactly real; t_0 = 0 with a plain left Riemann sum; the time phase
enters only through kappa (the stray "+ l n" of eq. equiv_rec is dropped).
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

__all__ = [
    "lattice", "omega_and_weight", "stage_lateral", "stage_temporal", "apply_weight",
    "inverse", "reconstruct", "spectrum_at", "half_spectrum",
]


def _threads() -> int:
    """Worker threads of the temporal stage: ORACLE_THREADS if set (the
    benchmark's single-thread timing), else the CPU count up to 16."""
    env = os.environ.get("ORACLE_THREADS")
    if env:
        return max(1, int(env))
    return max(1, min(16, os.cpu_count() or 1))


def lattice(n: int, length: float) -> np.ndarray:
    """Wavenumbers 2*pi*j/length for j = -n/2 .. n/2-1, in that (natural) order."""
    j = np.arange(-(n // 2), n - n // 2)
    return 2.0 * np.pi * j / length


def omega_and_weight(kx, ky, kz, c):
    """omega(K) = c*sign(Kz)*|K| and W(K) = 2c|Kz|/|K| with W := 0 where Kz = 0
    (eq. exact rewritten for the time variable; see the module docstring)."""
    kx, ky, kz = np.broadcast_arrays(kx, ky, kz)
    kabs = np.sqrt(kx * kx + ky * ky + kz * kz)
    omega = c * np.sign(kz) * kabs
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(kz != 0.0, 2.0 * c * np.abs(kz) / np.where(kabs > 0, kabs, 1.0), 0.0)
    return omega, w


def stage_lateral(xy, h, g, dt, nx, ny, X, Y, j_index=None) -> np.ndarray:
    """Stage L: G[j,k,n] = sum_m h_m dt g[m,n] exp(-i(Kx_j x_m + Ky_k y_m)).

    The sum over m is a complex matrix product per j (a library GEMM).
    Returns complex128 [nx, ny, Nt] in natural index order (j = -nx/2 first);
    with `j_index` (natural-order positions) only those rows, in that order.
    """
    xy = np.asarray(xy, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    hw = np.asarray(h, dtype=np.float64) * dt
    kx = lattice(nx, X)
    ky = lattice(ny, Y)
    c_in = hw[:, None] * g                                   # [M, Nt]
    ey = np.exp(-1j * np.outer(ky, xy[:, 1]))                # [ny, M]
    rows = np.arange(nx) if j_index is None else np.asarray(j_index)
    out = np.empty((len(rows), ny, g.shape[1]), dtype=np.complex128)

    for i, j in enumerate(rows):
        ex = np.exp(-1j * kx[j] * xy[:, 0])                  # [M]
        a = ey * ex[None, :]                                 # [ny, M]
        out[i] = (np.ascontiguousarray(a.real) @ c_in) + 1j * (np.ascontiguousarray(a.imag) @ c_in)
    return out


def stage_temporal(G, kx, ky, kz, c, dt, l_index=None) -> np.ndarray:
    """Stage T: S[j,k,l] = sum_n G[j,k,n] exp(-i omega(K_jkl) t_n), t_n = n dt.

    G is [nx, ny, Nt]; kx, ky, kz are the lattice vectors (natural order).
    `l_index` selects a subset of kz entries (default: all). Direct evaluation
    of every exponential, parallel over j.
    """
    nx, ny, nt = G.shape
    kzs = kz if l_index is None else kz[np.asarray(l_index)]
    t = np.arange(nt) * dt
    S = np.empty((nx, ny, len(kzs)), dtype=np.complex128)

    ychunk = max(1, int(2**22 // max(1, len(kzs) * nt)))

    def one(j):
        for y0 in range(0, ny, ychunk):
            ys = slice(y0, min(ny, y0 + ychunk))
            om, _ = omega_and_weight(kx[j], ky[ys, None], kzs[None, :], c)   # [y, L]
            ph = om[:, :, None] * t[None, None, :]                          # [y, L, Nt]
            e = np.cos(ph) - 1j * np.sin(ph)
            S[j, ys] = np.matmul(e, G[j, ys, :, None])[..., 0]

    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(one, range(nx)))
    return S


def apply_weight(S, kx, ky, kz, c, j_index=None) -> np.ndarray:
    """F = W*S with W = 2c|Kz|/|K| (0 on Kz = 0), then zero the Nyquist planes
    j = -nx/2, k = -ny/2, l = -nz/2 (index 0 of each natural-order axis).
    With `j_index`, S holds only those natural-order x rows of the lattice."""
    rows = np.arange(len(kx)) if j_index is None else np.asarray(j_index)
    _, w = omega_and_weight(kx[rows][:, None, None], ky[None, :, None], kz[None, None, :], c)
    F = w * S
    F[rows == 0, :, :] = 0.0
    F[:, 0, :] = 0.0
    F[:, :, 0] = 0.0
    return F


def inverse(F, X, Y, Z, return_complex=False):
    """f[a,b,e] = 1/(XYZ) sum_K F(K) exp(i(Kx x_a + Ky y_b + Kz z_e)).

    With x_a = (a - nx/2)dx the lateral phase is (-1)^j exp(2 pi i j a/nx);
    z_e = e dz gives exp(2 pi i l e/nz). numpy's ifftn (a library routine)
    evaluates the sums after the natural-order axes are shifted to FFT order.
    """
    nx, ny, nz = F.shape
    j = np.arange(-(nx // 2), nx - nx // 2)
    k = np.arange(-(ny // 2), ny - ny // 2)
    sign = ((-1.0) ** j)[:, None, None] * ((-1.0) ** k)[None, :, None]
    A = np.fft.ifftshift(F * sign, axes=(0, 1, 2))
    fc = np.fft.ifftn(A) * (nx * ny * nz) / (X * Y * Z)
    return fc if return_complex else fc.real


def reconstruct(xy, h, g, dt, c, shape, extent, return_stages=False):
    """Full reconstruction f from traces g (definition in the module docstring).

    shape = (Nx, Ny, Nz), extent = (X, Y, Z). Returns f [Nx, Ny, Nz] float64,
    or (f, stages) with stages = dict(G=..., S=..., F=..., fc=complex image).
    """
    nx, ny, nz = shape
    X, Y, Z = extent
    kx, ky, kz = lattice(nx, X), lattice(ny, Y), lattice(nz, Z)
    G = stage_lateral(xy, h, g, dt, nx, ny, X, Y)
    S = stage_temporal(G, kx, ky, kz, c, dt)
    F = apply_weight(S, kx, ky, kz, c)
    fc = inverse(F, X, Y, Z, return_complex=True)
    if return_stages:
        return fc.real, dict(G=G, S=S, F=F, fc=fc)
    return fc.real


def half_spectrum(F) -> np.ndarray:
    """Re-index a natural-order spectrum F[j,k,l] to the GPU output layout
    [j mod Nx, k mod Ny, l] for l = 0..Nz/2 (FFT order laterally, the
    non-negative half along z). Pure re-indexing."""
    nx, ny, nz = F.shape
    A = np.fft.ifftshift(F, axes=(0, 1))
    lz = np.arange(0, nz // 2 + 1)
    return A[:, :, (lz + nz // 2) % nz]


def spectrum_at(xy, h, g, dt, c, shape, extent, jkl) -> np.ndarray:
    """F(K) at selected lattice points, each summed directly over m and n.

    jkl: int array [P,3] of signed indices (j, k, l). Returns complex128 [P].
    Cost P*M*Nt; used to check large problems at sampled wavenumbers.
    """
    nx, ny, nz = shape
    X, Y, Z = extent
    jkl = np.asarray(jkl, dtype=np.int64).reshape(-1, 3)
    xy = np.asarray(xy, dtype=np.float64)
    c_in = (np.asarray(h, dtype=np.float64) * dt)[:, None] * np.asarray(g, dtype=np.float64)
    t = np.arange(c_in.shape[1]) * dt
    kx = 2 * np.pi * jkl[:, 0] / X
    ky = 2 * np.pi * jkl[:, 1] / Y
    kz = 2 * np.pi * jkl[:, 2] / Z
    om, w = omega_and_weight(kx, ky, kz, c)
    out = np.empty(len(jkl), dtype=np.complex128)
    step = 64
    for s in range(0, len(jkl), step):
        sl = slice(s, s + step)
        lat = np.exp(-1j * (np.outer(kx[sl], xy[:, 0]) + np.outer(ky[sl], xy[:, 1])))  # [p, M]
        Gs = (np.ascontiguousarray(lat.real) @ c_in) + 1j * (np.ascontiguousarray(lat.imag) @ c_in)  # [p, Nt]
        et = np.exp(-1j * np.outer(om[sl], t))                                          # [p, Nt]
        out[sl] = w[sl] * np.sum(Gs * et, axis=1)
    nyq = (jkl[:, 0] == -(nx // 2)) | (jkl[:, 1] == -(ny // 2)) | (jkl[:, 2] == -(nz // 2))
    out[nyq] = 0.0
    return out
