"""Image-quality measures of Appendix B (test infrastructure only).

Correlation coefficient (Appendix B, eq. corrcoeff), Tenenbaum sharpness with
the Sobel operator normalised by the element count (Appendix B), maximum
intensity projections, and the relative L2 distance used for parity.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
leg use this module. Pinned in tests/test_oracle_quality_pins.py (numpy's
correlation routine and exact affine and orthogonal cases; closed-form Sobel
responses of linear ramps and of an impulse; a one-hot volume).
"""
from __future__ import annotations

import numpy as np


def corrcoef(u1, u2) -> float:
    """rho = Cov(U1, U2) / sqrt(Var(U1) Var(U2)) over all elements."""
    a = np.asarray(u1, dtype=np.float64).ravel()
    b = np.asarray(u2, dtype=np.float64).ravel()
    a = a - a.mean()
    b = b - b.mean()
    return float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))


_SOBEL = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]])


def _conv2_valid(u, k):
    """2-D correlation of a 2-D array with a 3x3 kernel on interior points."""
    n0, n1 = u.shape
    out = np.zeros((n0 - 2, n1 - 2))
    for a in range(3):
        for b in range(3):
            out += k[a, b] * u[a:a + n0 - 2, b:b + n1 - 2]
    return out


def tenenbaum(u) -> float:
    """Normalised Tenenbaum sharpness: sum of (g*U)^2 + (g^T*U)^2 with the
    Sobel g, divided by the number of elements of U. For a 3-D volume the
    2-D operator is applied to every slice along the last axis."""
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 2:
        slices = [u]
    else:
        slices = [u[..., i] for i in range(u.shape[-1])]
    total = 0.0
    for s in slices:
        gx = _conv2_valid(s, _SOBEL)
        gy = _conv2_valid(s, _SOBEL.T)
        total += float(np.sum(gx * gx + gy * gy))
    return total / u.size


def mips(u):
    """Maximum intensity projections along x, y and z."""
    u = np.asarray(u)
    return u.max(axis=0), u.max(axis=1), u.max(axis=2)


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2."""
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def cylinder_roi(shape, extent, centre, diameter, height_ratio=8.0 / 9.0):
    """Voxels inside the region of interest of Section 6.3: a cylinder with
    its axis along z, the given diameter and height = height_ratio *
    diameter (8:9), centred at centre = (x, y, z) metres. Voxel centres are
    x_a = (a - Nx/2)X/Nx, y_b = (b - Ny/2)Y/Ny, z_e = e Z/Nz."""
    nx, ny, nz = shape
    X, Y, Z = extent
    x = (np.arange(nx) - nx // 2) * (X / nx)
    y = (np.arange(ny) - ny // 2) * (Y / ny)
    z = np.arange(nz) * (Z / nz)
    rad2 = (x[:, None, None] - centre[0]) ** 2 + (y[None, :, None] - centre[1]) ** 2
    half = 0.5 * height_ratio * diameter
    return (rad2 <= (0.5 * diameter) ** 2) & (np.abs(z[None, None, :] - centre[2]) <= half)


def roi_box(mask):
    """Index slices of the bounding box of a boolean mask."""
    idx = np.nonzero(mask)
    return tuple(slice(int(i.min()), int(i.max()) + 1) for i in idx)
