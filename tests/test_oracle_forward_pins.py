"""Pins of the oracle's forward model A, its adjoint A* and the Landweber
helpers against facts fixed by the wave equation and by linear algebra,
not by the oracle's own formulas:

* a lattice plane wave cos(K0.r + phi) launches the standing wave
  cos(K0.r + phi) cos(c|K0| t) (the Fourier-mode solution of the wave
  equation with zero initial velocity), exact at any sensor position;
* its derivative in x_m is -K0x sin(...) cos(c|K0| t) (and likewise in y);
* <A f, g> = <f, A* g> for random f, g (definition of the adjoint);
* A* equals a brute-force quadruple sum over voxels, lattice points,
  sensors and samples on a tiny problem (no separation of the sums);
* central differences of A f in the sensor positions match the derivative;
* power iteration converges to the largest squared singular value of the
  dense matrix of A, and Landweber residuals never increase for
  tau <= 1/||A||^2.
"""
import numpy as np
import pytest

from oracle import forward_model as fm

C = 1500.0


def _grid(shape, extent):
    nx, ny, nz = shape
    X, Y, Z = extent
    x = (np.arange(nx) - nx / 2) * X / nx
    y = (np.arange(ny) - ny / 2) * Y / ny
    z = np.arange(nz) * Z / nz
    return x, y, z


def _sensors(rng, m, extent):
    X, Y, _ = extent
    return np.stack([rng.uniform(-X / 2, X / 2, m), rng.uniform(-Y / 2, Y / 2, m)], axis=1)


SHAPE = (8, 10, 12)
EXT = (4e-3, 5e-3, 6e-3)
DT = 40e-9
NT = 50


@pytest.mark.parametrize("mode", [(3, -2, 5, 0.7), (1, 0, 0, 0.3), (-3, 4, -5, -1.1), (0, 0, 2, 0.0),
                                  (2, 1, 0, 1.9)])
def test_plane_wave_standing_wave(mode):
    j0, k0, l0, phi = mode
    rng = np.random.default_rng(11)
    xy = _sensors(rng, 13, EXT)
    kx, ky, kz = (2 * np.pi * j0 / EXT[0], 2 * np.pi * k0 / EXT[1], 2 * np.pi * l0 / EXT[2])
    x, y, z = _grid(SHAPE, EXT)
    f = np.cos(kx * x[:, None, None] + ky * y[None, :, None] + kz * z[None, None, :] + phi)
    g = fm.forward(f, xy, NT, DT, C, EXT)
    t = np.arange(NT) * DT
    kabs = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    ref = np.cos(kx * xy[:, 0] + ky * xy[:, 1] + phi)[:, None] * np.cos(C * kabs * t)[None, :]
    assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    for axis, kk in (("x", kx), ("y", ky)):
        gd = fm.forward(f, xy, NT, DT, C, EXT, deriv=axis)
        refd = -kk * np.sin(kx * xy[:, 0] + ky * xy[:, 1] + phi)[:, None] * np.cos(C * kabs * t)[None, :]
        scale = max(1.0, abs(kk))
        assert np.abs(gd - refd).max() <= 1e-12 * scale


def test_adjointness():
    rng = np.random.default_rng(12)
    xy = _sensors(rng, 17, EXT)
    f = rng.standard_normal(SHAPE)
    g = rng.standard_normal((17, NT))
    Af = fm.forward(f, xy, NT, DT, C, EXT)
    Asg = fm.adjoint(g, xy, DT, C, SHAPE, EXT)
    lhs, rhs = np.vdot(Af, g), np.vdot(f, Asg)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Af) * np.linalg.norm(g)


def test_adjoint_brute_force():
    """(A* g)(r) = dV/V sum_K sum_{m,n} g[m,n] cos(c|K| t_n) cos(K.(r - x_m)),
    summed with explicit loops over the lattice (Nyquist planes left out)."""
    rng = np.random.default_rng(13)
    shape, ext = (4, 4, 6), (2e-3, 3e-3, 2.5e-3)
    m, nt, dt = 5, 6, 50e-9
    xy = _sensors(rng, m, ext)
    g = rng.standard_normal((m, nt))
    got = fm.adjoint(g, xy, dt, C, shape, ext)
    nx, ny, nz = shape
    X, Y, Z = ext
    x, y, z = _grid(shape, ext)
    t = np.arange(nt) * dt
    dV_over_V = 1.0 / (nx * ny * nz)
    ref = np.zeros(shape)
    for j in range(-(nx // 2) + 1, nx // 2):
        for k in range(-(ny // 2) + 1, ny // 2):
            for l in range(-(nz // 2) + 1, nz // 2):
                Kx, Ky, Kz = 2 * np.pi * j / X, 2 * np.pi * k / Y, 2 * np.pi * l / Z
                kabs = np.sqrt(Kx * Kx + Ky * Ky + Kz * Kz)
                for mm in range(m):
                    amp = np.sum(g[mm] * np.cos(C * kabs * t))
                    ph = (Kx * (x[:, None, None] - xy[mm, 0]) + Ky * (y[None, :, None] - xy[mm, 1])
                          + Kz * z[None, None, :])
                    ref += dV_over_V * amp * np.cos(ph)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_position_derivative_central_differences():
    rng = np.random.default_rng(14)
    xy = _sensors(rng, 6, EXT) * 0.9
    f = rng.standard_normal(SHAPE)
    h = 1e-7 * EXT[0]
    for axis, col in (("x", 0), ("y", 1)):
        d = fm.forward(f, xy, NT, DT, C, EXT, deriv=axis)
        xp, xm = xy.copy(), xy.copy()
        xp[:, col] += h
        xm[:, col] -= h
        fd = (fm.forward(f, xp, NT, DT, C, EXT) - fm.forward(f, xm, NT, DT, C, EXT)) / (2 * h)
        assert np.linalg.norm(fd - d) <= 1e-6 * np.linalg.norm(d)


def _dense(shape, ext, xy, nt, dt):
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(fm.forward(e.reshape(shape), xy, nt, dt, C, ext).ravel())
    return np.stack(cols, axis=1)


def test_power_iteration_and_landweber():
    rng = np.random.default_rng(15)
    shape, ext = (4, 4, 6), (2e-3, 2e-3, 3e-3)
    m, nt, dt = 9, 24, 40e-9
    xy = _sensors(rng, m, ext)
    A = _dense(shape, ext, xy, nt, dt)
    smax2 = np.linalg.svd(A, compute_uv=False)[0] ** 2

    def normal(v):
        return fm.adjoint(fm.forward(v.reshape(shape), xy, nt, dt, C, ext), xy, dt, C, shape, ext).ravel()

    x0 = rng.standard_normal(int(np.prod(shape)))
    lam20 = fm.power_norm_sq(normal, x0, 20)
    lam300 = fm.power_norm_sq(normal, x0, 300)
    assert 0.5 * smax2 <= lam20 <= smax2 * (1 + 1e-12)
    assert abs(lam300 - smax2) <= 1e-6 * smax2
    g = A @ rng.standard_normal(A.shape[1]) + 0.1 * rng.standard_normal(A.shape[0])
    g = g.reshape(m, nt)
    f, res = fm.landweber(g, xy, dt, C, shape, ext, 10, 1.0 / smax2)
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))
    assert res[-1] < res[0]
    # the iterate is the truncated Neumann series tau sum_k (I - tau A*A)^k A* g
    N = np.eye(A.shape[1]) - A.T @ A / smax2
    acc = np.zeros(A.shape[1])
    term = A.T @ g.ravel() / smax2
    for _ in range(10):
        acc += term
        term = N @ term
    assert np.abs(f.ravel() - acc).max() <= 1e-10 * np.abs(acc).max()


def test_sampled_times_equal_full_columns():
    """forward(..., n_index=...) returns exactly the selected columns of the
    full result (each output is its own sum), with and without the position
    derivative."""
    rng = np.random.default_rng(19)
    xy = _sensors(rng, 7, EXT)
    f = rng.standard_normal(SHAPE)
    idx = np.array([0, 3, 17, 49, 22])
    for deriv in (None, "x", "y"):
        full = fm.forward(f, xy, NT, DT, C, EXT, deriv=deriv)
        part = fm.forward(f, xy, NT, DT, C, EXT, deriv=deriv, n_index=idx)
        assert part.shape == (7, len(idx))
        assert np.allclose(part, full[:, idx], rtol=0, atol=1e-13 * np.abs(full).max())
