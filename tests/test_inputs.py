"""Synthetic input generators: layouts, weights and the ball signal."""
import numpy as np
import pytest

from paper_1510_01078_amd import inputs


def test_warp_monotone_symmetric():
    x = inputs.warp_1d(64, 10e-3, 1.5)
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x, -x[::-1], rtol=0, atol=1e-18)
    # denser at the centre than at the edge
    d = np.diff(x)
    assert d[len(d) // 2] < 0.2 * d[0]


def test_weights_sum_to_plane_area():
    for ns, side in ((16, 10e-3), (64, 20e-3), (128, 25e-3)):
        xy, h = inputs.warped_sensors(ns, side)
        assert abs(h.sum() - side * side) <= 1e-14 * side * side
        assert np.all(h > 0)
        assert np.all(np.abs(xy) < side / 2)


def test_jitter_keeps_order_and_weights():
    rng = np.random.default_rng(1)
    xy0, h0 = inputs.warped_sensors(32, 25e-3)
    xy1, h1 = inputs.warped_sensors(32, 25e-3, jitter=0.05, rng=rng)
    assert np.array_equal(h0, h1)
    gx = xy1[:, 0].reshape(32, 32)
    gy = xy1[:, 1].reshape(32, 32)
    assert np.all(np.diff(gx, axis=0) > 0)
    assert np.all(np.diff(gy, axis=1) > 0)
    assert np.all(xy1 >= -12.5e-3) and np.all(xy1 < 12.5e-3)
    w = inputs.cell_widths_1d(inputs.warp_1d(32, 12.5e-3), 25e-3)
    dev = np.abs(xy1 - xy0).reshape(32, 32, 2)
    assert np.all(dev[:, :, 0] <= 0.05 * w[:, None] + 1e-18)


def test_seeded_workloads_reproducible():
    a = inputs.config_problem(1)
    b = inputs.config_problem(1)
    assert np.array_equal(a.g, b.g) and np.array_equal(a.xy, b.xy)
    c = inputs.config_problem(1, seed=5)
    assert not np.array_equal(a.g, c.g)


def _fibonacci_sphere(n):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def test_ball_signal_matches_spherical_mean_formula():
    """3-D Poisson/Kirchhoff formula: p(x,t) = d/dt [ t * M_{ct} f (x) ] with M_r the
    mean of f over the sphere of radius r about x; evaluated by quadrature on a
    Fibonacci sphere and a central difference in t, for a uniform ball."""
    c = inputs.C_SOUND
    R, p0 = 1e-3, 0.8
    centre = np.array([0.4e-3, -0.3e-3, 3e-3])
    balls = inputs.Balls(centre[None, :], np.array([R]), np.array([p0]))
    xy = np.array([[0.0, 0.0], [1e-3, 2e-3]])
    dt = 20e-9
    nt = 400
    g = inputs.ball_traces(xy, balls, nt, dt, c)
    pts = _fibonacci_sphere(400000)
    for m in range(2):
        x = np.array([xy[m, 0], xy[m, 1], 0.0])
        d = np.linalg.norm(centre - x)
        for n in range(int((d - 0.9 * R) / (c * dt)), int((d + 0.9 * R) / (c * dt)), 7):
            t = n * dt
            eps = 0.5 * dt

            def tm(tt):
                r = c * tt
                inside = np.linalg.norm(x + r * pts - centre, axis=1) < R
                return tt * p0 * inside.mean()
            p_num = (tm(t + eps) - tm(t - eps)) / (2 * eps)
            assert abs(p_num - g[m, n]) < 0.02 * p0, (m, n, p_num, g[m, n])


def test_vessel_phantom_inside_cube():
    rng = np.random.default_rng(1002)
    b = inputs.vessel_phantom(rng, 40, 25e-3, 25e-3)
    assert 500 < len(b) < 20000
    assert np.all(np.abs(b.centres[:, :2]) < 12.5e-3)
    assert np.all(b.centres[:, 2] > 0) and np.all(b.centres[:, 2] < 25e-3)
    assert np.all((b.radii >= 50e-6) & (b.radii <= 200e-6))


def test_smooth235():
    assert inputs.smooth235(257) == 270
    assert inputs.smooth235(512) == 512
    assert inputs.smooth235(7) == 8
    assert inputs.smooth235(11) == 12


# ----------------------------------------------------------------------------
# equi-steradian placement (Appendix A) and the r^3 weights (Section 6.2)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,r0,drd", [(360, 8e-3, 16e-3), (870, 6e-3, 18e-3), (100, 10e-3, 8e-3)])
def test_equi_steradian_rings_follow_the_slice_recursion(n, r0, drd):
    """Rings hold 1 (the pole), then powers of two non-decreasing outward;
    rebuilding the slice boundaries from the ring counts with
    cos(th_k) = cos(th_{k-1}) - omega j_k/(2 pi), cos(th_1) = 1 - omega/(2 pi),
    omega = 2 pi (1 - cos th_max)/n, puts every ring at the projected
    mid-angle of its slice exactly (the last slice is cut at th_max)."""
    import math
    xy, r = inputs.equi_steradian_sensors(n, r0, drd)
    rho = np.hypot(xy[:, 0], xy[:, 1])
    radii, counts = np.unique(np.round(rho, 12), return_counts=True)
    assert counts[0] == 1 and radii[0] == 0.0
    assert all(c & (c - 1) == 0 for c in counts[1:])
    assert all(a <= b for a, b in zip(counts[1:], counts[2:]))
    assert np.all(rho < 0.5 * drd)
    assert n <= len(xy) <= 1.25 * n
    th_max = math.atan2(0.5 * drd, r0)
    omega = 2 * math.pi * (1 - math.cos(th_max)) / n
    cos_prev = 1 - omega / (2 * math.pi)
    for rad, j in zip(radii[1:], counts[1:]):
        cos_next = max(cos_prev - omega * j / (2 * math.pi), math.cos(th_max))
        th_mid = 0.5 * (math.acos(cos_prev) + math.acos(cos_next))
        assert abs(r0 * math.tan(th_mid) - rad) <= 1e-12 + 1e-9 * rad
        cos_prev = cos_next


def test_equi_steradian_local_equidistance():
    """Seen from the centre of interest, nearest-neighbour angular spacings
    vary little (the aim of the power-of-two doubling rule)."""
    xy, _ = inputs.equi_steradian_sensors(360, 8e-3, 16e-3)
    v = np.stack([xy[:, 0], xy[:, 1], -np.full(len(xy), 8e-3)], 1)
    v /= np.linalg.norm(v, axis=1)[:, None]
    ang = np.arccos(np.clip(v @ v.T, -1, 1))
    np.fill_diagonal(ang, np.inf)
    nn = ang.min(1)
    assert nn.std() / nn.mean() < 0.15 and nn.max() / nn.min() < 1.6


def test_r_cubed_weights():
    xy, r = inputs.equi_steradian_sensors(360, 8e-3, 16e-3)
    area = np.pi * 8e-3 ** 2
    h = inputs.power_weights(xy, r, 3.0, area)
    ratio = h / r ** 3
    assert np.ptp(ratio) <= 1e-12 * ratio.mean()
    assert abs(h.sum() - area) <= 1e-15 * area * len(h)
