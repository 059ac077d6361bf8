"""Pins of the image-quality measures of Appendix B (oracle/quality.py).

Each measure is fixed by values the mathematics determines without the
oracle's code path: numpy's own correlation routine and exact cases of the
correlation coefficient (Appendix B, eq. corrcoeff), the closed-form Sobel
response of linear ramps and of a single impulse for the Tenenbaum sharpness
(Appendix B, the Sobel operator g and its transpose, divided by the element
count), and a one-hot volume for the maximum-intensity projections.

Every pin is also run against a copy of the measure with one plausible
mistake planted (mean not removed, wrong normalisation, Sobel used twice
instead of with its transpose, slices taken along the wrong axis, projection
axes swapped): each planted copy must fail at least one pin.
"""
import numpy as np
import pytest

from oracle import quality


# ---------------------------------------------------------------------------
# pin predicates: True when the measure passes
# ---------------------------------------------------------------------------

def _corr_pins(fn):
    rng = np.random.default_rng(11)
    ok = True
    for shape in [(50,), (7, 9), (5, 6, 4)]:
        a = rng.standard_normal(shape) + 3.0
        b = 0.4 * a + rng.standard_normal(shape) - 2.0
        ok &= abs(fn(a, b) - np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 1e-13
        # affine relations: rho(u, s*u + t) = sign(s)
        ok &= abs(fn(a, 2.5 * a + 7.0) - 1.0) < 1e-13
        ok &= abs(fn(a, -0.3 * a + 1.0) + 1.0) < 1e-13
    # zero-mean orthogonal patterns over whole periods: rho = 0 exactly, also
    # with constant offsets added (the mean must be removed)
    n = 64
    i = np.arange(n)
    s, c = np.sin(2 * np.pi * 3 * i / n), np.cos(2 * np.pi * 5 * i / n)
    ok &= abs(fn(s + 10.0, c - 4.0)) < 1e-13
    return bool(ok)


def _ramp(shape, coeffs):
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    return sum(c * g for c, g in zip(coeffs, grids)) + 0.7


def _tenenbaum_pins(fn):
    ok = True
    # 2-D ramp A*i + B*j: the Sobel responses at every interior point are 8B
    # (g, along the second axis) and 8A (g^T), so
    # T = (n0-2)(n1-2) * 64 (A^2 + B^2) / (n0 n1)
    for (n0, n1), (A, B) in [((9, 13), (0.5, -1.25)), ((12, 7), (2.0, 0.0)), ((6, 6), (0.0, 3.0))]:
        want = (n0 - 2) * (n1 - 2) * 64.0 * (A * A + B * B) / (n0 * n1)
        ok &= abs(fn(_ramp((n0, n1), (A, B))) - want) < 1e-12 * max(1.0, want)
    # 3-D ramp A*i + B*j + C*k: the operator acts on every slice along the
    # last axis, where C*k is a constant; each of the n2 slices gives the 2-D
    # value, and the sum is divided by all n0 n1 n2 elements
    n0, n1, n2 = 8, 11, 5
    A, B, Cc = 1.5, -0.5, 4.0
    want = n2 * (n0 - 2) * (n1 - 2) * 64.0 * (A * A + B * B) / (n0 * n1 * n2)
    ok &= abs(fn(_ramp((n0, n1, n2), (A, B, Cc))) - want) < 1e-12 * want
    # impulse of height v at an interior point away from the border: each of
    # the two responses holds the Sobel entries once (squares summing to 12)
    u = np.zeros((10, 12))
    u[4, 6] = 2.0
    ok &= abs(fn(u) - 2.0 * 12.0 * 4.0 / u.size) < 1e-14
    return bool(ok)


def _mips_pins(fn):
    ok = True
    shape = (5, 7, 9)
    a, b, c = 3, 1, 6
    u = np.zeros(shape)
    u[a, b, c] = 2.5
    px, py, pz = fn(u)
    ok &= px.shape == (7, 9) and py.shape == (5, 9) and pz.shape == (5, 7)
    if not ok:
        return False
    ok &= px[b, c] == 2.5 and np.count_nonzero(px) == 1
    ok &= py[a, c] == 2.5 and np.count_nonzero(py) == 1
    ok &= pz[a, b] == 2.5 and np.count_nonzero(pz) == 1
    # a second, smaller value on the same ray does not change the projection
    u[a, b, 0] = 1.0
    ok &= fn(u)[2][a, b] == 2.5
    return bool(ok)


# ---------------------------------------------------------------------------
# the oracle's measures pass
# ---------------------------------------------------------------------------

def test_corrcoef_pins():
    assert _corr_pins(quality.corrcoef)


def test_tenenbaum_pins():
    assert _tenenbaum_pins(quality.tenenbaum)


def test_mips_pins():
    assert _mips_pins(quality.mips)


def test_rel_l2_closed_form():
    b = np.array([3.0, 4.0])
    assert quality.rel_l2(np.array([3.0, 4.0 + 0.5]), b) == pytest.approx(0.1, rel=1e-15)
    bc = np.array([3.0 + 4.0j])
    assert quality.rel_l2(bc * (1 + 1e-3j), bc) == pytest.approx(1e-3, rel=1e-12)


# ---------------------------------------------------------------------------
# planted mistakes: each fails a pin
# ---------------------------------------------------------------------------

def _corr_no_mean(u1, u2):
    a = np.asarray(u1, float).ravel()
    b = np.asarray(u2, float).ravel()
    return float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))


def _corr_wrong_norm(u1, u2):
    a = np.asarray(u1, float).ravel()
    b = np.asarray(u2, float).ravel()
    a, b = a - a.mean(), b - b.mean()
    return float(np.dot(a, b) / np.dot(a, a))


_SOBEL = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]])


def _tenen_variant(u, second, axis_last=True, per_slice_norm=False):
    u = np.asarray(u, float)
    if u.ndim == 2:
        slices = [u]
    elif axis_last:
        slices = [u[..., i] for i in range(u.shape[-1])]
    else:
        slices = [u[i] for i in range(u.shape[0])]
    total = 0.0
    for s in slices:
        n0, n1 = s.shape
        gx = np.zeros((n0 - 2, n1 - 2))
        gy = np.zeros((n0 - 2, n1 - 2))
        for a in range(3):
            for b in range(3):
                gx += _SOBEL[a, b] * s[a:a + n0 - 2, b:b + n1 - 2]
                gy += second[a, b] * s[a:a + n0 - 2, b:b + n1 - 2]
        total += float(np.sum(gx * gx + gy * gy))
    return total / (slices[0].size if per_slice_norm else u.size)


def test_planted_mistakes_are_caught():
    assert not _corr_pins(_corr_no_mean)
    assert not _corr_pins(_corr_wrong_norm)
    # the variant with the right choices passes, so the planted differences are what fail
    assert _tenenbaum_pins(lambda u: _tenen_variant(u, _SOBEL.T))
    assert not _tenenbaum_pins(lambda u: _tenen_variant(u, _SOBEL))            # g twice, no transpose
    assert not _tenenbaum_pins(lambda u: _tenen_variant(u, _SOBEL.T, axis_last=False))  # wrong slicing axis
    assert not _tenenbaum_pins(lambda u: _tenen_variant(u, _SOBEL.T, per_slice_norm=True))  # wrong normalisation
    assert not _mips_pins(lambda u: (np.asarray(u).max(axis=1), np.asarray(u).max(axis=0),
                                     np.asarray(u).max(axis=2)))
    assert not _mips_pins(lambda u: (np.asarray(u).min(axis=0), np.asarray(u).min(axis=1),
                                     np.asarray(u).min(axis=2)))
