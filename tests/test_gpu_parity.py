"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP32 results must match the oracle within 1e-5 relative L2
(the accuracy contract of the method's FP32 form); the FP64 plain form must
match within its window error for the chosen oversampling and width, which
is far below that (frozen bounds below, each with margin over the value
measured when the bound was set).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.quality import rel_l2
from paper_1510_01078_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _plan(p, precision="fp32", **kw):
    from paper_1510_01078_amd import Plan
    return Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision=precision, **kw)


def _gpu(p, precision="fp32", spectrum=False, **kw):
    pl = _plan(p, precision, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    g = torch.from_numpy(np.ascontiguousarray(p.g)).to(dev_of(pl), dt)
    out = pl.spectrum(g) if spectrum else pl.reconstruct(g)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.complex128 if spectrum else np.float64)
    pl.close()
    return res


def dev_of(pl):
    return pl.device


_ORACLE_CACHE = {}


def _oracle(p, key):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent, return_stages=True)
    return _ORACLE_CACHE[key]


# --------------------------------------------------------------------------
# tiny workload (16x16 sensors, 128 samples -> 32^3): image and spectrum
# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-5), ("fp32_kahan", 1e-5)])
def test_tiny_workload(dev, precision, tol):
    p = inputs.config_problem(0)
    f_or, st = _oracle(p, "c0")
    _say(f"[gpu] tiny workload {precision}")
    f = _gpu(p, precision)
    e_f = rel_l2(f, f_or)
    F = _gpu(p, precision, spectrum=True)
    e_F = rel_l2(F, oracle.half_spectrum(st["F"]))
    _say(f"[gpu] tiny {precision}: image rel-L2 {e_f:.3e}, spectrum rel-L2 {e_F:.3e}")
    assert e_f <= tol and e_F <= tol


# --------------------------------------------------------------------------
# ragged random problem: odd M and Nt, non-cubic grid with radix-3/5 sizes,
# partial spread tiles, sensors anywhere on a rectangular plane
# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-5)])
@pytest.mark.parametrize("kernel,w,sig", [("kaiser_bessel", 8, 2.0), ("gaussian", 12, 2.0),
                                          ("kaiser_bessel", 10, 1.25)])
def test_random_ragged(dev, precision, tol, kernel, w, sig):
    rng = np.random.default_rng(77)
    p = inputs.random_problem(rng, 333, 97, (20, 12, 18), (6e-3, 4e-3, 5e-3), dt=30e-9)
    f_or, st = _oracle(p, "ragged")
    _say(f"[gpu] ragged {precision} {kernel} w={w} sigma={sig}")
    kw = dict(kernel=kernel, width_xy=w, width_t=w, sigma_xy=sig, sigma_t=sig)
    f = _gpu(p, precision, **kw)
    F = _gpu(p, precision, spectrum=True, **kw)
    e_f = rel_l2(f, f_or)
    e_F = rel_l2(F, oracle.half_spectrum(st["F"]))
    _say(f"[gpu] ragged {precision} {kernel} w={w} sigma={sig}: image {e_f:.3e} spectrum {e_F:.3e}")
    assert e_f <= tol and e_F <= tol


# --------------------------------------------------------------------------
# 64x64 sensors, 1024 samples -> 128^3, FP32 beside the FP64 plain form,
# Gaussian width 12 at oversampling 2 (and the Kaiser-Bessel default)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kernel,w", [("gaussian", 12), ("kaiser_bessel", 8)])
def test_config_64x64(dev, kernel, w):
    p = inputs.config_problem(1)
    _say("[gpu] 64x64 oracle ...")
    f_or, st = _oracle(p, "c1")
    for precision, tol in (("fp64", 1e-6), ("fp32", 1e-5)):
        _say(f"[gpu] 64x64 {precision} {kernel} w={w}")
        f = _gpu(p, precision, kernel=kernel, width_xy=w, width_t=w)
        e = rel_l2(f, f_or)
        _say(f"[gpu] 64x64 {precision} {kernel} w={w}: image rel-L2 {e:.3e}")
        assert e <= tol


# --------------------------------------------------------------------------
# determinism: the spread is atomic-free, so repeated runs are bitwise equal
# --------------------------------------------------------------------------

def test_bitwise_repeatable(dev):
    from paper_1510_01078_amd import Plan
    p = inputs.config_problem(1)
    pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32")
    g = torch.from_numpy(p.g).to(dev, torch.float32)
    _say("[gpu] repeatability")
    a = pl.reconstruct(g).clone()
    b = pl.reconstruct(g).clone()
    torch.cuda.synchronize()
    pl.close()
    assert torch.equal(a, b)
