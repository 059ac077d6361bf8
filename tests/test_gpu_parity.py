"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP32 results must match the oracle within 1e-5 relative L2
(the accuracy contract of the method's FP32 form); the FP64 plain form must
match within its window error for the chosen oversampling and width, which
is far below that (frozen bounds below, each with margin over the value
measured when the bound was set).
"""
import hashlib
import json
import os
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

# the benchmark's tuned setting: lateral sigma 1.5 / w 8, temporal sigma 1.25 / w 10
TUNED = dict(kernel="kaiser_bessel", sigma_xy=1.5, width_xy=8, sigma_t=1.25, width_t=10)


@pytest.mark.parametrize("params", [dict(kernel="gaussian", width_xy=12, width_t=12),
                                    dict(kernel="kaiser_bessel", width_xy=8, width_t=8), TUNED],
                         ids=["gaussian12", "kb8", "tuned"])
def test_config_64x64(dev, params):
    p = inputs.config_problem(1)
    _say("[gpu] 64x64 oracle ...")
    f_or, st = _oracle(p, "c1")
    for precision, tol in (("fp64", 1e-6), ("fp32", 1e-5)):
        _say(f"[gpu] 64x64 {precision} {params}")
        f = _gpu(p, precision, **params)
        e = rel_l2(f, f_or)
        _say(f"[gpu] 64x64 {precision} {params}: image rel-L2 {e:.3e}")
        assert e <= tol


def test_tiny_tuned(dev):
    p = inputs.config_problem(0)
    f_or, _ = _oracle(p, "c0")
    for precision, tol in (("fp64", 1e-6), ("fp32", 1e-5)):
        f = _gpu(p, precision, **TUNED)
        e = rel_l2(f, f_or)
        _say(f"[gpu] tiny tuned {precision}: image rel-L2 {e:.3e}")
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


# --------------------------------------------------------------------------
# headline size (128x128 sensors x 2048 samples -> 256^3) in the benchmark's
# configuration: the whole image against the FP64 oracle's image (written by
# tests/golden/make_headline_image.py, checked by its SHA-256), for FP32 and
# for FP32 with compensated spreading; and the spectrum against the oracle on
# sampled lateral x-modes (the oracle computes those one x-mode at a time)
# --------------------------------------------------------------------------

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _headline_oracle_image():
    meta_path = os.path.join(GOLDEN, "headline_oracle_image.json")
    with open(meta_path) as fh:
        meta = json.load(fh)
    path = os.path.join(GOLDEN, meta["file"])
    if not os.path.exists(path):
        pytest.skip(f"{path} missing: run python tests/golden/make_headline_image.py (about 5 CPU-minutes)")
    h = hashlib.sha256()
    with open(path, "rb") as fh:
        for blk in iter(lambda: fh.read(1 << 22), b""):
            h.update(blk)
    assert h.hexdigest() == meta["sha256"], "headline oracle image does not match its recorded SHA-256"
    return np.load(path), meta


@pytest.mark.parametrize("precision", ["fp32", "fp32_kahan"])
def test_headline_full_image(dev, precision):
    from paper_1510_01078_amd import Plan
    ref32, meta = _headline_oracle_image()
    p = inputs.config_problem(2)
    pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision=precision, **TUNED)
    g = torch.from_numpy(np.ascontiguousarray(p.g)).to(dev, torch.float32)
    _say(f"[gpu] headline full image {precision}")
    f = pl.reconstruct(g)
    torch.cuda.synchronize()
    pl.close()
    ref = torch.from_numpy(ref32).to(dev, torch.float64)
    d = f.double() - ref
    e = float(torch.linalg.vector_norm(d) / meta["l2_norm_fp64"])
    amax = int(torch.argmax(d.abs()))
    max_abs = float(d.abs().flatten()[amax])
    where = np.unravel_index(amax, p.shape)
    _say(f"[gpu] headline {precision}: image rel-L2 vs oracle {e:.3e}; max |error| {max_abs:.3e} at voxel {where} "
         f"({max_abs / meta['max_abs_fp64']:.3e} of the image's largest magnitude)")
    assert e <= 1e-5
    # no localised defect: the worst voxel stays a small fraction of the image's range
    assert max_abs <= 1e-4 * meta["max_abs_fp64"]


def test_headline_size_sampled(dev):
    from paper_1510_01078_amd import Plan
    p = inputs.config_problem(2)
    Nx, Ny, Nz = p.shape
    X, Y, Z = p.extent
    pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32", **TUNED)
    g = torch.from_numpy(np.ascontiguousarray(p.g)).to(dev, torch.float32)
    _say("[gpu] headline size: spectrum on sampled x-modes")
    H = pl.spectrum(g).cpu().numpy().astype(np.complex128)
    torch.cuda.synchronize()
    pl.close()
    # natural-order x positions: the lowest and highest |j| (band edges), and a spread in between
    rows = np.array([1, 2, 40, 77, 100, 127, 128, 129, 131, 160, 200, 254, 255])
    kx, ky, kz = oracle.lattice(Nx, X), oracle.lattice(Ny, Y), oracle.lattice(Nz, Z)
    G = oracle.stage_lateral(p.xy, p.h, p.g, p.dt, Nx, Ny, X, Y, j_index=rows)
    S = oracle.stage_temporal(G, kx[rows], ky, kz, p.c, p.dt)
    F = oracle.apply_weight(S, kx, ky, kz, p.c, j_index=rows)
    lz = np.arange(Nz // 2 + 1)
    ref = np.fft.ifftshift(F, axes=1)[:, :, (lz + Nz // 2) % Nz]
    got = H[(rows - Nx // 2) % Nx]
    e_spec = rel_l2(got, ref)
    per_row = [rel_l2(got[i], ref[i]) for i in range(len(rows)) if np.linalg.norm(ref[i]) > 0]
    _say(f"[gpu] headline: spectrum rel-L2 on {len(rows)} x-modes {e_spec:.3e}; worst row {max(per_row):.3e}")
    assert e_spec <= 1e-5
