"""Parity of the compile-time-length FFT kernels (lateral 256/288/384/512,
inverse 128/192/256/512, temporal 1920/2048/2560/4096) against the FP64 oracle on
small problems chosen so that every instantiated length runs at least once,
for the reconstruction and the forward model, and the x transform once with
a partial last group of rows. The benchmark-size tests cover
384/256/2560 at full size; these cover the rest.

Tolerances: FP32 1e-5 relative L2 (the method's FP32 target); FP64 within
the window error of the case's lateral setting: sigma 2 / w 8 measured below
1e-7 (bound 1e-6), sigma 1.5 / w 8 about 1e-6 for the forward model (bound
3e-6, as in the forward-model tests at the benchmark setting).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import forward_model as fm
from oracle.quality import rel_l2
from paper_1510_01078_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (grid, Nt, extent, lateral sigma, the lengths the plan must reach)
CASES = [
    ((128, 4, 4), 1024, (16e-3, 2e-3, 2e-3), 2.0, dict(nx_over=256, nt_over=2048)),   # lateral 256, inverse x 128, temporal 2048
    ((256, 4, 8), 2048, (16e-3, 1e-3, 2e-3), 2.0, dict(nx_over=512, nt_over=4096)),   # lateral 512, inverse x 256, temporal 4096
    # lateral y 384, inverse y 256; the 4-point x axis oversampled by 1.5 would be 6 < w = 8 points,
    # so the plan widens it to 8 (one footprint meets each grid point once)
    ((4, 256, 4), 1024, (1e-3, 16e-3, 2e-3), 1.5, dict(ny_over=384, nx_over=8)),
    ((512, 4, 4), 512, (16e-3, 1e-3, 2e-3), 2.0, dict()),                             # inverse x 512
    ((4, 4, 512), 512, (1e-3, 1e-3, 16e-3), 2.0, dict()),                             # inverse z 512 (C2R / R2C)
    # lateral 256 over 12 grid rows: the x transform's last group of rows is partial (12 = 8 + 4)
    ((128, 6, 4), 1024, (16e-3, 0.75e-3, 2e-3), 2.0, dict(nx_over=256, ny_over=12)),
    ((144, 4, 4), 960, (18e-3, 1e-3, 2e-3), 2.0, dict(nx_over=288, nt_over=1920)),    # lateral x 288, temporal 1920
    ((4, 192, 4), 512, (1e-3, 24e-3, 2e-3), 1.5, dict(ny_over=288)),                  # lateral y 288, inverse y 192
    ((192, 4, 4), 512, (24e-3, 1e-3, 2e-3), 2.0, dict(nx_over=384)),                  # inverse x 192 (fused gather)
    ((4, 4, 192), 512, (1e-3, 1e-3, 24e-3), 2.0, dict()),                             # inverse z 192 (C2R / R2C)
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("case", CASES, ids=["x256-t2048", "x512-t4096", "y384", "inv-x512", "inv-z512",
                                              "x256-partial-rows", "x288-t1920", "y288-inv-y192", "inv-x192",
                                              "inv-z192"])
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-6)])
def test_ct_lengths_vs_oracle(dev, case, precision, tol):
    from paper_1510_01078_amd import Plan
    shape, nt, ext, sxy, lengths = case
    rng = np.random.default_rng(77)
    p = inputs.random_problem(rng, 40, nt, shape, ext, dt=10e-9)
    f_img = rng.standard_normal(shape)
    ref = oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent)
    ref_a = fm.forward(f_img, p.xy, p.nt, p.dt, p.c, p.extent)
    pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision=precision, kernel="kaiser_bessel",
              sigma_xy=sxy, width_xy=8, sigma_t=2.0, width_t=8)
    for key, val in lengths.items():
        assert pl.info[key] == val, (key, pl.info[key])
    g = torch.from_numpy(p.g).to(pl.device, pl.dtype)
    fi = torch.from_numpy(f_img).to(pl.device, pl.dtype)
    e_r = rel_l2(pl.reconstruct(g).cpu().numpy().astype(np.float64), ref)
    e_a = rel_l2(pl.forward(fi).cpu().numpy().astype(np.float64), ref_a)
    info = {k: pl.info[k] for k in ("nx_over", "ny_over", "nt_over", "forward_fused")}
    pl.close()
    _say(f"[gpu] {shape} Nt {nt} {precision} {info}: reconstruction {e_r:.3e}, forward {e_a:.3e}")
    if precision == "fp64" and sxy < 2.0:
        tol = 3e-6  # the sigma 1.5 / w 8 window's own error
    assert e_r <= tol and e_a <= tol
