"""GPU forward model A (pat_forward), its adjoint A* (pat_adjoint) and the
position derivatives (pat_forward_dxy), through the C ABI, against the FP64
oracle of the forward model; adjointness of the GPU pair; the autograd
wrapper and Landweber iteration.

Tolerances: FP32 results within 1e-5 relative L2 of the oracle (the
method's FP32 accuracy target); the FP64 plain form within its setting's
window error (frozen per setting below). The GPU kernels of A are the exact
transposes of those of A*, so <A f, g> = <f, A* g> holds to rounding:
1e-12 relative in FP64, 1e-6 in FP32.
"""
import sys

import numpy as np
import pytest

from oracle import forward_model as fm
from oracle.quality import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C = 1500.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _problem(seed=31, m=211, nt=97, shape=(24, 20, 18), extent=(6e-3, 5e-3, 5e-3), dt=30e-9):
    rng = np.random.default_rng(seed)
    X, Y, _ = extent
    xy = np.stack([rng.uniform(-X / 2, X / 2, m), rng.uniform(-Y / 2, Y / 2, m)], axis=1)
    f = rng.standard_normal(shape)
    g = rng.standard_normal((m, nt))
    return dict(xy=xy, nt=nt, dt=dt, shape=shape, extent=extent, f=f, g=g)


def _plan(p, precision, **kw):
    from paper_1510_01078_amd import Plan
    return Plan(p["xy"], p["nt"], p["dt"], C, p["shape"], p["extent"], precision=precision, **kw)


def _t(a, pl):
    return torch.from_numpy(np.ascontiguousarray(a)).to(pl.device, pl.dtype)


_OR = {}


def _oracle(p, key):
    if key not in _OR:
        _OR[key] = dict(
            A=fm.forward(p["f"], p["xy"], p["nt"], p["dt"], C, p["extent"]),
            As=fm.adjoint(p["g"], p["xy"], p["dt"], C, p["shape"], p["extent"]),
            Ax=fm.forward(p["f"], p["xy"], p["nt"], p["dt"], C, p["extent"], deriv="x"),
            Ay=fm.forward(p["f"], p["xy"], p["nt"], p["dt"], C, p["extent"], deriv="y"),
        )
    return _OR[key]


# (window setting, FP64 bound): the FP64 plain form is limited by the window
# error of its setting; bounds frozen with margin over the measured values
# (sigma 2, KB w 8: 9e-8; benchmark setting sigma 1.5/1.25: 1.1e-6 for the
# position derivative, whose i*K factor weights the high modes)
SETTINGS = [(dict(kernel="kaiser_bessel", sigma_xy=2.0, width_xy=8, sigma_t=2.0, width_t=8), 1e-6),
            (dict(kernel="kaiser_bessel", sigma_xy=1.5, width_xy=8, sigma_t=1.25, width_t=10), 3e-6),
            (dict(kernel="gaussian", sigma_xy=2.0, width_xy=12, sigma_t=2.0, width_t=12), 1e-6)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("setting", SETTINGS, ids=["kb8", "tuned", "gauss12"])
def test_forward_adjoint_vs_oracle(dev, precision, setting):
    kw, tol64 = setting
    tol = tol64 if precision == "fp64" else 1e-5
    p = _problem()
    ref = _oracle(p, "base")
    pl = _plan(p, precision, **kw)
    _say(f"[gpu] forward/adjoint {precision} {kw}")
    A = pl.forward(_t(p["f"], pl)).cpu().numpy().astype(np.float64)
    As = pl.adjoint(_t(p["g"], pl)).cpu().numpy().astype(np.float64)
    Ax = pl.forward_dxy(_t(p["f"], pl), 0).cpu().numpy().astype(np.float64)
    Ay = pl.forward_dxy(_t(p["f"], pl), 1).cpu().numpy().astype(np.float64)
    pl.close()
    e = [rel_l2(A, ref["A"]), rel_l2(As, ref["As"]), rel_l2(Ax, ref["Ax"]), rel_l2(Ay, ref["Ay"])]
    _say(f"[gpu] {precision} {kw['kernel']} s{kw['sigma_xy']}/{kw['sigma_t']}: A {e[0]:.3e} A* {e[1]:.3e} "
         f"dA/dx {e[2]:.3e} dA/dy {e[3]:.3e}")
    assert max(e) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_gpu_pair_adjointness(dev, precision, tol):
    p = _problem(seed=32, m=150, nt=64, shape=(20, 16, 24), extent=(5e-3, 4e-3, 6e-3))
    pl = _plan(p, precision, sigma_xy=1.5, sigma_t=1.25, width_t=10)
    f, g = _t(p["f"], pl), _t(p["g"], pl)
    Af = pl.forward(f).double()
    Asg = pl.adjoint(g).double()
    lhs = float((Af * g.double()).sum())
    rhs = float((f.double() * Asg).sum())
    scale = float(torch.linalg.vector_norm(Af) * torch.linalg.vector_norm(g.double()))
    pl.close()
    _say(f"[gpu] adjointness {precision}: |<Af,g> - <f,A*g>| / (|Af||g|) = {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= tol * scale


@pytest.mark.parametrize("precision,width,fused,tol", [
    ("fp64", 16, 0, 1e-10), ("fp64", 8, 1, 1e-6), ("fp32", 16, 1, 1e-5)],
    ids=["fp64-w16-two-kernel", "fp64-w8-fused", "fp32-w16-fused"])
def test_forward_fused_and_two_kernel_paths(dev, precision, width, fused, tol):
    """Oversampled x length 320: the strip of 16 + w - 1 rows that the fused
    x-FFT + interpolation kernel holds in LDS fits for FP32 and for FP64 with
    w = 8, not for FP64 with w = 16, which takes the two-kernel form. Both
    forms against the oracle."""
    p = _problem(seed=33, m=40, nt=24, shape=(160, 12, 8), extent=(8e-3, 3e-3, 2e-3))
    ref = fm.forward(p["f"], p["xy"], p["nt"], p["dt"], C, p["extent"])
    pl = _plan(p, precision, kernel="kaiser_bessel", sigma_xy=2.0, width_xy=width, sigma_t=2.0, width_t=width)
    assert pl.info["nx_over"] == 320
    path = pl.info["forward_fused"]
    A = pl.forward(_t(p["f"], pl)).cpu().numpy().astype(np.float64)
    pl.close()
    e = rel_l2(A, ref)
    _say(f"[gpu] forward n_x 320 {precision} w{width}: fused={path} rel-L2 {e:.3e}")
    assert path == fused
    assert e <= tol


def test_plane_wave_headline_geometry(dev):
    """At the benchmark's size (128x128 warped sensors, 2048 samples, 256^3),
    a lattice plane wave must come back as the standing wave
    cos(K0x x_m + K0y y_m + phi) cos(c|K0| t_n) at every sensor (exact for A)."""
    from paper_1510_01078_amd import Plan, inputs
    p = inputs.config_problem(2)
    Nx, Ny, Nz = p.shape
    X, Y, Z = p.extent
    pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32", kernel="kaiser_bessel",
              sigma_xy=1.5, width_xy=8, sigma_t=1.25, width_t=10)
    assert pl.info["forward_fused"] == 1
    x = (np.arange(Nx) - Nx / 2) * X / Nx
    y = (np.arange(Ny) - Ny / 2) * Y / Ny
    z = np.arange(Nz) * Z / Nz
    worst = 0.0
    for (j0, k0, l0, phi) in [(37, -11, 23, 0.4), (-90, 101, 7, 1.3), (5, 0, 110, -0.6)]:
        kx, ky, kz = 2 * np.pi * j0 / X, 2 * np.pi * k0 / Y, 2 * np.pi * l0 / Z
        f = np.cos(kx * x[:, None, None] + ky * y[None, :, None] + kz * z[None, None, :] + phi)
        g = pl.forward(torch.from_numpy(f).to(pl.device, torch.float32)).cpu().numpy().astype(np.float64)
        t = np.arange(p.nt) * p.dt
        kabs = np.sqrt(kx * kx + ky * ky + kz * kz)
        ref = np.cos(kx * p.xy[:, 0] + ky * p.xy[:, 1] + phi)[:, None] * np.cos(p.c * kabs * t)[None, :]
        e = rel_l2(g, ref)
        _say(f"[gpu] plane wave ({j0},{k0},{l0}) at 256^3: rel-L2 {e:.3e}")
        worst = max(worst, e)
    pl.close()
    assert worst <= 1e-5


def test_autograd_position_gradient(dev):
    """d/dxy of L = <w, A f> through torch.autograd: against the oracle's
    analytic gradient, and against central differences of the GPU forward
    model (FP64, plans rebuilt at shifted positions)."""
    from paper_1510_01078_amd import Plan
    from paper_1510_01078_amd.autograd import forward_model
    p = _problem(seed=33, m=40, nt=80, shape=(16, 16, 16), extent=(4e-3, 4e-3, 4e-3))
    w = np.random.default_rng(34).standard_normal((40, 80))
    kw = dict(kernel="kaiser_bessel", sigma_xy=2.0, width_xy=12, sigma_t=2.0, width_t=12)
    pl = _plan(p, "fp64", **kw)
    f = _t(p["f"], pl).requires_grad_(True)
    xy = torch.from_numpy(p["xy"].copy()).requires_grad_(True)
    wt = _t(w, pl)
    loss = (forward_model(f, xy, pl) * wt).sum()
    gf, gxy = torch.autograd.grad(loss, (f, xy))
    gf_ref = pl.adjoint(wt).cpu().numpy()
    pl.close()
    ax = fm.forward(p["f"], p["xy"], p["nt"], p["dt"], C, p["extent"], deriv="x")
    ay = fm.forward(p["f"], p["xy"], p["nt"], p["dt"], C, p["extent"], deriv="y")
    gxy_or = np.stack([(w * ax).sum(1), (w * ay).sum(1)], 1)
    e_or = rel_l2(gxy.numpy(), gxy_or)
    assert np.array_equal(gf.cpu().numpy(), gf_ref)
    # central differences in FP64 on the GPU for a few sensors
    h = 1e-6 * p["extent"][0]
    fd = np.zeros((4, 2))
    for i, m in enumerate([0, 7, 19, 33]):
        for ax_i in range(2):
            vals = []
            for sgn in (1, -1):
                q = p["xy"].copy()
                q[m, ax_i] += sgn * h
                plq = Plan(q, p["nt"], p["dt"], C, p["shape"], p["extent"], precision="fp64", **kw)
                vals.append(float((plq.forward(_t(p["f"], plq)).cpu().numpy() * w).sum()))
                plq.close()
            fd[i, ax_i] = (vals[0] - vals[1]) / (2 * h)
    e_fd = rel_l2(gxy.numpy()[[0, 7, 19, 33]], fd)
    _say(f"[gpu] position gradient: vs oracle {e_or:.3e}, vs GPU central differences {e_fd:.3e}")
    assert e_or <= 1e-6
    assert e_fd <= 1e-5


def test_landweber_vs_oracle(dev):
    from paper_1510_01078_amd.iterative import landweber
    p = _problem(seed=35, m=64, nt=48, shape=(8, 8, 12), extent=(3e-3, 3e-3, 4.5e-3), dt=40e-9)
    pl = _plan(p, "fp64", kernel="kaiser_bessel", sigma_xy=2.0, width_xy=12, sigma_t=2.0, width_t=12)
    g = _t(p["g"], pl)
    x0 = _t(np.random.default_rng(36).standard_normal(p["shape"]), pl)
    f, res, tau = landweber(pl, g, iters=10, x0=x0, power_iters=20)
    f = f.cpu().numpy()
    pl.close()
    f_or, res_or = fm.landweber(p["g"], p["xy"], p["dt"], C, p["shape"], p["extent"], 10, tau)
    e = rel_l2(f, f_or)
    _say(f"[gpu] Landweber x10: tau {tau:.4e}, residuals {res[0]:.4e} -> {res[-1]:.4e}; vs oracle {e:.3e}")
    assert all(res[i + 1] <= res[i] * (1 + 1e-9) for i in range(10))
    assert e <= 1e-6
    assert abs(res[-1] - res_or[-1]) <= 1e-6 * res_or[-1]
