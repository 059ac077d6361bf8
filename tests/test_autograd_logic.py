"""The autograd wrapper of the forward model on the CPU, with the plan
replaced by an analytic model that has the same interface (forward,
adjoint, forward_dxy, sensor_xy): g[m, n] = sum_e f[e] cos(kx_e x_m + ky_e y_m + w_n).
Pins: the image gradient of L = sum(W * g) is A^T W written out directly;
the position gradient matches central differences of L over plans rebuilt
at shifted positions (FP64, h = 1e-6); positions other than the plan's are
refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1510_01078_amd.autograd import forward_model  # noqa: E402

SHAPE = (3, 2, 2)
NT = 5


class CosPlan:
    def __init__(self, xy, seed=8):
        rng = np.random.default_rng(seed)
        self.sensor_xy = np.asarray(xy, dtype=np.float64)
        n = int(np.prod(SHAPE))
        self.kx = torch.from_numpy(rng.uniform(-3, 3, n))
        self.ky = torch.from_numpy(rng.uniform(-3, 3, n))
        self.w = torch.from_numpy(rng.uniform(0, 2, NT))
        self.shape = SHAPE
        self.dtype = torch.float64
        self.device = torch.device("cpu")

    def _phase(self):
        xy = torch.from_numpy(self.sensor_xy)
        # [M, NT, E]
        return (xy[:, 0, None, None] * self.kx[None, None, :] + xy[:, 1, None, None] * self.ky[None, None, :]
                + self.w[None, :, None])

    def forward(self, f):
        return torch.einsum("mne,e->mn", torch.cos(self._phase()), f.reshape(-1))

    def adjoint(self, g):
        return torch.einsum("mne,mn->e", torch.cos(self._phase()), g).reshape(SHAPE)

    def forward_dxy(self, f, axis):
        k = self.kx if axis == 0 else self.ky
        return torch.einsum("mne,e->mn", -torch.sin(self._phase()) * k[None, None, :], f.reshape(-1))


def _setup():
    rng = np.random.default_rng(9)
    xy = rng.uniform(-1, 1, (4, 2))
    f = torch.from_numpy(rng.standard_normal(SHAPE))
    W = torch.from_numpy(rng.standard_normal((4, NT)))
    return xy, f, W


def test_image_gradient_is_the_adjoint():
    xy, f, W = _setup()
    pl = CosPlan(xy)
    fr = f.clone().requires_grad_(True)
    (forward_model(fr, torch.from_numpy(xy), pl) * W).sum().backward()
    phase = (xy[:, 0, None, None] * pl.kx.numpy() + xy[:, 1, None, None] * pl.ky.numpy() + pl.w.numpy()[None, :, None])
    direct = np.einsum("mne,mn->e", np.cos(phase), W.numpy()).reshape(SHAPE)
    assert np.allclose(fr.grad.numpy(), direct, rtol=1e-13, atol=1e-13)


def test_position_gradient_matches_central_differences():
    xy, f, W = _setup()
    xt = torch.from_numpy(xy.copy()).requires_grad_(True)
    (forward_model(f, xt, CosPlan(xy)) * W).sum().backward()
    h = 1e-6
    fd = np.zeros_like(xy)
    for m in range(xy.shape[0]):
        for a in range(2):
            xp, xm = xy.copy(), xy.copy()
            xp[m, a] += h
            xm[m, a] -= h
            lp = float((CosPlan(xp).forward(f) * W).sum())
            lm = float((CosPlan(xm).forward(f) * W).sum())
            fd[m, a] = (lp - lm) / (2 * h)
    assert np.allclose(xt.grad.numpy(), fd, rtol=1e-6, atol=1e-8)


def test_other_positions_are_refused():
    xy, f, _ = _setup()
    with pytest.raises(ValueError):
        forward_model(f, torch.from_numpy(xy + 1e-3), CosPlan(xy))
