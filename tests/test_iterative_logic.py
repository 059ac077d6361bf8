"""Landweber iteration and the power-iteration norm estimate on the CPU,
with the plan's forward model and adjoint replaced by a small dense matrix A
and its transpose (the functions only use forward, adjoint, shape, dtype and
device). Pins: the power iteration reaches the largest eigenvalue of A^T A
(numpy's symmetric eigensolver); the k-th iterate equals the closed form
f_k = sum_{i<k} (I - tau A^T A)^i tau A^T g; with tau = 1/||A||^2 the residual
norms never increase (a property of Landweber iteration for
0 < tau <= 1/||A||^2); tau None without x0 is refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1510_01078_amd.iterative import landweber, operator_norm_sq  # noqa: E402


class MatrixPlan:
    """A acting on images of shape (3, 4, 2) (24 unknowns) -> traces (5, 6)."""

    def __init__(self, rng):
        self.shape = (3, 4, 2)
        self.dtype = torch.float64
        self.device = torch.device("cpu")
        self.A = rng.standard_normal((30, 24))
        self.At = torch.from_numpy(self.A)

    def forward(self, f):
        return (self.At @ f.reshape(-1)).reshape(5, 6)

    def adjoint(self, g):
        return (self.At.T @ g.reshape(-1)).reshape(self.shape)


def test_power_iteration_reaches_largest_eigenvalue():
    rng = np.random.default_rng(3)
    pl = MatrixPlan(rng)
    lam = operator_norm_sq(pl, torch.from_numpy(rng.standard_normal(pl.shape)), iters=200)
    exact = np.linalg.eigvalsh(pl.A.T @ pl.A)[-1]
    assert abs(lam - exact) <= 1e-6 * exact


def test_iterates_match_closed_form_and_residuals_decrease():
    rng = np.random.default_rng(4)
    pl = MatrixPlan(rng)
    g = torch.from_numpy(rng.standard_normal((5, 6)))
    tau = 1.0 / np.linalg.eigvalsh(pl.A.T @ pl.A)[-1]
    k = 7
    f, res, tau_out = landweber(pl, g, iters=k, tau=tau)
    assert tau_out == tau and len(res) == k + 1
    AtA = pl.A.T @ pl.A
    M = np.eye(24) - tau * AtA
    b = tau * pl.A.T @ g.numpy().reshape(-1)
    closed = sum(np.linalg.matrix_power(M, i) @ b for i in range(k))
    assert np.allclose(f.numpy().reshape(-1), closed, rtol=1e-12, atol=1e-12)
    gv = g.numpy().reshape(-1)
    assert np.isclose(res[0], np.linalg.norm(gv))
    assert np.isclose(res[-1], np.linalg.norm(gv - pl.A @ closed))
    assert all(b2 <= b1 * (1 + 1e-12) for b1, b2 in zip(res, res[1:]))


def test_tau_needs_a_start_image():
    pl = MatrixPlan(np.random.default_rng(5))
    with pytest.raises(ValueError):
        landweber(pl, torch.zeros((5, 6), dtype=torch.float64), iters=2)
