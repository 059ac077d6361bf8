"""The packed lateral spread on the layouts that stress it, against the FP64
oracle: a dense cluster of sensors (its patches hold many more slots than
one staging round of eight, so the multi-round path runs and the lane tables
are reread per bin group), sensors on the plane's edges and corners (their
footprints wrap around the periodic grid, so one slot mixes both sides), and
a last bin group shorter than sixteen (the 16-byte loads to LDS past the
band's end are moved onto its last 16-byte unit; the band's bin count is
even, so every sensor's row starts on a 16-byte boundary).

Checks: reconstruction and adjoint within 1e-5 (FP32) and 1e-6 (FP64 at the
window setting below) of the oracle; the batched reconstruction equal bit for
bit to single plans; the plan's slot count between a quarter of the (sensor,
patch) pairs and all of them.
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

SETTINGS = dict(kernel="kaiser_bessel", sigma_xy=2.0, width_xy=8, sigma_t=2.0, width_t=8)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _problem(seed, nt):
    """400 sensors in a 0.6 mm square near the centre of an 8 x 6 mm plane,
    48 on its edges and corners, 40 spread over the rest; random traces."""
    rng = np.random.default_rng(seed)
    X, Y = 8e-3, 6e-3
    cluster = rng.uniform(-0.3e-3, 0.3e-3, size=(400, 2)) + np.array([0.4e-3, -0.2e-3])
    edge = []
    for t in np.linspace(-0.5, 0.5, 12, endpoint=False):
        edge += [(t * X, -0.5 * Y), (t * X, 0.4999 * Y), (-0.5 * X, t * Y), (0.4999 * X, t * Y)]
    rest = np.column_stack([rng.uniform(-0.5 * X, 0.5 * X, 40), rng.uniform(-0.5 * Y, 0.5 * Y, 40)])
    xy = np.vstack([cluster, np.array(edge), rest])
    h = np.full(len(xy), X * Y / len(xy))
    g = rng.standard_normal((len(xy), nt))
    return inputs.Problem("cluster", xy, h, g, 20e-9, 1500.0, (24, 20, 12), (X, Y, 3e-3))


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-6)])
def test_cluster_and_edges_vs_oracle(dev, precision, tol):
    from paper_1510_01078_amd import Plan
    p = _problem(91, 75)
    ref = oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent)
    ref_a = fm.adjoint(p.g, p.xy, p.dt, p.c, p.shape, p.extent)
    pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision=precision, **SETTINGS)
    info = pl.info
    g = torch.from_numpy(p.g).to(pl.device, pl.dtype)
    e_r = rel_l2(pl.reconstruct(g).cpu().numpy().astype(np.float64), ref)
    e_a = rel_l2(pl.adjoint(g).cpu().numpy().astype(np.float64), ref_a)
    pl.close()
    _say(f"[gpu] cluster + edges {precision}: band bins {info['band_bins']}, slots {info['spread_slots']} for "
         f"{info['spread_pairs']} (sensor, patch) pairs; reconstruction {e_r:.3e}, adjoint {e_a:.3e}")
    assert info["band_bins"] % 2 == 0 and info["band_bins"] % 16 != 0
    # every pass serves at most four sensors, and the cluster's patches need several rounds of 8 slots
    assert info["spread_pairs"] / 4 <= info["spread_slots"] <= info["spread_pairs"]
    assert info["spread_slots"] > 8 * 4
    assert e_r <= tol and e_a <= tol


def test_cluster_batch_equals_single(dev):
    from paper_1510_01078_amd import Plan
    from paper_1510_01078_amd.batch import Batch, problem_dict
    probs = [_problem(92, 75), _problem(93, 80)]
    b = Batch([problem_dict(p) for p in probs], precision="fp32", defaults=SETTINGS)
    gs = [torch.from_numpy(np.ascontiguousarray(p.g)).to("cuda", torch.float32) for p in probs]
    outs = b.reconstruct(gs)
    torch.cuda.synchronize()
    same = []
    for p, g, o in zip(probs, gs, outs):
        pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32", **SETTINGS)
        same.append(bool(torch.equal(pl.reconstruct(g), o)))
        pl.close()
    b.close()
    _say(f"[gpu] cluster batch vs single plans bitwise: {same}")
    assert all(same)
