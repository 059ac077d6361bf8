"""Batched reconstruction (pat_batch_*) through the C ABI: 32 uneven problems
(Ns ~ U{24..96} sensors per side, Nt ~ U{512..2048}, grids 64^3..192^3) in
one launch per stage.

* Every problem's image equals pat_reconstruct's for the same plan bit for
  bit (same kernels, same summation order), so the batch inherits the
  single-problem parity; the two smallest problems are also checked against
  the FP64 oracle (1e-5 relative L2, the FP32 target).
* The persistent grid (work-groups looping over the work items), smaller
  or absent, gives the same bits.
* The call captured in a HIP graph (torch.cuda.CUDAGraph) and replayed with
  new inputs, with eager work between replays, matches the eager call on
  every replay.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.quality import rel_l2
from paper_1510_01078_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SETTINGS = dict(kernel="kaiser_bessel", sigma_xy=1.5, width_xy=8, sigma_t=1.25, width_t=10)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch_setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_01078_amd.batch import Batch, problem_dict
    probs = inputs.batched_problems(32, seed=1003)
    _say(f"[gpu] batch of {len(probs)}: M {min(p.m for p in probs)}..{max(p.m for p in probs)}, "
         f"Nt {min(p.nt for p in probs)}..{max(p.nt for p in probs)}, "
         f"N {min(p.shape[0] for p in probs)}..{max(p.shape[0] for p in probs)}")
    b = Batch([problem_dict(p) for p in probs], precision="fp32", defaults=SETTINGS)
    gs = [torch.from_numpy(np.ascontiguousarray(p.g)).to("cuda", torch.float32) for p in probs]
    yield probs, b, gs
    b.close()


def test_batch_equals_single_plans(batch_setup):
    from paper_1510_01078_amd import Plan
    probs, b, gs = batch_setup
    outs = b.reconstruct(gs)
    torch.cuda.synchronize()
    mismatched = []
    for i, (p, g, o) in enumerate(zip(probs, gs, outs)):
        pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32", **SETTINGS)
        ref = pl.reconstruct(g)
        torch.cuda.synchronize()
        if not torch.equal(ref, o):
            mismatched.append((i, float((ref - o).abs().max())))
        pl.close()
    _say(f"[gpu] batch vs single plans: {len(probs) - len(mismatched)}/{len(probs)} bitwise equal {mismatched}")
    assert not mismatched


def test_batch_smallest_vs_oracle(batch_setup):
    probs, b, gs = batch_setup
    outs = b.reconstruct(gs)
    torch.cuda.synchronize()
    order = np.argsort([p.m * p.nt * np.prod(p.shape) for p in probs])[:2]
    for i in order:
        p = probs[i]
        ref = oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent)
        e = rel_l2(outs[i].cpu().numpy().astype(np.float64), ref)
        _say(f"[gpu] batch problem {i} (M={p.m}, Nt={p.nt}, N={p.shape[0]}) vs oracle: rel-L2 {e:.3e}")
        assert e <= 1e-5


def test_batch_grid_shapes_same_bits(batch_setup):
    """Default persistent grid, a small persistent grid and one work-group
    per work item give the same bits."""
    probs, b, gs = batch_setup
    a = [o.clone() for o in b.reconstruct(gs)]
    results = []
    for blocks in (1024, 0):
        b.set_grid(blocks)
        results.append([o.clone() for o in b.reconstruct(gs)])
    torch.cuda.synchronize()
    b.set_grid(16384)
    for c in results:
        assert all(torch.equal(x, y) for x, y in zip(a, c))


def test_batch_graph_replays(batch_setup):
    probs, b, gs = batch_setup
    static_in = [g.clone() for g in gs]
    static_out = [torch.empty(s, dtype=torch.float32, device="cuda") for s in b.shapes]
    b.reconstruct(static_in, static_out)  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.reconstruct(static_in, static_out)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda").manual_seed(7)
    for r in range(3):
        for s_in, g in zip(static_in, gs):
            s_in.copy_(g * (1.0 + 0.5 * r) + 0.01 * torch.randn(g.shape, device="cuda", generator=gen))
        torch.cuda.synchronize()
        eager = [o.clone() for o in b.reconstruct([s.clone() for s in static_in])]
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        same = all(torch.equal(x, y) for x, y in zip(eager, static_out))
        _say(f"[gpu] graph replay {r}: equal to eager = {same}")
        assert same
