"""Batched reconstruction (pat_batch_*) through the C ABI on the uneven
problems of the batched workload (Ns ~ U{24..96} sensors per side, Nt ~
U{512..2048}, grids 64^3..192^3), each with the window setting the
autotuner picks for it (oversampling in {1.25, 1.5, 2}, widths in
{6, 8, 12}, FP32 target 1e-5 with half of it as margin), in one launch per
stage.

* Every problem's image equals pat_reconstruct's for the same plan bit for
  bit (same kernels, same summation order), so the batch inherits the
  single-problem parity. Against the FP64 oracle: the two smallest problems
  on the whole image, the largest problem (192^3 with the longest traces
  of the draw) and one mid-size problem on the spectrum of sampled x-modes
  (the oracle computes those one x-mode at a time), all within 1e-5.
* The tuner's own accuracy reference (FP64 GPU reconstruction at sigma 2,
  Kaiser-Bessel width 12) is checked against the oracle.
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

# problems of the 32-problem draw used here: the two smallest, the largest,
# one of mid size and four more (tuning all 32 belongs to the benchmark)
N_TUNED = 8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cost(p):
    return p.m * p.nt * int(np.prod(p.shape))


@pytest.fixture(scope="module")
def batch_setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_01078_amd.autotune import Autotuner
    from paper_1510_01078_amd.batch import Batch, problem_dict
    draw = inputs.batched_problems(32, seed=1003)
    order = np.argsort([_cost(p) for p in draw])
    pick = [int(order[0]), int(order[1]), int(order[-1]), int(order[len(order) // 2])]
    pick += [int(i) for i in order[3:len(order):6] if int(i) not in pick][:N_TUNED - len(pick)]
    probs = [draw[i] for i in pick]
    _say(f"[gpu] batch of {len(probs)} of the draw: M {[p.m for p in probs]}, Nt {[p.nt for p in probs]}, "
         f"N {[p.shape[0] for p in probs]}")
    tuner = Autotuner(timed_candidates=2, reps=2)
    settings, entries = tuner.tune_batch([problem_dict(p) for p in probs], [p.g for p in probs])
    for p, e in zip(probs, entries):
        s = e["settings"]
        _say(f"[gpu] tuned M={p.m} Nt={p.nt} N={p.shape[0]}: lateral {s['sigma_xy']}/{s['width_xy']}, temporal "
             f"{s['sigma_t']}/{s['width_t']}, error vs FP64 reference {e['rel_err']:.2e}")
    b = Batch([problem_dict(p, **st) for p, st in zip(probs, settings)], precision="fp32")
    gs = [torch.from_numpy(np.ascontiguousarray(p.g)).to("cuda", torch.float32) for p in probs]
    yield probs, b, gs, settings, tuner
    b.close()


def test_tuner_reference_vs_oracle(batch_setup):
    from paper_1510_01078_amd.batch import problem_dict
    probs, b, gs, settings, tuner = batch_setup
    p = min(probs, key=_cost)
    ref = tuner.reference(problem_dict(p), p.g).cpu().numpy()
    e = rel_l2(ref, oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent))
    _say(f"[gpu] tuner reference (FP64, sigma 2, KB w 12) vs oracle: {e:.2e}")
    assert e <= 1e-8


def test_batch_equals_single_plans(batch_setup):
    from paper_1510_01078_amd import Plan
    probs, b, gs, settings, _ = batch_setup
    outs = b.reconstruct(gs)
    torch.cuda.synchronize()
    mismatched = []
    for i, (p, g, o, st) in enumerate(zip(probs, gs, outs, settings)):
        pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32", **st)
        ref = pl.reconstruct(g)
        torch.cuda.synchronize()
        if not torch.equal(ref, o):
            mismatched.append((i, float((ref - o).abs().max())))
        pl.close()
    _say(f"[gpu] batch vs single plans: {len(probs) - len(mismatched)}/{len(probs)} bitwise equal {mismatched}")
    assert not mismatched


def test_batch_vs_oracle(batch_setup):
    """The two smallest problems on the whole image; the largest and the
    mid-size problem on the spectrum of sampled lateral x-modes (the batch's
    images equal the single plans' bit for bit, so the single plan's
    spectrum stands for the batch's)."""
    from paper_1510_01078_amd import Plan
    probs, b, gs, settings, _ = batch_setup
    outs = b.reconstruct(gs)
    torch.cuda.synchronize()
    for i in (0, 1):
        p = probs[i]
        ref = oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent)
        e = rel_l2(outs[i].cpu().numpy().astype(np.float64), ref)
        _say(f"[gpu] batch problem M={p.m}, Nt={p.nt}, N={p.shape[0]} vs oracle (whole image): rel-L2 {e:.3e}")
        assert e <= 1e-5
    for i in (2, 3):
        p = probs[i]
        Nx, Ny, Nz = p.shape
        X, Y, Z = p.extent
        pl = Plan(p.xy, p.nt, p.dt, p.c, p.shape, p.extent, sensor_h=p.h, precision="fp32", **settings[i])
        H = pl.spectrum(gs[i]).cpu().numpy().astype(np.complex128)
        pl.close()
        rows = np.array([1, Nx // 4, Nx // 2 - 1, Nx // 2, Nx // 2 + 3, 3 * Nx // 4, Nx - 1])
        kx, ky, kz = oracle.lattice(Nx, X), oracle.lattice(Ny, Y), oracle.lattice(Nz, Z)
        G = oracle.stage_lateral(p.xy, p.h, p.g, p.dt, Nx, Ny, X, Y, j_index=rows)
        S = oracle.stage_temporal(G, kx[rows], ky, kz, p.c, p.dt)
        F = oracle.apply_weight(S, kx, ky, kz, p.c, j_index=rows)
        lz = np.arange(Nz // 2 + 1)
        ref = np.fft.ifftshift(F, axes=1)[:, :, (lz + Nz // 2) % Nz]
        e = rel_l2(H[(rows - Nx // 2) % Nx], ref)
        _say(f"[gpu] batch problem M={p.m}, Nt={p.nt}, N={Nx} vs oracle (spectrum, {len(rows)} x-modes): {e:.3e}")
        assert e <= 1e-5


def test_batch_grid_shapes_same_bits(batch_setup):
    """Default persistent grid, a small persistent grid and one work-group
    per work item give the same bits."""
    probs, b, gs, _, _ = batch_setup
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
    probs, b, gs, _, _ = batch_setup
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
