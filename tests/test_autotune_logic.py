"""The autotuner's selection logic on the CPU, with plans replaced by a model
whose error and cost depend on the window settings in a known way: settings
beyond the error limit are rejected, refused settings (PAT_ERR_UNSUPPORTED)
are recorded and skipped, the cheapest passing pair is chosen when time
follows cost, nothing passing falls back to the reference setting, and
results are cached per problem in memory and in the JSON file, under a key
that changes with the sensor positions, the sampling step, the speed of sound
and the extent.
The GPU test (tests/test_gpu_autotune.py) runs the same code on real plans.
"""
import json
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1510_01078_amd import autotune as at  # noqa: E402
from paper_1510_01078_amd._native import PAT_ERR_UNSUPPORTED, PatError  # noqa: E402


def _lateral_err(s, w):
    return 0.0 if (s, w) == (2.0, 12) else (1e-7 if w >= 8 else (4e-6 if s == 2.0 else 1e-3))


def _temporal_err(s, w):
    return 0.0 if (s, w) == (2.0, 12) else (2e-7 if w >= 8 else 1e-3)


class FakePlan:
    made = 0
    floor = 0.0  # error added to every working-precision setting (not to the FP64 reference)

    def __init__(self, precision, settings, refuse):
        FakePlan.made += 1
        key = (settings["sigma_xy"], settings["width_xy"], settings["sigma_t"], settings["width_t"])
        if key in refuse:
            raise PatError(PAT_ERR_UNSUPPORTED, "refused")
        self.settings = settings
        self.precision = precision
        self.shape = (4, 4, 4)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cpu")
        n = int(round(settings["sigma_xy"] * 32))
        self.info = dict(nx_over=n, ny_over=n, band_bins=int(round(settings["sigma_t"] * 40)))

    def reconstruct(self, g, out=None):
        s = self.settings
        e = _lateral_err(s["sigma_xy"], s["width_xy"]) + _temporal_err(s["sigma_t"], s["width_t"])
        if self.precision != "fp64":
            e += FakePlan.floor
        ref = torch.arange(1, 65, dtype=torch.float64).reshape(self.shape)
        # time grows with the grid points, the band bins and the two widths (about 2 ms for the cheapest pair)
        time.sleep(1.5e-9 * self.info["nx_over"] ** 2 * self.info["band_bins"] * (s["width_xy"] + s["width_t"]))
        r = (ref * (1.0 + e)).to(self.dtype)
        if out is not None:
            out.copy_(r)
            return out
        return r

    def close(self):
        pass


@pytest.fixture
def cpu_tuner(monkeypatch):
    monkeypatch.setattr(torch.Tensor, "cuda", lambda self, *a, **k: self, raising=False)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    refuse = set()

    def make(self, p, precision, settings, kernel=None):
        return FakePlan(precision, settings, refuse)

    monkeypatch.setattr(at.Autotuner, "_plan", make)
    FakePlan.made = 0
    FakePlan.floor = 0.0
    return refuse


def _problem():
    xy = np.zeros((6, 2))
    return dict(sensor_xy=xy, n_t=16, dt=1e-8, c=1500.0, shape=(4, 4, 4), extent=(1e-3, 1e-3, 1e-3))


def test_cheapest_passing_pair_is_chosen(cpu_tuner):
    t = at.Autotuner(target=1e-5, margin=0.5, timed_candidates=3, reps=1)
    best = t.tune(_problem(), np.zeros((6, 16)))
    s = best["settings"]
    # lateral passes for w >= 8 (any sigma) or w = 6 at sigma 2; temporal for w >= 8:
    # the cheapest pair by grid points x band bins is sigma 1.25 on both axes, w = 8
    assert (s["sigma_xy"], s["width_xy"], s["sigma_t"], s["width_t"]) == (1.25, 8, 1.25, 8)
    assert best["rel_err"] <= 0.5e-5
    tried = {(d["settings"]["sigma_xy"], d["settings"]["width_xy"], d["settings"]["sigma_t"],
              d["settings"]["width_t"]): d["rel_err"] for d in best["tried"]}
    assert tried[(1.25, 6, 2.0, 12)] > 0.5e-5      # screened and rejected
    assert tried[(2.0, 12, 1.25, 6)] > 0.5e-5


def test_refused_settings_are_recorded_and_skipped(cpu_tuner):
    cpu_tuner.add((1.25, 8, 2.0, 12))                 # the plan refuses this lateral screen
    t = at.Autotuner(target=1e-5, timed_candidates=3, reps=1)
    best = t.tune(_problem(), np.zeros((6, 16)))
    refused = [d for d in best["tried"] if d["settings"]["sigma_xy"] == 1.25 and d["settings"]["width_xy"] == 8
               and d["settings"]["sigma_t"] == 2.0]
    assert refused and refused[0]["rel_err"] == float("inf")
    assert (best["settings"]["sigma_xy"], best["settings"]["width_xy"]) != (1.25, 8)


def test_nothing_passing_falls_back_to_reference(cpu_tuner):
    FakePlan.floor = 1e-6  # every candidate, the reference setting included, misses half of 1e-6
    t = at.Autotuner(target=1e-6, timed_candidates=3, reps=1)
    best = t.tune(_problem(), np.zeros((6, 16)))
    assert best["settings"] == at.REFERENCE and best["ms"] is None


def test_cache_in_memory_and_file(cpu_tuner, tmp_path):
    path = tmp_path / "tune.json"
    t = at.Autotuner(target=1e-5, timed_candidates=2, reps=1, cache_path=str(path))
    first = t.tune(_problem(), np.zeros((6, 16)))
    made = FakePlan.made
    again = t.tune(_problem(), np.zeros((6, 16)))
    assert again is first and FakePlan.made == made  # served from memory, no plan built
    stored = json.loads(path.read_text())
    assert t.key(_problem()) in stored
    t2 = at.Autotuner(target=1e-5, cache_path=str(path))
    assert t2.tune(_problem(), np.zeros((6, 16)))["settings"] == first["settings"]
    assert FakePlan.made == made                     # served from the file


def test_key_separates_problems_of_one_shape():
    base = _problem()
    k0 = at.problem_key(base, "fp32", "kaiser_bessel", 1e-5)
    moved = dict(base, sensor_xy=base["sensor_xy"] + 1e-6)
    for other in (moved, dict(base, dt=2e-8), dict(base, c=1540.0), dict(base, extent=(2e-3, 1e-3, 1e-3)),
                  dict(base, sensor_h=np.ones(6))):
        assert at.problem_key(other, "fp32", "kaiser_bessel", 1e-5) != k0
    assert at.problem_key(base, "fp32", "gaussian", 1e-5) != k0
    assert at.problem_key(base, "fp32", "kaiser_bessel", 1e-6) != k0
    assert at.problem_key(dict(base), "fp32", "kaiser_bessel", 1e-5) == k0
