"""Python binding of the batched reconstruction (argument marshalling only).

A Batch holds up to 64 independent problems (own sensors, trace length,
grid and window settings; one precision) and reconstructs all of them with
one launch per stage (pat_batch_reconstruct).
"""
from __future__ import annotations

import ctypes as C

from . import _native as N
from .plan import build_desc, torch_allocator

_SETTINGS = ("sigma_xy", "width_xy", "sigma_t", "width_t", "kernel", "temporal_interp")


class Batch:
    """problems: sequence of dicts with keys sensor_xy, n_t, dt, c, shape,
    extent and optionally sensor_h and the window settings (sigma_xy,
    width_xy, sigma_t, width_t, kernel, temporal_interp); `defaults` fills
    settings a problem leaves out. precision applies to the whole batch;
    group_bytes is the cache budget of a group of problems (0: the
    library's default; a huge value: one group)."""

    def __init__(self, problems, precision="fp32", device=None, defaults=None, group_bytes=0):
        import torch

        self._torch = torch
        self._lib = N.load()
        problems = list(problems)
        if not 1 <= len(problems) <= N.PAT_BATCH_MAX:
            raise ValueError(f"a batch holds 1..{N.PAT_BATCH_MAX} problems")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self._blocks = {}
        self._alloc_cb, self._free_cb = torch_allocator(self.device, self._blocks)
        base = dict(sigma_xy=2.0, width_xy=8, sigma_t=2.0, width_t=8, kernel="kaiser_bessel",
                    temporal_interp="window")
        base.update(defaults or {})
        descs = (N.PlanDesc * len(problems))()
        keep = []
        self.shapes, self.traces = [], []
        for i, pr in enumerate(problems):
            kw = {k: pr.get(k, base[k]) for k in _SETTINGS}
            d, arrays = build_desc(pr["sensor_xy"], pr["n_t"], pr["dt"], pr["c"], pr["shape"], pr["extent"],
                                   pr.get("sensor_h"), precision=precision, **kw)
            d.alloc = self._alloc_cb
            d.free = self._free_cb
            descs[i] = d
            keep.append(arrays)
            self.shapes.append(tuple(int(s) for s in pr["shape"]))
            self.traces.append((int(arrays[0].shape[0]), int(pr["n_t"])))
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            N.check(self._lib.pat_batch_create(descs, len(problems), int(group_bytes),
                                               C.c_void_p(stream.cuda_stream), C.byref(handle)), "pat_batch_create")
        self._handle = handle
        self.count = len(problems)
        ng = C.c_int32()
        N.check(self._lib.pat_batch_groups(handle, C.byref(ng)), "pat_batch_groups")
        self.groups = ng.value
        self.info = []
        for i in range(self.count):
            plan = C.c_void_p()
            N.check(self._lib.pat_batch_get_plan(handle, i, C.byref(plan)), "pat_batch_get_plan")
            info = N.PlanInfo()
            N.check(self._lib.pat_plan_get_info(plan, C.byref(info)), "pat_plan_get_info")
            self.info.append({f: getattr(info, f) for f, _ in N.PlanInfo._fields_})

    def set_grid(self, blocks: int):
        """0: one work-group per work item; > 0: a persistent grid of that many."""
        N.check(self._lib.pat_batch_set_grid(self._handle, int(blocks)), "pat_batch_set_grid")

    def reconstruct(self, traces, outs=None):
        """traces: list of [M_p, Nt_p] device tensors; returns list of images."""
        torch = self._torch
        if self._handle is None:
            raise RuntimeError("batch is closed")
        if len(traces) != self.count:
            raise ValueError(f"expected {self.count} trace tensors")
        if outs is None:
            outs = [torch.empty(s, dtype=self.dtype, device=self.device) for s in self.shapes]
        for g, (m, nt), o, s in zip(traces, self.traces, outs, self.shapes):
            if g.device != self.device or g.dtype != self.dtype or tuple(g.shape) != (m, nt) or not g.is_contiguous():
                raise ValueError(f"traces must be contiguous {self.dtype} [{m}, {nt}] on {self.device}")
            if o.device != self.device or o.dtype != self.dtype or tuple(o.shape) != s or not o.is_contiguous():
                raise ValueError(f"outputs must be contiguous {self.dtype} {s} on {self.device}")
        gp = (C.c_void_p * self.count)(*[g.data_ptr() for g in traces])
        fp = (C.c_void_p * self.count)(*[o.data_ptr() for o in outs])
        stream = C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        N.check(self._lib.pat_batch_reconstruct(self._handle, gp, fp, stream), "pat_batch_reconstruct")
        return outs

    def close(self):
        if getattr(self, "_handle", None) is not None:
            self._lib.pat_batch_destroy(self._handle)
            self._handle = None
            self._blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def problem_dict(p, **settings):
    """Batch entry from an inputs.Problem (plus optional window settings)."""
    d = dict(sensor_xy=p.xy, sensor_h=p.h, n_t=p.nt, dt=p.dt, c=p.c, shape=p.shape, extent=p.extent)
    d.update(settings)
    return d


__all__ = ["Batch", "problem_dict"]
