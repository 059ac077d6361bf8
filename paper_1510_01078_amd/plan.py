"""Python binding of the NEDNER-NUFFT library (argument marshalling only).

Every step of the reconstruction runs in the HIP kernels of libpatnufft.so;
this module only builds the plan descriptor, hands PyTorch device memory to
the library (the plan's tables through an allocator callback, the workspace
and outputs as tensors) and passes torch's current HIP stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N

_KERNELS = {"gaussian": N.PAT_KERNEL_GAUSSIAN, "kaiser_bessel": N.PAT_KERNEL_KAISER_BESSEL,
            "kb": N.PAT_KERNEL_KAISER_BESSEL}
_PRECISIONS = {"fp64": N.PAT_FP64, "fp32": N.PAT_FP32, "fp32_kahan": N.PAT_FP32_KAHAN}


def build_desc(sensor_xy, n_t, dt, c, shape, extent, sensor_h=None, sigma_xy=2.0, width_xy=8, sigma_t=2.0,
               width_t=8, kernel="kaiser_bessel", precision="fp32", temporal_interp="window"):
    """A pat_plan_desc for one problem and the host arrays it points to
    (keep them alive until the plan is built)."""
    lib = N.load()
    xy = np.ascontiguousarray(sensor_xy, dtype=np.float64).reshape(-1, 2)
    h = None if sensor_h is None else np.ascontiguousarray(sensor_h, dtype=np.float64).reshape(-1)
    if h is not None and h.shape[0] != xy.shape[0]:
        raise ValueError("sensor_h must have one entry per sensor")
    d = N.PlanDesc()
    N.check(lib.pat_plan_desc_init(C.byref(d)), "pat_plan_desc_init")
    d.n_sensors = xy.shape[0]
    d.n_t = int(n_t)
    d.dt = float(dt)
    d.c = float(c)
    d.sensor_xy = xy.ctypes.data_as(C.POINTER(C.c_double))
    d.sensor_h = h.ctypes.data_as(C.POINTER(C.c_double)) if h is not None else None
    d.nx, d.ny, d.nz = (int(v) for v in shape)
    d.lx, d.ly, d.lz = (float(v) for v in extent)
    d.sigma_xy = float(sigma_xy)
    d.width_xy = int(width_xy)
    d.sigma_t = float(sigma_t)
    d.width_t = int(width_t)
    d.kernel = _KERNELS[kernel]
    d.precision = _PRECISIONS[precision]
    d.temporal_interp = {"window": N.PAT_INTERP_WINDOW, "linear": N.PAT_INTERP_LINEAR}[temporal_interp]
    return d, (xy, h)


def torch_allocator(device, blocks):
    """Allocator callbacks handing torch's caching allocator to the library:
    each block is a uint8 tensor kept in `blocks` (keyed by address) until freed."""
    import torch

    def _alloc(nbytes, ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
            p = t.data_ptr()
            blocks[p] = t
            return p
        except Exception:  # allocation failure -> NULL -> PAT_ERR_ALLOC
            return None

    def _free(ptr, ctx):
        blocks.pop(ptr, None)

    return N.ALLOC_FN(_alloc), N.FREE_FN(_free)


class Plan:
    """A reconstruction plan for one sensor geometry, trace length and grid.

    Parameters mirror pat_plan_desc: sensor_xy [M,2] (metres, plane-centred),
    sensor_h [M] (m^2, None for X*Y/M), n_t, dt, c, shape (Nx,Ny,Nz),
    extent (X,Y,Z), lateral/temporal oversampling and window widths, window
    kernel ('kaiser_bessel' or 'gaussian'), precision ('fp32',
    'fp32_kahan' or 'fp64') and temporal interpolation ('window': the
    NER-NUFFT; 'linear': the zero-padded FFT with linear interpolation that
    the paper compares against). The plan lives on `device` (default: the
    current CUDA/HIP device) and uses torch's current stream there. With
    workspace=False the plan allocates no workspace tensor (for callers that
    only use reconstruct_noalloc or pass their own workspace).
    """

    def __init__(self, sensor_xy, n_t, dt, c, shape, extent, sensor_h=None, sigma_xy=2.0, width_xy=8,
                 sigma_t=2.0, width_t=8, kernel="kaiser_bessel", precision="fp32", device=None,
                 temporal_interp="window", workspace=True):
        import torch

        self._torch = torch
        self._lib = N.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("Plan needs a GPU device")
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.m = int(np.asarray(sensor_xy).reshape(-1, 2).shape[0])
        self.n_t = int(n_t)
        self.shape = tuple(int(s) for s in shape)
        self.extent = tuple(float(e) for e in extent)
        d, keep = build_desc(sensor_xy, n_t, dt, c, shape, extent, sensor_h, sigma_xy, width_xy, sigma_t, width_t,
                             kernel, precision, temporal_interp)
        self._xy, self._h = keep

        self._blocks = {}
        self._alloc_cb, self._free_cb = torch_allocator(self.device, self._blocks)
        d.alloc = self._alloc_cb
        d.free = self._free_cb
        self._desc = d
        handle = C.c_void_p()
        dev = self.device
        with torch.cuda.device(dev):
            stream = torch.cuda.current_stream(dev)
            N.check(self._lib.nufft_plan(C.byref(d), C.c_void_p(stream.cuda_stream), C.byref(handle)), "nufft_plan")
        self._handle = handle
        info = N.PlanInfo()
        N.check(self._lib.pat_plan_get_info(handle, C.byref(info)), "pat_plan_get_info")
        self.info = {f: getattr(info, f) for f, _ in N.PlanInfo._fields_ if not f.startswith("pad")}
        self.workspace = (torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=dev)
                          if workspace else None)

    # ------------------------------------------------------------------
    def _stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def _check_traces(self, g):
        torch = self._torch
        if not isinstance(g, torch.Tensor) or g.device != self.device:
            raise ValueError(f"traces must be a tensor on {self.device}")
        if g.dtype != self.dtype or tuple(g.shape) != (self.m, self.n_t) or not g.is_contiguous():
            raise ValueError(f"traces must be contiguous {self.dtype} of shape {(self.m, self.n_t)}")

    def _check_image(self, f):
        torch = self._torch
        if not isinstance(f, torch.Tensor) or f.device != self.device:
            raise ValueError(f"image must be a tensor on {self.device}")
        if f.dtype != self.dtype or tuple(f.shape) != self.shape or not f.is_contiguous():
            raise ValueError(f"image must be contiguous {self.dtype} of shape {self.shape}")

    def _out(self, out, shape, dtype):
        if out is None:
            return self._torch.empty(shape, dtype=dtype, device=self.device)
        if (out.dtype != dtype or tuple(out.shape) != tuple(shape) or not out.is_contiguous()
                or out.device != self.device):
            raise ValueError(f"output must be contiguous {dtype} of shape {tuple(shape)} on {self.device}")
        return out

    def _ws(self, workspace):
        ws = self.workspace if workspace is None else workspace
        if ws is None:
            raise ValueError("the plan was built without a workspace: pass one")
        if ws.device != self.device or ws.numel() * ws.element_size() < self.info["workspace_bytes"]:
            raise ValueError("workspace too small or on another device")
        return ws

    def reconstruct(self, g, out=None, workspace=None):
        """f = R g (pat_reconstruct). g: [M, Nt] device tensor. Returns [Nx,Ny,Nz]."""
        self._check_handle()
        self._check_traces(g)
        out = self._out(out, self.shape, self.dtype)
        ws = self._ws(workspace)
        N.check(self._lib.pat_reconstruct(self._handle, C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()),
                                          C.c_void_p(ws.data_ptr()), self._stream()), "pat_reconstruct")
        return out

    def reconstruct_noalloc(self, g, out):
        """f = R g (pat_reconstruct_noalloc) into the caller's `out` with the
        library's fixed scratch as workspace: nothing is allocated. Raises
        PatError (PAT_ERR_WORKSPACE_TOO_LARGE) when the plan's workspace
        exceeds the scratch. Calls overlapping in time on one GPU race."""
        self._check_handle()
        self._check_traces(g)
        if out is None:
            raise ValueError("reconstruct_noalloc writes into a caller-provided output")
        out = self._out(out, self.shape, self.dtype)
        N.check(self._lib.pat_reconstruct_noalloc(self._handle, C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()),
                                                  self._stream()), "pat_reconstruct_noalloc")
        return out

    def spectrum(self, g, out=None, workspace=None):
        """F(K) half spectrum [Nx, Ny, Nz/2+1] complex (pat_spectrum)."""
        self._check_handle()
        self._check_traces(g)
        shp = (self.shape[0], self.shape[1], self.shape[2] // 2 + 1)
        out = self._out(out, shp, self.cdtype)
        ws = self._ws(workspace)
        N.check(self._lib.pat_spectrum(self._handle, C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(ws.data_ptr()), self._stream()), "pat_spectrum")
        return out

    def forward(self, f, out=None, workspace=None):
        """g = A f (pat_forward): image [Nx,Ny,Nz] -> traces [M, Nt]."""
        self._check_handle()
        self._check_image(f)
        out = self._out(out, (self.m, self.n_t), self.dtype)
        ws = self._ws(workspace)
        N.check(self._lib.pat_forward(self._handle, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()),
                                      C.c_void_p(ws.data_ptr()), self._stream()), "pat_forward")
        return out

    def adjoint(self, g, out=None, workspace=None):
        """f = A* g (pat_adjoint): traces [M, Nt] -> image [Nx,Ny,Nz]."""
        self._check_handle()
        self._check_traces(g)
        out = self._out(out, self.shape, self.dtype)
        ws = self._ws(workspace)
        N.check(self._lib.pat_adjoint(self._handle, C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()),
                                      C.c_void_p(ws.data_ptr()), self._stream()), "pat_adjoint")
        return out

    def forward_dxy(self, f, axis, out=None, workspace=None):
        """d(A f)/d(x_m) (axis 0) or d(A f)/d(y_m) (axis 1) per trace (pat_forward_dxy)."""
        self._check_handle()
        self._check_image(f)
        out = self._out(out, (self.m, self.n_t), self.dtype)
        ws = self._ws(workspace)
        N.check(self._lib.pat_forward_dxy(self._handle, C.c_void_p(f.data_ptr()), int(axis),
                                          C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), self._stream()),
                "pat_forward_dxy")
        return out

    @property
    def sensor_xy(self):
        """The sensor positions the plan was built for (host copy, [M, 2])."""
        return self._xy.copy()

    def timing_begin(self, max_calls: int, stages=None):
        """Per-stage event timing of the next max_calls compute calls; `stages`
        (stage indices) limits the events to those stages' ends
        (pat_timing_begin_stages), None times every stage."""
        self._check_handle()
        if stages is None:
            N.check(self._lib.pat_timing_begin(self._handle, int(max_calls)), "pat_timing_begin")
        else:
            mask = 0
            for st in stages:
                mask |= 1 << int(st)
            N.check(self._lib.pat_timing_begin_stages(self._handle, int(max_calls), mask),
                    "pat_timing_begin_stages")

    def timing_end(self):
        """Returns (per-stage summed milliseconds [6], number of calls recorded)."""
        self._check_handle()
        ms = (C.c_double * N.PAT_TIMING_STAGES)()
        calls = C.c_int32()
        N.check(self._lib.pat_timing_end(self._handle, ms, N.PAT_TIMING_STAGES, C.byref(calls)), "pat_timing_end")
        return list(ms), calls.value

    def _check_handle(self):
        if self._handle is None:
            raise RuntimeError("plan is closed")

    def close(self):
        if getattr(self, "_handle", None) is not None:
            self._lib.nufft_plan_destroy(self._handle)
            self._handle = None
            self._blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
