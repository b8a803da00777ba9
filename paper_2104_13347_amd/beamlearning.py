"""Thin ctypes binding of the BeamLearning forward pass in libism.so (C-ABI
declared in include/beamlearning.h).

Argument marshalling only: the weight folding, the 18 filterbank layers, the
pseudo-energy and the head all run in the library's HIP kernels.  torch
supplies device memory and streams.  If the library is not built the first use
fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import weakref

import numpy as np

from . import ism

REGRESSION, CLASSIFICATION = 0, 1
NF = 128
MARGIN = 189

EXPORTS = ["bl_param_count", "bl_model_create", "bl_model_destroy", "bl_workspace_bytes", "bl_forward",
           "bl_noalloc_scratch_bytes", "bl_forward_noalloc"]

_ready = False


def load():
    global _ready
    L = ism.load()
    if not _ready:
        vp, ci, sz, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_int64
        L.bl_param_count.argtypes = [ci, ci]
        L.bl_param_count.restype = sz
        L.bl_model_create.argtypes = [vp, ci, ci, ci, ctypes.c_float, vp, vp, ctypes.POINTER(vp)]
        L.bl_model_create.restype = ci
        L.bl_model_destroy.argtypes = [vp]
        L.bl_model_destroy.restype = None
        L.bl_workspace_bytes.argtypes = [ci, ci]
        L.bl_workspace_bytes.restype = sz
        L.bl_forward.argtypes = [vp, vp, ci, ci, vp, vp, i64, i64, vp, sz, vp, vp, vp]
        L.bl_forward.restype = ci
        L.bl_noalloc_scratch_bytes.argtypes = []
        L.bl_noalloc_scratch_bytes.restype = sz
        L.bl_forward_noalloc.argtypes = [vp, vp, ci, ci, vp, vp, i64, i64, vp, vp, vp]
        L.bl_forward_noalloc.restype = ci
        _ready = True
    return L


def param_count(c_in, n_out):
    return int(load().bl_param_count(int(c_in), int(n_out)))


def workspace_bytes(batch, n_t):
    return int(load().bl_workspace_bytes(int(batch), int(n_t)))


class Model:
    """A prepared network (folded FP16-pair weights in device memory).

    params: the flat FP32 parameter array (numpy or a device tensor) in the
    layout of include/beamlearning.h.
    """

    def __init__(self, handle, params, c_in=7, n_out=2, mode=REGRESSION, ln_eps=1e-6, stream=None):
        import torch
        self.lib = load()
        self.handle = handle
        self.c_in, self.n_out, self.mode = int(c_in), int(n_out), int(mode)
        if not torch.is_tensor(params):
            params = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32))
        with ism._on(stream):   # the folding kernel reads the copy on `stream`
            self._params = params.to(device="cuda", dtype=torch.float32).contiguous()
        need = param_count(self.c_in, self.n_out)
        if need == 0 or self._params.numel() != need:
            raise ValueError(f"params hold {self._params.numel()} floats, the layout {need}")
        m = ctypes.c_void_p()
        rc = self.lib.bl_model_create(handle.h, self.c_in, self.n_out, self.mode, float(ln_eps),
                                      ctypes.c_void_p(self._params.data_ptr()), ism._stream_handle(stream),
                                      ctypes.byref(m))
        handle._check(rc)
        self.m = m
        # the folding kernel ran on `stream`; forward passes may use other streams
        torch.cuda.synchronize()

    def close(self):
        if getattr(self, "m", None):
            import torch
            torch.cuda.synchronize()
            self.lib.bl_model_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_extent(self, x, n_t, batch, offsets, ex_stride, ch_stride):
        """Explicit frame layout: every element the kernels read, frame b < batch, channel
        c < c_in, sample n < n_t at off_b + c * ch_stride + n, must lie in x (contiguous).
        Device offsets are read back to check them, once per offsets storage (its base tensor,
        held by a weak reference, so a new tensor that reuses a freed one's memory is read
        again), element offset into it, batch and torch's version counter (shared by a tensor
        and its views, so a fresh slice of the same offsets, offsets[:b] on every call, keeps
        the check); a tensor rewritten outside torch keeps its old check."""
        if n_t is None or batch is None or ch_stride is None:
            raise ValueError("n_t, batch and ch_stride are required with an explicit frame layout")
        if offsets is None and ex_stride is None:
            raise ValueError("either offsets or ex_stride is required with an explicit frame layout")
        batch, n_t, ch_stride = int(batch), int(n_t), int(ch_stride)
        if batch < 0 or n_t < 1 or ch_stride < 0 or (ex_stride is not None and int(ex_stride) < 0):
            raise ValueError("batch, strides and offsets must be non-negative and n_t >= 1")
        if batch == 0:
            return
        if not x.is_contiguous():
            raise ValueError("x must be contiguous with an explicit frame layout (offsets index its storage)")
        span = (self.c_in - 1) * ch_stride + n_t   # elements of one frame from its offset
        if offsets is None:
            hi = (batch - 1) * int(ex_stride) + span
            if hi > x.numel():
                raise ValueError(f"frames reach element {hi} of x, which holds {x.numel()}")
            return
        if offsets.numel() < batch:
            raise ValueError(f"offsets holds {offsets.numel()} entries for {batch} frames")
        base = offsets._base if offsets._base is not None else offsets
        key = (offsets.storage_offset(), offsets._version, batch)
        cache = getattr(self, "_off_range", None)
        if cache is None or cache[0]() is not base or cache[1] != key:
            o = offsets[:batch]
            lo, hi = int(o.min().item()), int(o.max().item())
            self._off_range = cache = (weakref.ref(base), key, lo, hi)
        lo, hi = cache[2], cache[3]
        if lo < 0 or hi + span > x.numel():
            raise ValueError(f"frame offsets in [{lo}, {hi}] reach past the {x.numel()} elements of x")

    def forward(self, x, n_t=None, batch=None, offsets=None, ex_stride=None, ch_stride=None,
                workspace=None, features=True, out=None, stream=None, noalloc=False):
        """Forward pass.  x: device FP32 tensor [B, c_in, n_t] (contiguous), or any
        device FP32 tensor with explicit batch, n_t, offsets (device int64 tensor
        or None), ex_stride and ch_stride in elements.  Returns (features or None, out).
        noalloc=True calls bl_forward_noalloc (the library's fixed workspace; no
        workspace argument)."""
        import torch
        if x.dtype != torch.float32 or not x.is_cuda:
            raise ValueError("x must be a CUDA float32 tensor")
        if offsets is not None and (offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous()):
            raise ValueError("offsets must be a contiguous CUDA int64 tensor")
        if x.dim() == 3 and n_t is None:
            batch, c, n_t = x.shape
            if c != self.c_in:
                raise ValueError(f"x has {c} channels, the model {self.c_in}")
            with ism._on(stream):
                x = x.contiguous()
            ex_stride, ch_stride = c * n_t, n_t
            offsets = None
        else:
            self._check_extent(x, n_t, batch, offsets, ex_stride, ch_stride)
        batch, n_t = int(batch), int(n_t)
        if out is not None and (out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous()
                                or out.numel() < batch * self.n_out):
            raise ValueError(f"out must be a contiguous CUDA float32 tensor of at least {batch} x {self.n_out} "
                             f"elements")
        if noalloc and workspace is not None:
            raise ValueError("the no-allocation form takes no workspace")
        need = workspace_bytes(batch, n_t)
        with ism._on(stream):
            if workspace is None and not noalloc:
                workspace = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
            feat = torch.empty((batch, NF), dtype=torch.float32, device="cuda") if features else None
            if out is None:
                out = torch.empty((batch, self.n_out), dtype=torch.float32, device="cuda")
        if noalloc:
            rc = self.lib.bl_forward_noalloc(self.handle.h, self.m, batch, n_t, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(offsets.data_ptr() if offsets is not None else 0),
                                             int(ex_stride or 0), int(ch_stride or 0),
                                             ctypes.c_void_p(feat.data_ptr() if feat is not None else 0),
                                             ctypes.c_void_p(out.data_ptr()), ism._stream_handle(stream))
            self.handle._check(rc)
            return feat, out
        rc = self.lib.bl_forward(self.handle.h, self.m, batch, n_t, ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(offsets.data_ptr() if offsets is not None else 0),
                                 int(ex_stride or 0), int(ch_stride or 0), ctypes.c_void_p(workspace.data_ptr()),
                                 int(workspace.numel()), ctypes.c_void_p(feat.data_ptr() if feat is not None else 0),
                                 ctypes.c_void_p(out.data_ptr()), ism._stream_handle(stream))
        self.handle._check(rc)
        return feat, out
