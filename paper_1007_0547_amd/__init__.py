"""Python binding of the gfx950 hierarchical slope-intercept Hough vote.

A thin ctypes layer over ``libhough_hier.so`` (C ABI in
``include/hough_hier.h``): it marshals arguments and results, nothing else.
Every step of the vote runs in the library's HIP kernels.  PyTorch is used
only to hand over device memory (``torch.Tensor.data_ptr()``) and streams.

Importing this package requires the built library; build it with
``python paper_1007_0547_amd/_build.py``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

__all__ = ["HoughHier", "Result", "HHError", "CELL_DTYPE", "STATS_DTYPE", "LIB_PATH",
           "status_name", "library"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhough_hier.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python paper_1007_0547_amd/_build.py)")

# PyTorch ships its own copy of the HIP runtime (same soname).  Loading torch
# first lets the library bind to that copy: two HIP runtimes in one process
# cannot both open the GPU.
try:
    import torch as _torch  # noqa: F401
except ImportError:
    _torch = None

_lib = C.CDLL(LIB_PATH)

STATUS = {1: "HH_PENDING", 0: "HH_OK", -1: "HH_EINVAL", -2: "HH_ENOMEM", -3: "HH_ECAPACITY", -4: "HH_EDEVICE",
          -5: "HH_EBUSY", -6: "HH_ECANCELED", -7: "HH_EINTERNAL"}
INT32_MIN = -(1 << 31)


def status_name(s: int) -> str:
    return STATUS.get(int(s), str(s))


class HHError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{status_name(status)}: {msg}" if msg else status_name(status))
        self.status = int(status)


class _Config(C.Structure):
    _fields_ = [("threshold", C.c_int32), ("max_depth", C.c_int32), ("passes", C.c_uint32),
                ("variant", C.c_int32), ("membership", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p), ("flags", C.c_int32), ("arena_limit_mib", C.c_int32),
                ("arena_hint", C.c_uint64), ("arena", C.c_void_p), ("arena_bytes", C.c_uint64),
                ("hbm_budget_bytes", C.c_uint64)]


class _Input(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("on_device", C.c_int32), ("x", C.c_void_p), ("y", C.c_void_p),
                ("n_points", C.c_int64), ("image", C.c_void_p), ("row_stride", C.c_int64),
                ("threshold", C.c_int32), ("max_depth", C.c_int32), ("edge_threshold", C.c_int32),
                ("reserved", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("width", C.c_int32), ("height", C.c_int32),
                ("side_pow2", C.c_int32), ("depth", C.c_int32), ("threshold", C.c_int32),
                ("passes", C.c_uint32), ("n_cells", C.c_int64 * 2), ("code_tests", C.c_int64),
                ("member_slots", C.c_int64), ("compare_bits", C.c_int32), ("reserved", C.c_int32)]


class _Timing(C.Structure):
    _fields_ = [("vote_launches", C.c_int32), ("decide_launches", C.c_int32),
                ("vote_ms", C.c_double), ("decide_ms", C.c_double), ("extract_ms", C.c_double),
                ("total_ms", C.c_double), ("vote_entries", C.c_int64), ("vote_written", C.c_int64),
                ("count_ms", C.c_double), ("write_ms", C.c_double), ("groups", C.c_int32),
                ("resumes", C.c_int32), ("queue_ms", C.c_double), ("service_ms", C.c_double),
                ("graph_replayed", C.c_int32), ("reserved", C.c_int32)]


class _ServeConfig(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("max_batch", C.c_int32), ("max_batch_pixels", C.c_int64),
                ("queue_capacity", C.c_int32), ("reserved", C.c_int32)]


class _ServeStats(C.Structure):
    _fields_ = [("slab_bytes", C.c_int64), ("slab_used", C.c_int64), ("slab_batches", C.c_int64),
                ("outside_batches", C.c_int64), ("retries", C.c_int64), ("pending", C.c_int64),
                ("bytes_per_unit", C.c_double), ("internal_reruns", C.c_int64),
                ("internal_failures", C.c_int64), ("first_internal_error", C.c_char * 512)]


class _Launch(C.Structure):
    _fields_ = [("task_steps", C.c_int32), ("queue_batch", C.c_int32), ("wg_per_cu", C.c_int32),
                ("reserved", C.c_int32)]


class _Solution(C.Structure):
    _fields_ = [("keep", C.c_void_p), ("n_cells", C.c_int64), ("plotted", C.c_void_p), ("n_points", C.c_int64),
                ("kept", C.c_int64), ("plotted_points", C.c_int64),
                ("rounds", C.c_int64)]


CELL_DTYPE = np.dtype([("i", np.int32), ("j", np.int32), ("votes", np.int32), ("pass", np.int32),
                       ("key", np.int64), ("member_off", np.int64)])
STATS_DTYPE = np.dtype([("evaluated", np.int64), ("votes", np.int64), ("split", np.int64),
                        ("detected", np.int64), ("code_tests", np.int64), ("entries", np.int64)])
assert CELL_DTYPE.itemsize == 32 and STATS_DTYPE.itemsize == 48

MAX_DEPTH = 15          # HH_MAX_DEPTH
NOALLOC_SCRATCH_BYTES = 256 << 20   # HH_NOALLOC_SCRATCH_BYTES
_p = C.c_void_p
_lib.hough_hier_create.restype = C.c_int
_lib.hough_hier_create.argtypes = [C.POINTER(_Config), C.POINTER(_p)]
_lib.hough_hier_destroy.restype = None
_lib.hough_hier_destroy.argtypes = [_p]
_lib.hough_hier_last_error.restype = C.c_char_p
_lib.hough_hier_last_error.argtypes = [_p]
_lib.hough_hier_detect.restype = C.c_int
_lib.hough_hier_detect.argtypes = [_p, C.POINTER(_Input), C.POINTER(_p)]
_lib.hough_hier_detect_batch.restype = C.c_int
_lib.hough_hier_detect_batch.argtypes = [_p, C.POINTER(_Input), C.c_int32, C.POINTER(_p)]
_lib.hough_hier_serve_start.restype = C.c_int
_lib.hough_hier_serve_start.argtypes = [_p, C.POINTER(_ServeConfig)]
_lib.hough_hier_serve_stats.restype = C.c_int
_lib.hough_hier_serve_stats.argtypes = [_p, C.POINTER(_ServeStats)]
_lib.hough_hier_submit.restype = C.c_int
_lib.hough_hier_submit.argtypes = [_p, C.POINTER(_Input), C.POINTER(C.c_uint64)]
_lib.hough_hier_poll.restype = C.c_int
_lib.hough_hier_poll.argtypes = [_p, C.c_uint64, C.c_int32, C.POINTER(_p)]
_lib.hough_hier_result_cells.restype = C.c_int
_lib.hough_hier_result_cells.argtypes = [_p, C.c_int32, C.c_int32, C.POINTER(_p), C.POINTER(C.c_int64)]
_lib.hough_hier_result_members.restype = C.c_int
_lib.hough_hier_result_members.argtypes = [_p, C.c_int32, C.POINTER(_p), C.POINTER(C.c_int64)]
_lib.hough_hier_result_member_points.restype = C.c_int
_lib.hough_hier_result_member_points.argtypes = [_p, C.POINTER(_p), C.POINTER(C.c_int64),
                                                 C.POINTER(C.c_int32)]
_lib.hough_hier_result_stats.restype = C.c_int
_lib.hough_hier_result_stats.argtypes = [_p, C.c_int32, C.POINTER(_p), C.POINTER(C.c_int32)]
_lib.hough_hier_result_info.restype = C.c_int
_lib.hough_hier_result_info.argtypes = [_p, C.POINTER(_Info)]
_lib.hough_hier_result_timing.restype = C.c_int
_lib.hough_hier_result_timing.argtypes = [_p, C.POINTER(_Timing)]
_lib.hough_hier_solution.restype = C.c_int
_lib.hough_hier_solution.argtypes = [C.POINTER(_p), C.c_int32, C.POINTER(C.c_double)]
_lib.hough_hier_result_solution.restype = C.c_int
_lib.hough_hier_result_solution.argtypes = [_p, C.c_int32, C.c_int32, C.POINTER(_Solution)]
_lib.hough_hier_result_solution_image.restype = C.c_int
_lib.hough_hier_result_solution_image.argtypes = [_p, C.c_void_p, C.c_int64, C.c_int32]
_lib.hough_hier_set_launch.restype = C.c_int
_lib.hough_hier_set_launch.argtypes = [_p, C.POINTER(_Launch)]
_lib.hough_hier_autotune.restype = C.c_int
_lib.hough_hier_autotune.argtypes = [_p, C.POINTER(_Input), C.c_int32, C.POINTER(_Launch), C.POINTER(C.c_int32)]
_lib.hough_hier_get_launch.restype = C.c_int
_lib.hough_hier_get_launch.argtypes = [_p, C.POINTER(_Launch)]
_lib.hough_hier_detect_noalloc.restype = C.c_int
_lib.hough_hier_detect_noalloc.argtypes = [_p, C.POINTER(_Input), C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
_lib.hough_hier_result_last_error.restype = C.c_char_p
_lib.hough_hier_result_last_error.argtypes = [_p]
_lib.hough_hier_result_free.restype = None
_lib.hough_hier_result_free.argtypes = [_p]


def library() -> C.CDLL:
    """The loaded ``libhough_hier.so``."""
    return _lib


def _is_torch_cuda(t) -> bool:
    return hasattr(t, "is_cuda") and bool(t.is_cuda)


def _host_array(a, dtype) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Result:
    """A detection result; owns device memory until :meth:`free`."""

    def __init__(self, ctx: "HoughHier", handle: int):
        self._ctx = ctx
        self._h = C.c_void_p(handle)
        inf = _Info()
        self._check(_lib.hough_hier_result_info(self._h, C.byref(inf)))
        self.info = {k: (list(getattr(inf, k)) if k == "n_cells" else getattr(inf, k))
                     for k, _ in _Info._fields_ if k != "reserved"}

    def _check(self, s):
        if s != 0:
            raise HHError(s, (_lib.hough_hier_result_last_error(self._h) or b"").decode())

    def timing(self) -> dict:
        """Kernel timings of the call (contexts created with ``timing=True``)."""
        t = _Timing()
        self._check(_lib.hough_hier_result_timing(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _Timing._fields_}

    def cells(self, pass_: int) -> np.ndarray:
        """Host copy of one pass's cells (structured array, ``CELL_DTYPE``);
        ``member_off`` indexes :meth:`members`."""
        ptr, n = C.c_void_p(), C.c_int64()
        self._check(_lib.hough_hier_result_cells(self._h, pass_, 0, C.byref(ptr), C.byref(n)))
        if n.value == 0:
            return np.zeros(0, dtype=CELL_DTYPE)
        buf = (C.c_char * (n.value * CELL_DTYPE.itemsize)).from_address(ptr.value)
        return np.frombuffer(buf, dtype=CELL_DTYPE).copy()

    def device_cells(self, pass_: int):
        """``(device_pointer, count)`` of one pass's cells on the device."""
        ptr, n = C.c_void_p(), C.c_int64()
        self._check(_lib.hough_hier_result_cells(self._h, pass_, 1, C.byref(ptr), C.byref(n)))
        return (ptr.value or 0), n.value

    def members(self) -> np.ndarray:
        """Host copy of all voters, compact, cells in (pass, key) order."""
        ptr, n = C.c_void_p(), C.c_int64()
        self._check(_lib.hough_hier_result_members(self._h, 0, C.byref(ptr), C.byref(n)))
        if n.value == 0:
            return np.zeros(0, dtype=np.int32)
        buf = (C.c_int32 * n.value).from_address(ptr.value)
        return np.frombuffer(buf, dtype=np.int32).copy()

    def device_members(self):
        """``(device_pointer, slots)`` of the device voter buffer."""
        ptr, n = C.c_void_p(), C.c_int64()
        self._check(_lib.hough_hier_result_members(self._h, 1, C.byref(ptr), C.byref(n)))
        return (ptr.value or 0), n.value

    def member_points(self):
        """``(device_pointer, entries, entry_bytes)`` of the voter entries as
        the kernels left them (``hough_hier_result_member_points``)."""
        ptr, n, eb = C.c_void_p(), C.c_int64(), C.c_int32()
        self._check(_lib.hough_hier_result_member_points(self._h, C.byref(ptr), C.byref(n), C.byref(eb)))
        return (ptr.value or 0), n.value, eb.value

    def stats(self, pass_: int) -> np.ndarray:
        """Per-level statistics (``STATS_DTYPE``), level 0 first."""
        ptr, n = C.c_void_p(), C.c_int32()
        self._check(_lib.hough_hier_result_stats(self._h, pass_, C.byref(ptr), C.byref(n)))
        if n.value == 0:
            return np.zeros(0, dtype=STATS_DTYPE)
        buf = (C.c_char * (n.value * STATS_DTYPE.itemsize)).from_address(ptr.value)
        return np.frombuffer(buf, dtype=STATS_DTYPE).copy()

    def stats_array(self, pass_: int) -> np.ndarray:
        """Statistics as an int64 array of shape (depth + 1, 6)."""
        s = self.stats(pass_)
        return s.view(np.int64).reshape(len(s), 6) if len(s) else np.zeros((0, 6), np.int64)

    def solution(self, pass_: int) -> dict:
        """Outcome of :func:`solution` for one pass, host copies: ``keep``
        (bool per cell of :meth:`cells`), ``plotted`` (bool per point id),
        ``kept`` and ``plotted_points``."""
        out = _Solution()
        self._check(_lib.hough_hier_result_solution(self._h, pass_, 0, C.byref(out)))
        keep = np.zeros(out.n_cells, dtype=bool)
        plotted = np.zeros(out.n_points, dtype=bool)
        if out.n_cells:
            keep = np.frombuffer((C.c_uint8 * out.n_cells).from_address(out.keep), dtype=np.uint8).astype(bool)
        if out.n_points and out.plotted:
            plotted = np.frombuffer((C.c_uint8 * out.n_points).from_address(out.plotted),
                                    dtype=np.uint8).astype(bool)
        return {"keep": keep, "plotted": plotted, "kept": out.kept, "plotted_points": out.plotted_points,
                "rounds": out.rounds}

    def solution_image(self, out=None) -> np.ndarray:
        """The output image of :func:`solution` (255 at plotted points of any
        pass, else 0), ``height x width`` uint8.  ``out`` may be a torch
        device tensor or a numpy array of that shape (rows may be strided);
        by default a new numpy array is returned."""
        H, W = self.info["height"], self.info["width"]
        if out is None:
            out = np.empty((H, W), dtype=np.uint8)
        if _is_torch_cuda(out):
            assert tuple(out.shape) == (H, W) and out.stride(1) == 1
            self._check(_lib.hough_hier_result_solution_image(self._h, C.c_void_p(out.data_ptr()),
                                                              out.stride(0), 1))
        else:
            assert out.shape == (H, W) and out.dtype == np.uint8 and out.strides[1] == 1
            self._check(_lib.hough_hier_result_solution_image(self._h, out.ctypes.data, out.strides[0], 0))
        return out

    def device_solution(self, pass_: int) -> dict:
        """Device pointers of one pass's keep and plotted flags and the counts."""
        out = _Solution()
        self._check(_lib.hough_hier_result_solution(self._h, pass_, 1, C.byref(out)))
        return {k: (getattr(out, k) or 0) for k, _ in _Solution._fields_}

    def free(self):
        if self._h:
            _lib.hough_hier_result_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if self._ctx._h:
                self.free()
        except Exception:
            pass


class HoughHier:
    """A context on one gfx950 device (``hough_hier_create``)."""

    def __init__(self, threshold: int = 0, max_depth: int = 0, passes: int = 3,
                 variant: str = "code", membership: bool = True, device: int = 0,
                 stream=None, wide_compare: bool = False, timing: bool = False,
                 arena_hint: int = 0, arena_limit_mib: int = 0, arena=None, hbm_budget_bytes: int = 0,
                 graph: bool = False):
        cfg = _Config()
        cfg.threshold = int(threshold)
        cfg.max_depth = int(max_depth)
        cfg.passes = int(passes)
        cfg.variant = {"code": 0, "circle": 1}[variant]
        cfg.membership = 1 if membership else 0
        cfg.device = int(device)
        cfg.stream = self._stream_handle(stream)
        cfg.flags = (1 if wide_compare else 0) | (2 if timing else 0) | (4 if graph else 0)
        cfg.arena_hint = int(arena_hint)
        cfg.arena_limit_mib = int(arena_limit_mib)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        if arena is not None:   # a torch device tensor: its memory backs every call
            assert _is_torch_cuda(arena) and arena.is_contiguous()
            cfg.arena = arena.data_ptr()
            cfg.arena_bytes = arena.numel() * arena.element_size()
            self._arena = arena   # kept alive with the context
        h = C.c_void_p()
        s = _lib.hough_hier_create(C.byref(cfg), C.byref(h))
        if s != 0:
            raise HHError(s, "hough_hier_create failed")
        self._h = h

    @staticmethod
    def _stream_handle(stream) -> Optional[int]:
        if stream is None:
            return None
        if isinstance(stream, int):
            return stream
        return int(stream.cuda_stream)   # torch.cuda.Stream

    def set_launch(self, task_steps: int = 0, queue_batch: int = 0, wg_per_cu: int = 0):
        """Launch shape of the list kernels (``hough_hier_set_launch``)."""
        ln = _Launch(int(task_steps), int(queue_batch), int(wg_per_cu), 0)
        s = _lib.hough_hier_set_launch(self._h, C.byref(ln))
        if s != 0:
            raise HHError(s, self.last_error())

    def autotune(self, inputs) -> dict:
        """``hough_hier_autotune`` for calls like ``inputs`` (a list of
        ``detect`` keyword dicts): the launch shape chosen (and set on the
        context), and whether it came from the cache."""
        arr = (_Input * len(inputs))()
        keep = []
        for k, kw in enumerate(inputs):
            inp, kp = self._input(**kw)
            arr[k] = inp
            keep.append(kp)
        ln = _Launch()
        cached = C.c_int32()
        s = _lib.hough_hier_autotune(self._h, arr, len(inputs), C.byref(ln), C.byref(cached))
        del keep
        if s != 0:
            raise HHError(s, self.last_error())
        out = {k: getattr(ln, k) for k, _ in _Launch._fields_ if k != "reserved"}
        out["from_cache"] = bool(cached.value)
        return out

    def launch(self) -> dict:
        """The current launch shape (``hough_hier_get_launch``)."""
        ln = _Launch()
        s = _lib.hough_hier_get_launch(self._h, C.byref(ln))
        if s != 0:
            raise HHError(s, self.last_error())
        return {k: getattr(ln, k) for k, _ in _Launch._fields_ if k != "reserved"}

    def last_error(self) -> str:
        if not self._h:
            return ""
        return (_lib.hough_hier_last_error(self._h) or b"").decode()

    @staticmethod
    def _input(x=None, y=None, *, image=None, gray=None, edge_threshold: int = 0, width: int, height: int,
               threshold: int = -1, max_depth: Optional[int] = None):
        """An ``hh_input`` and the objects that must outlive the call."""
        inp = _Input()
        inp.width, inp.height = int(width), int(height)
        inp.threshold = int(threshold)
        inp.max_depth = INT32_MIN if max_depth is None else int(max_depth)
        keep = []
        if gray is not None:   # gray image through the Sobel front end
            image = gray
            inp.edge_threshold = int(edge_threshold)
        if image is not None:
            inp.kind = 2 if gray is not None else 1
            if _is_torch_cuda(image):
                assert image.dtype.itemsize == 1 and image.dim() == 2
                inp.on_device = 1
                inp.image = image.data_ptr()
                inp.row_stride = int(image.stride(0))
                keep.append(image)
            else:
                img = _host_array(image, np.uint8)
                inp.on_device = 0
                inp.image = img.ctypes.data
                inp.row_stride = int(img.strides[0])
                keep.append(img)
        else:
            inp.kind = 0
            if _is_torch_cuda(x):
                assert x.is_contiguous() and y.is_contiguous()
                assert str(x.dtype) == "torch.int32" and str(y.dtype) == "torch.int32"
                inp.on_device = 1
                inp.x, inp.y = x.data_ptr(), y.data_ptr()
                inp.n_points = int(x.numel())
                keep += [x, y]
            else:
                hx, hy = _host_array(x, np.int32), _host_array(y, np.int32)
                if hx.shape != hy.shape:
                    raise ValueError("x and y must have the same length")
                inp.on_device = 0
                inp.x, inp.y = hx.ctypes.data, hy.ctypes.data
                inp.n_points = int(hx.size)
                keep += [hx, hy]
        return inp, keep

    def detect(self, x=None, y=None, *, image=None, gray=None, edge_threshold: int = 0, width: int,
               height: int, threshold: int = -1, max_depth: Optional[int] = None) -> Result:
        """Run the vote on a point list ``(x, y)``, a binary ``image`` (H x W,
        nonzero = edge) or a ``gray`` image through the Sobel front end (edge
        points by gradient magnitude, pass 0 / pass 1 by gradient direction).
        Torch device tensors are passed as device pointers; anything else is
        copied from host memory."""
        inp, keep = self._input(x, y, image=image, gray=gray, edge_threshold=edge_threshold, width=width,
                                height=height, threshold=threshold, max_depth=max_depth)
        out = C.c_void_p()
        s = _lib.hough_hier_detect(self._h, C.byref(inp), C.byref(out))
        del keep
        if s != 0:
            raise HHError(s, self.last_error())
        return Result(self, out.value)

    def detect_noalloc(self, x=None, y=None, *, image=None, gray=None, edge_threshold: int = 0, width: int,
                       height: int, threshold: int = -1, max_depth: Optional[int] = None, cells_out,
                       members_out=None) -> dict:
        """``hough_hier_detect_noalloc``: one detection in the library's fixed
        device scratch, cells and voter ids written to the caller's torch
        device tensors ``cells_out`` (uint8, 32 bytes per cell) and
        ``members_out`` (int32).  Returns the counts and the statistics."""
        assert _is_torch_cuda(cells_out) and cells_out.is_contiguous()
        inp, keep = self._input(x, y, image=image, gray=gray, edge_threshold=edge_threshold, width=width,
                                height=height, threshold=threshold, max_depth=max_depth)
        nst = 2 * (MAX_DEPTH + 1)
        stats = np.zeros(nst * 6, dtype=np.int64)
        n_cells = (C.c_int64 * 2)()
        n_members = C.c_int64()
        mptr, mcap = None, 0
        if members_out is not None:
            assert _is_torch_cuda(members_out) and members_out.is_contiguous()
            mptr, mcap = members_out.data_ptr(), members_out.numel()
        s = _lib.hough_hier_detect_noalloc(self._h, C.byref(inp), C.c_void_p(cells_out.data_ptr()),
                                           cells_out.numel() * cells_out.element_size() // CELL_DTYPE.itemsize,
                                           mptr, mcap, stats.ctypes.data, n_cells, C.byref(n_members))
        del keep
        if s != 0:
            raise HHError(s, self.last_error())
        st = stats.reshape(2, MAX_DEPTH + 1, 6)
        return {"n_cells": [n_cells[0], n_cells[1]], "n_members": n_members.value,
                "stats": {p: st[p] for p in (0, 1)}}

    def detect_batch(self, inputs) -> list:
        """Run the vote on several inputs of one kind in one call
        (``hough_hier_detect_batch``).  ``inputs`` holds dicts with the
        keyword arguments of :meth:`detect`; the results come in input
        order."""
        n = len(inputs)
        arr = (_Input * n)()
        keep = []
        for k, d in enumerate(inputs):
            inp, kp = self._input(**d)
            arr[k] = inp
            keep += kp
        out = (C.c_void_p * n)()
        s = _lib.hough_hier_detect_batch(self._h, arr, n, out)
        del keep
        if s != 0:
            raise HHError(s, self.last_error())
        return [Result(self, out[k]) for k in range(n)]

    def solution(self, results) -> float:
        """solution() with point removal (``hough_hier_solution``) on the
        device for the given results; returns the walk's kernel time in ms.
        Read the outcome with :meth:`Result.solution`."""
        return solution(results)

    # ---- serving (continuous batching)

    def serve_start(self, lanes: int = 0, max_batch: int = 0, max_batch_pixels: int = 0,
                    queue_capacity: int = 0):
        """Start the serving lanes (``hough_hier_serve_start``)."""
        cfg = _ServeConfig()
        cfg.lanes, cfg.max_batch = int(lanes), int(max_batch)
        cfg.max_batch_pixels, cfg.queue_capacity = int(max_batch_pixels), int(queue_capacity)
        s = _lib.hough_hier_serve_start(self._h, C.byref(cfg))
        if s != 0:
            raise HHError(s, self.last_error())
        self._inflight = {}

    def serve_stats(self) -> dict:
        """Serving counters (``hough_hier_serve_stats``): the slab's size and
        use, batches run inside and outside it, reruns in a larger interval,
        waiting requests, the footprint model's bytes per unit, and batches
        whose internal consistency check failed (rerun, failed again, the
        first failure's text)."""
        st = _ServeStats()
        s = _lib.hough_hier_serve_stats(self._h, C.byref(st))
        if s != 0:
            raise HHError(s, self.last_error())
        out = {k: getattr(st, k) for k, _ in _ServeStats._fields_}
        out["first_internal_error"] = st.first_internal_error.decode(errors="replace")
        return out

    def submit(self, x=None, y=None, *, image=None, gray=None, edge_threshold: int = 0, width: int,
               height: int, threshold: int = -1, max_depth: Optional[int] = None) -> int:
        """Queue one input (``hough_hier_submit``, the arguments of
        :meth:`detect`); returns its ticket.  The input objects are kept alive
        until the ticket is polled."""
        inp, keep = self._input(x, y, image=image, gray=gray, edge_threshold=edge_threshold, width=width,
                                height=height, threshold=threshold, max_depth=max_depth)
        t = C.c_uint64()
        s = _lib.hough_hier_submit(self._h, C.byref(inp), C.byref(t))
        if s != 0:
            raise HHError(s, self.last_error())
        self._inflight[t.value] = keep
        return t.value

    def poll(self, ticket: int, wait_us: int = -1) -> Optional[Result]:
        """The result of a ticket, or ``None`` while it is pending
        (``hough_hier_poll``)."""
        out = C.c_void_p()
        s = _lib.hough_hier_poll(self._h, int(ticket), int(wait_us), C.byref(out))
        if s == 1:
            return None
        self._inflight.pop(int(ticket), None)
        if s != 0:
            raise HHError(s, self.last_error())
        return Result(self, out.value)

    def close(self):
        if self._h:
            _lib.hough_hier_destroy(self._h)
            self._h = C.c_void_p()
        self._arena = None   # a caller arena is released with the context

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solution(results) -> float:
    """solution() with point removal (Sec. 3) for a list of results (or one):
    per pass, a detected cell is kept iff more than T of its voters were not
    plotted by an earlier kept cell in key order; kept cells plot their
    voters.  Returns the summed kernel time of the walk in ms."""
    if isinstance(results, Result):
        results = [results]
    n = len(results)
    arr = (C.c_void_p * max(n, 1))()
    for k, r in enumerate(results):
        arr[k] = r._h
    ms = C.c_double()
    s = _lib.hough_hier_solution(arr, n, C.byref(ms))
    if s != 0:
        msg = results[0]._ctx.last_error() if n else ""
        raise HHError(s, msg)
    return ms.value
