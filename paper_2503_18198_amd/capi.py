"""ctypes binding of the C ABI in ``include/mttkrp.h`` (argument marshalling only).

Every function has the C name.  Device buffers are passed as ``torch.Tensor``
objects on the current HIP device (only their pointers are used) and streams
as ``torch.cuda.Stream`` objects or raw ``hipStream_t`` integers; host
buffers are numpy arrays.  All computation happens in the HIP library; if it
is not built, importing this module raises instead of falling back.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MTTKRP_HIP_LIB") or os.path.join(_HERE, "libmttkrp_hip.so")

MTTKRP_OK, MTTKRP_EINVAL, MTTKRP_ERANGE, MTTKRP_ENOMEM, MTTKRP_EUNSUPPORTED, MTTKRP_ENOTSPD, MTTKRP_EHIP = range(7)
MTTKRP_FP32, MTTKRP_BF16 = 0, 1
MTTKRP_PART_NNZ, MTTKRP_PART_ROWS_LPT = 0, 1
MTTKRP_MAX_MODES = 8
STATUS_NAMES = {0: "MTTKRP_OK", 1: "MTTKRP_EINVAL", 2: "MTTKRP_ERANGE", 3: "MTTKRP_ENOMEM",
                4: "MTTKRP_EUNSUPPORTED", 5: "MTTKRP_ENOTSPD", 6: "MTTKRP_EHIP"}

# Every symbol the header declares.
EXPORTED = ["mttkrp_opts_default", "mttkrp_footprint", "mttkrp_layout_build", "mttkrp_layout_bytes", "mttkrp_run",
            "mttkrp_run_bf16", "cpd_als_init", "cpd_als_iter", "mttkrp_layout_free", "mttkrp_last_error",
            "mttkrp_layout_view", "mttkrp_layout_info", "mttkrp_batch_create", "mttkrp_batch_run",
            "mttkrp_batch_free", "cpd_als_iter_async", "cpd_als_status", "cpd_als_batch_iter_async",
            "mttkrp_gather_probe", "mttkrp_batch_autotune", "mttkrp_run_scheme2", "mttkrp_launch_plan",
            "mttkrp_build_scratch_bytes", "mttkrp_layout_build_in", "mttkrp_batch_bytes", "mttkrp_batch_create_in",
            "mttkrp_run_noalloc", "mttkrp_noalloc_scratch_bytes", "mttkrp_lpt_partition", "mttkrp_batch_run_bf16",
            "mttkrp_batch_autotune_shape", "mttkrp_batch_autotune_default_shapes", "mttkrp_autotune_shape",
            "mttkrp_layout_perm"]


class MttkrpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class mttkrp_opts(ctypes.Structure):
    _fields_ = [("parts_per_cu", ctypes.c_int), ("factor_dtype", ctypes.c_int), ("max_R", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_uint64), ("host_only", ctypes.c_int), ("hot_rows", ctypes.c_int),
                ("build_on_host", ctypes.c_int), ("partitioner", ctypes.c_int), ("lpt_parts", ctypes.c_int),
                ("hot_steps", ctypes.c_int), ("wide_indices", ctypes.c_int), ("part_threads", ctypes.c_int),
                ("part_gathers", ctypes.c_int), ("relabel", ctypes.c_int), ("als_solve", ctypes.c_int)]


class mttkrp_mode_view(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_uint64), ("nnz_pad", ctypes.c_uint64), ("nrows_nz", ctypes.c_uint64),
                ("nempty", ctypes.c_uint64), ("n_in", ctypes.c_int),
                ("in_modes", ctypes.c_int * (MTTKRP_MAX_MODES - 1)),
                ("idx", ctypes.POINTER(ctypes.c_uint32) * (MTTKRP_MAX_MODES - 1)),
                ("val", ctypes.POINTER(ctypes.c_float)), ("winfo", ctypes.POINTER(ctypes.c_uint32)),
                ("row_id", ctypes.POINTER(ctypes.c_uint32)), ("empty_rows", ctypes.POINTER(ctypes.c_uint32)),
                ("src_pos", ctypes.POINTER(ctypes.c_uint64)), ("nhot", ctypes.c_uint64),
                ("hot_rows", ctypes.POINTER(ctypes.c_uint32) * (MTTKRP_MAX_MODES - 1)),
                ("step_entries", ctypes.c_uint64), ("nsteps", ctypes.c_uint64),
                ("nparts", ctypes.c_uint64), ("part_range", ctypes.POINTER(ctypes.c_uint64))]


class mttkrp_info(ctypes.Structure):
    _fields_ = [("cu_count", ctypes.c_uint32), ("lds_per_workgroup", ctypes.c_uint32), ("hot_rows", ctypes.c_uint32),
                ("wg_threads", ctypes.c_uint32), ("parts_per_cu", ctypes.c_uint32), ("lpt_parts", ctypes.c_uint32),
                ("step_entries", ctypes.c_uint32), ("idx16_modes", ctypes.c_uint32),
                ("gathers_in_flight", ctypes.c_uint32)]


class mttkrp_part_shape(ctypes.Structure):
    _fields_ = [("parts_per_cu", ctypes.c_int), ("threads", ctypes.c_int), ("gathers", ctypes.c_int)]


class mttkrp_plan(ctypes.Structure):
    _fields_ = [("wg_threads", ctypes.c_uint32), ("lane_groups", ctypes.c_uint32),
                ("lanes_per_group", ctypes.c_uint32), ("nonzeros_per_group", ctypes.c_uint32),
                ("nonzeros_per_part", ctypes.c_uint64), ("nparts", ctypes.c_uint32), ("carry_bytes", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2503_18198_amd.build.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32p, f32p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)
    lib.mttkrp_opts_default.argtypes = [ctypes.POINTER(mttkrp_opts)]
    lib.mttkrp_opts_default.restype = None
    lib.mttkrp_footprint.argtypes = [u32p, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(mttkrp_opts),
                                     ctypes.POINTER(ctypes.c_uint64)]
    lib.mttkrp_layout_build.argtypes = [u32p, f32p, ctypes.c_uint64, u32p, ctypes.c_int, ctypes.POINTER(mttkrp_opts),
                                        vp, ctypes.POINTER(vp)]
    lib.mttkrp_layout_bytes.argtypes = [vp]
    lib.mttkrp_layout_bytes.restype = ctypes.c_uint64
    lib.mttkrp_run.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), vp, ctypes.c_int, vp]
    lib.mttkrp_run_bf16.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), vp, ctypes.c_int, vp]
    lib.mttkrp_run_scheme2.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), vp, ctypes.c_int, vp]
    lib.mttkrp_run_noalloc.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), vp, ctypes.c_int, vp]
    lib.mttkrp_lpt_partition.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)]
    lib.mttkrp_noalloc_scratch_bytes.argtypes = []
    lib.mttkrp_noalloc_scratch_bytes.restype = ctypes.c_uint64
    lib.cpd_als_init.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.cpd_als_iter.argtypes = [vp, ctypes.POINTER(vp), vp, ctypes.c_int, vp, vp]
    lib.mttkrp_layout_free.argtypes = [vp]
    lib.mttkrp_layout_free.restype = None
    lib.mttkrp_last_error.argtypes = []
    lib.mttkrp_last_error.restype = ctypes.c_char_p
    lib.mttkrp_layout_view.argtypes = [vp, ctypes.c_int, ctypes.POINTER(mttkrp_mode_view)]
    lib.mttkrp_layout_info.argtypes = [vp, ctypes.POINTER(mttkrp_info)]
    lib.mttkrp_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(mttkrp_opts),
                                        ctypes.POINTER(vp)]
    lib.mttkrp_batch_run.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.mttkrp_batch_run_bf16.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.cpd_als_iter_async.argtypes = [vp, ctypes.POINTER(vp), vp, ctypes.c_int, vp, vp]
    lib.cpd_als_status.argtypes = [vp, vp]
    lib.mttkrp_batch_autotune.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp,
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
    lib.mttkrp_batch_autotune_shape.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(mttkrp_part_shape), ctypes.c_int, ctypes.POINTER(vp),
                                                ctypes.POINTER(vp), ctypes.c_int, vp,
                                                ctypes.POINTER(mttkrp_part_shape), ctypes.POINTER(ctypes.c_float)]
    lib.mttkrp_autotune_shape.argtypes = [vp, ctypes.c_int, ctypes.POINTER(mttkrp_part_shape), ctypes.c_int,
                                          ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp,
                                          ctypes.POINTER(mttkrp_part_shape), ctypes.POINTER(ctypes.c_float)]
    lib.mttkrp_layout_perm.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]
    lib.mttkrp_batch_autotune_default_shapes.argtypes = [ctypes.c_int, ctypes.POINTER(mttkrp_part_shape)]
    lib.mttkrp_batch_autotune_default_shapes.restype = ctypes.c_int
    lib.mttkrp_gather_probe.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    lib.cpd_als_batch_iter_async.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.mttkrp_batch_free.argtypes = [vp]
    lib.mttkrp_batch_free.restype = None
    lib.mttkrp_launch_plan.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint32, ctypes.POINTER(mttkrp_plan)]
    lib.mttkrp_build_scratch_bytes.argtypes = [u32p, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(mttkrp_opts),
                                               ctypes.POINTER(ctypes.c_uint64)]
    lib.mttkrp_layout_build_in.argtypes = [u32p, f32p, ctypes.c_uint64, u32p, ctypes.c_int,
                                           ctypes.POINTER(mttkrp_opts), vp, ctypes.c_uint64, vp, ctypes.c_uint64,
                                           vp, ctypes.POINTER(vp)]
    lib.mttkrp_batch_bytes.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
    lib.mttkrp_batch_create_in.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(mttkrp_opts), vp, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
    for name in ("mttkrp_footprint", "mttkrp_layout_build", "mttkrp_run", "mttkrp_run_bf16", "cpd_als_init",
                 "cpd_als_iter", "mttkrp_layout_view", "mttkrp_layout_info", "mttkrp_batch_create",
                 "mttkrp_batch_run", "cpd_als_iter_async", "cpd_als_status", "cpd_als_batch_iter_async",
                 "mttkrp_gather_probe", "mttkrp_batch_autotune", "mttkrp_run_scheme2", "mttkrp_launch_plan",
                 "mttkrp_build_scratch_bytes", "mttkrp_layout_build_in", "mttkrp_batch_bytes",
                 "mttkrp_batch_create_in", "mttkrp_run_noalloc", "mttkrp_lpt_partition", "mttkrp_batch_run_bf16",
                 "mttkrp_batch_autotune_shape", "mttkrp_autotune_shape", "mttkrp_layout_perm"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()


def _check(status: int):
    if status != MTTKRP_OK:
        raise MttkrpError(status, _lib.mttkrp_last_error().decode(errors="replace"))


def mttkrp_last_error() -> str:
    return _lib.mttkrp_last_error().decode(errors="replace")


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) if torch.cuda.is_available() else 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def mttkrp_opts_default(**overrides) -> mttkrp_opts:
    o = mttkrp_opts()
    _lib.mttkrp_opts_default(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def _opts(opts) -> Optional[mttkrp_opts]:
    if opts is None or isinstance(opts, mttkrp_opts):
        return opts
    return mttkrp_opts_default(**opts)


def _dims(dims) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(dims, dtype=np.uint32))


def mttkrp_footprint(dims: Sequence[int], nnz: int, opts=None) -> int:
    d = _dims(dims)
    out = ctypes.c_uint64()
    o = _opts(opts)
    _check(_lib.mttkrp_footprint(d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), d.shape[0], int(nnz),
                                 ctypes.byref(o) if o is not None else None, ctypes.byref(out)))
    return int(out.value)


class Layout:
    """Owns an ``mttkrp_handle``; released by ``mttkrp_layout_free`` or on collection."""

    def __init__(self, ptr: int, dims, nnz: int, host_only: bool, dev_mem=None):
        self._ptr = ptr
        self.dims = tuple(int(x) for x in dims)
        self.nnz = int(nnz)
        self.host_only = host_only
        self.dev_mem = dev_mem      # caller-owned device memory the handle borrows (mttkrp_layout_build_in)

    @property
    def ptr(self) -> int:
        if not self._ptr:
            raise MttkrpError(MTTKRP_EINVAL, "layout already freed")
        return self._ptr

    def free(self):
        if self._ptr:
            _lib.mttkrp_layout_free(ctypes.c_void_p(self._ptr))
            self._ptr = 0
        self.dev_mem = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mttkrp_layout_build(idx: np.ndarray, vals: np.ndarray, dims: Sequence[int], opts=None, stream=None) -> Layout:
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.float32).reshape(-1)
    d = _dims(dims)
    if idx.ndim != 2 or idx.shape[1] != d.shape[0] or idx.shape[0] != vals.shape[0]:
        raise MttkrpError(MTTKRP_EINVAL, "idx must be (nnz, N) with N = len(dims) and len(vals) = nnz")
    o = _opts(opts)
    host_only = bool(o.host_only) if o is not None else False
    h = ctypes.c_void_p()
    _check(_lib.mttkrp_layout_build(idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    vals.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), idx.shape[0],
                                    d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), d.shape[0],
                                    ctypes.byref(o) if o is not None else None,
                                    ctypes.c_void_p(0 if host_only else _stream(stream)), ctypes.byref(h)))
    return Layout(h.value, dims, idx.shape[0], host_only)


def mttkrp_build_scratch_bytes(dims: Sequence[int], nnz: int, opts=None) -> int:
    d = _dims(dims)
    out = ctypes.c_uint64()
    o = _opts(opts)
    _check(_lib.mttkrp_build_scratch_bytes(d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), d.shape[0], int(nnz),
                                           ctypes.byref(o) if o is not None else None, ctypes.byref(out)))
    return int(out.value)


def mttkrp_layout_build_in(idx: np.ndarray, vals: np.ndarray, dims: Sequence[int], dev_mem, dev_scratch=None,
                           opts=None, stream=None) -> Layout:
    """Build into caller-owned device memory: ``dev_mem`` (a uint8 device
    tensor of at least ``mttkrp_footprint`` bytes) is kept by the returned
    layout until it is freed; ``dev_scratch`` (``mttkrp_build_scratch_bytes``,
    or None for a host build) is used during the call only."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.float32).reshape(-1)
    d = _dims(dims)
    if idx.ndim != 2 or idx.shape[1] != d.shape[0] or idx.shape[0] != vals.shape[0]:
        raise MttkrpError(MTTKRP_EINVAL, "idx must be (nnz, N) with N = len(dims) and len(vals) = nnz")
    o = _opts(opts)
    h = ctypes.c_void_p()
    nb = lambda t: 0 if t is None else int(t.numel() * t.element_size())
    _check(_lib.mttkrp_layout_build_in(idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                       vals.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), idx.shape[0],
                                       d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), d.shape[0],
                                       ctypes.byref(o) if o is not None else None,
                                       ctypes.c_void_p(int(dev_mem.data_ptr())), nb(dev_mem),
                                       ctypes.c_void_p(0 if dev_scratch is None else int(dev_scratch.data_ptr())),
                                       nb(dev_scratch), ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
    return Layout(h.value, dims, idx.shape[0], False, dev_mem=dev_mem)


def mttkrp_layout_bytes(h: Layout) -> int:
    return int(_lib.mttkrp_layout_bytes(ctypes.c_void_p(h.ptr)))


def mttkrp_layout_info(h: Layout) -> dict:
    i = mttkrp_info()
    _check(_lib.mttkrp_layout_info(ctypes.c_void_p(h.ptr), ctypes.byref(i)))
    return {k: int(getattr(i, k)) for k, _ in mttkrp_info._fields_}


def mttkrp_layout_perm(h: Layout, mode: int) -> np.ndarray:
    """For a layout built with relabel=1: the new index of each original index
    of ``mode`` (uint32 array of length I_mode)."""
    if not 0 <= int(mode) < len(h.dims):
        raise MttkrpError(MTTKRP_EINVAL, f"mode {mode} out of range")
    out = np.zeros(int(h.dims[mode]), dtype=np.uint32)
    _check(_lib.mttkrp_layout_perm(ctypes.c_void_p(h.ptr), int(mode), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return out


def mttkrp_launch_plan(nnz: int, N: int, R: int, factor_dtype: int = MTTKRP_FP32, parts_per_cu: int = 0,
                       cu_count: int = 0) -> dict:
    p = mttkrp_plan()
    _check(_lib.mttkrp_launch_plan(int(nnz), int(N), int(R), int(factor_dtype), int(parts_per_cu), int(cu_count),
                                   ctypes.byref(p)))
    return {k: int(getattr(p, k)) for k, _ in mttkrp_plan._fields_}


def mttkrp_layout_free(h: Layout):
    h.free()


def _ptr_array(tensors, n):
    arr = (ctypes.c_void_p * n)()
    for m, t in enumerate(tensors):
        arr[m] = None if t is None else int(t.data_ptr())
    return arr


def _check_factor(t, rows, R, dtype_name, what):
    import torch
    want = torch.float32 if dtype_name == "fp32" else torch.bfloat16
    if t.dtype != want or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (rows, R):
        raise MttkrpError(MTTKRP_EINVAL, f"{what} must be a contiguous {want} device tensor of shape ({rows}, {R})")


def mttkrp_run(h: Layout, mode: int, factors, out, R: Optional[int] = None, stream=None):
    """out <- MTTKRP of the layout along ``mode`` with fp32 ``factors`` (list of N
    device tensors; the entry at ``mode`` may be None)."""
    _run(_lib.mttkrp_run, "fp32", h, mode, factors, out, R, stream)


def mttkrp_run_noalloc(h: Layout, mode: int, factors, out, R: Optional[int] = None, stream=None):
    """As mttkrp_run, with the carry rows in the library's fixed per-device
    scratch array: allocates nothing.  Calls that overlap on one device race."""
    _run(_lib.mttkrp_run_noalloc, "fp32", h, mode, factors, out, R, stream)


def mttkrp_noalloc_scratch_bytes() -> int:
    """Bytes of the fixed per-device scratch array mttkrp_run_noalloc uses."""
    return int(_lib.mttkrp_noalloc_scratch_bytes())


def mttkrp_run_scheme2(h: Layout, mode: int, factors, out, R: Optional[int] = None, stream=None):
    """For comparison: the MTTKRP with the paper's scheme 2 (global atomics for
    rows cut by partition boundaries) instead of the deterministic fix-up."""
    _run(_lib.mttkrp_run_scheme2, "fp32", h, mode, factors, out, R, stream)


def mttkrp_run_bf16(h: Layout, mode: int, factors, out, R: Optional[int] = None, stream=None):
    """As mttkrp_run, with bfloat16 factor tensors."""
    _run(_lib.mttkrp_run_bf16, "bf16", h, mode, factors, out, R, stream)


def mttkrp_gather_probe(h: Layout, mode: int, factors, R: int, what: int = 1, stream=None):
    """Measurement aid: the stream (what=0), stream and row gathers (what=1),
    the same gather instructions with one lane per row reading (what=2) or
    with L1-resident rows (what=3), of the MTTKRP along ``mode`` without its
    arithmetic or stores.  ``factors`` are fp32 or bfloat16 device tensors
    (all the same dtype)."""
    import torch
    N = len(h.dims)
    if not 0 <= int(mode) < N:
        raise MttkrpError(MTTKRP_EINVAL, f"mode {mode} out of range for a {N}-mode tensor")
    if len(factors) != N:
        raise MttkrpError(MTTKRP_EINVAL, f"need {N} factors (entry {mode} may be None)")
    dts = {f.dtype for m, f in enumerate(factors) if m != mode}
    if len(dts) != 1 or next(iter(dts)) not in (torch.float32, torch.bfloat16):
        raise MttkrpError(MTTKRP_EINVAL, "factors must all be float32 or all bfloat16")
    dt = "fp32" if next(iter(dts)) == torch.float32 else "bf16"
    for m, f in enumerate(factors):
        if m != mode:
            _check_factor(f, h.dims[m], R, dt, f"factor {m}")
    _check(_lib.mttkrp_gather_probe(ctypes.c_void_p(h.ptr), int(mode), _ptr_array(factors, N),
                                    MTTKRP_FP32 if dt == "fp32" else MTTKRP_BF16, int(R), int(what),
                                    ctypes.c_void_p(_stream(stream))))


def _run(fn, dt, h, mode, factors, out, R, stream):
    import torch
    N = len(h.dims)
    if not 0 <= int(mode) < N:
        raise MttkrpError(MTTKRP_EINVAL, f"mode {mode} out of range for a {N}-mode tensor")
    if len(factors) != N:
        raise MttkrpError(MTTKRP_EINVAL, f"need {N} factors (entry {mode} may be None)")
    if R is None:
        R = int(out.shape[1])
    for m, f in enumerate(factors):
        if m != mode:
            _check_factor(f, h.dims[m], R, dt, f"factor {m}")
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or tuple(out.shape) != (h.dims[mode], R):
        raise MttkrpError(MTTKRP_EINVAL, f"out must be a contiguous float32 device tensor of shape ({h.dims[mode]}, {R})")
    _check(fn(ctypes.c_void_p(h.ptr), int(mode), _ptr_array(factors, N), ctypes.c_void_p(out.data_ptr()), int(R),
              ctypes.c_void_p(_stream(stream))))


def cpd_als_init(h: Layout, factors, R: int, stream=None):
    N = len(h.dims)
    for m, f in enumerate(factors):
        _check_factor(f, h.dims[m], R, "fp32", f"factor {m}")
    _check(_lib.cpd_als_init(ctypes.c_void_p(h.ptr), _ptr_array(factors, N), int(R), ctypes.c_void_p(_stream(stream))))


def cpd_als_iter(h: Layout, factors, lam, R: int, fit_out=None, stream=None):
    import torch
    N = len(h.dims)
    for m, f in enumerate(factors):
        _check_factor(f, h.dims[m], R, "fp32", f"factor {m}")
    if lam.dtype != torch.float64 or not lam.is_cuda or lam.numel() < R:
        raise MttkrpError(MTTKRP_EINVAL, "lambda must be a float64 device tensor with R entries")
    if fit_out is not None and (fit_out.dtype != torch.float64 or not fit_out.is_cuda):
        raise MttkrpError(MTTKRP_EINVAL, "fit_out must be a float64 device tensor")
    _check(_lib.cpd_als_iter(ctypes.c_void_p(h.ptr), _ptr_array(factors, N), ctypes.c_void_p(lam.data_ptr()), int(R),
                             ctypes.c_void_p(fit_out.data_ptr() if fit_out is not None else 0),
                             ctypes.c_void_p(_stream(stream))))


def cpd_als_iter_async(h: Layout, factors, lam, R: int, fit_out=None, stream=None):
    """One CP-ALS sweep, enqueued only (capturable into a HIP graph)."""
    import torch
    N = len(h.dims)
    for m, f in enumerate(factors):
        _check_factor(f, h.dims[m], R, "fp32", f"factor {m}")
    if lam.dtype != torch.float64 or not lam.is_cuda or lam.numel() < R:
        raise MttkrpError(MTTKRP_EINVAL, "lambda must be a float64 device tensor with R entries")
    _check(_lib.cpd_als_iter_async(ctypes.c_void_p(h.ptr), _ptr_array(factors, N), ctypes.c_void_p(lam.data_ptr()),
                                   int(R), ctypes.c_void_p(fit_out.data_ptr() if fit_out is not None else 0),
                                   ctypes.c_void_p(_stream(stream))))


def cpd_als_status(h: Layout, stream=None):
    _check(_lib.cpd_als_status(ctypes.c_void_p(h.ptr), ctypes.c_void_p(_stream(stream))))


def mttkrp_lpt_partition(loads, kappa: int):
    """Scheme 1's partitioner (host): returns (partition of each row, load of
    each partition)."""
    ld = np.ascontiguousarray(np.asarray(loads, dtype=np.uint64))
    part = np.zeros(ld.shape[0], dtype=np.uint32)
    pl = np.zeros(int(kappa), dtype=np.uint64)
    _check(_lib.mttkrp_lpt_partition(ld.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ld.shape[0], int(kappa),
                                     part.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                     pl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return part, pl


def mttkrp_layout_view(h: Layout, mode: int) -> dict:
    """Copies of the host arrays of one mode copy (host-only layouts)."""
    v = mttkrp_mode_view()
    _check(_lib.mttkrp_layout_view(ctypes.c_void_p(h.ptr), int(mode), ctypes.byref(v)))

    def arr(p, n, dt):
        if n == 0:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(p, shape=(int(n),)).astype(dt, copy=True)

    return dict(nnz=int(v.nnz), nnz_pad=int(v.nnz_pad), nrows_nz=int(v.nrows_nz), nempty=int(v.nempty),
                in_modes=[int(v.in_modes[j]) for j in range(v.n_in)],
                idx=[arr(v.idx[j], v.nnz_pad, np.uint32) for j in range(v.n_in)],
                val=arr(v.val, v.nnz_pad, np.float32),
                winfo=arr(v.winfo, 2 * ((v.nnz_pad // v.step_entries if v.step_entries else v.nnz_pad) // 32), np.uint32),
                row_id=arr(v.row_id, v.nrows_nz, np.uint32), empty_rows=arr(v.empty_rows, v.nempty, np.uint32),
                src_pos=arr(v.src_pos, 0 if v.step_entries else (v.nnz_pad if v.nparts else v.nnz), np.uint64),
                nhot=int(v.nhot),
                hot_rows=[arr(v.hot_rows[j], v.nhot, np.uint32) for j in range(v.n_in)],
                part_range=arr(v.part_range, 2 * v.nparts, np.uint64).reshape(-1, 2),
                step_entries=int(v.step_entries), nsteps=int(v.nsteps))


class Batch:
    """Owns an ``mttkrp_batch_handle``; keeps its layouts alive."""

    def __init__(self, ptr: int, layouts, R: int, dev_mem=None):
        self._ptr = ptr
        self.layouts = list(layouts)
        self.R = R
        self.dev_mem = dev_mem      # caller-owned device memory (mttkrp_batch_create_in)

    @property
    def ptr(self) -> int:
        if not self._ptr:
            raise MttkrpError(MTTKRP_EINVAL, "batch already freed")
        return self._ptr

    def free(self):
        if self._ptr:
            _lib.mttkrp_batch_free(ctypes.c_void_p(self._ptr))
            self._ptr = 0
        self.dev_mem = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mttkrp_batch_create(layouts, R: int, opts=None) -> Batch:
    arr = (ctypes.c_void_p * len(layouts))(*[h.ptr for h in layouts])
    o = _opts(opts)
    b = ctypes.c_void_p()
    _check(_lib.mttkrp_batch_create(arr, len(layouts), int(R), ctypes.byref(o) if o is not None else None,
                                    ctypes.byref(b)))
    return Batch(b.value, layouts, R)


def mttkrp_batch_bytes(layouts, R: int) -> int:
    arr = (ctypes.c_void_p * len(layouts))(*[h.ptr for h in layouts])
    out = ctypes.c_uint64()
    _check(_lib.mttkrp_batch_bytes(arr, len(layouts), int(R), ctypes.byref(out)))
    return int(out.value)


def mttkrp_batch_create_in(layouts, R: int, dev_mem, opts=None, stream=None) -> Batch:
    """A batch whose tables live in ``dev_mem`` (a uint8 device tensor of at
    least ``mttkrp_batch_bytes``), kept by the returned batch until freed."""
    arr = (ctypes.c_void_p * len(layouts))(*[h.ptr for h in layouts])
    o = _opts(opts)
    b = ctypes.c_void_p()
    _check(_lib.mttkrp_batch_create_in(arr, len(layouts), int(R), ctypes.byref(o) if o is not None else None,
                                       ctypes.c_void_p(int(dev_mem.data_ptr())), int(dev_mem.numel()),
                                       ctypes.c_void_p(_stream(stream)), ctypes.byref(b)))
    return Batch(b.value, layouts, R, dev_mem=dev_mem)


def _autotune_args(layouts, R, factors, outs):
    count = len(layouts)
    N = len(layouts[0].dims)
    if len(factors) != count or len(outs) != count:
        raise MttkrpError(MTTKRP_EINVAL, "need factors and outputs for every tensor")
    for t, h in enumerate(layouts):
        if len(factors[t]) != N or len(outs[t]) != N:
            raise MttkrpError(MTTKRP_EINVAL, f"tensor {t}: need N factors and N outputs")
        for m in range(N):
            _check_factor(factors[t][m], h.dims[m], R, "fp32", f"tensor {t} factor {m}")
            _check_factor(outs[t][m], h.dims[m], R, "fp32", f"tensor {t} output {m}")
    arr = (ctypes.c_void_p * count)(*[h.ptr for h in layouts])
    fac = (ctypes.c_void_p * (count * N))(*[int(f.data_ptr()) for fs in factors for f in fs])
    out = (ctypes.c_void_p * (count * N))(*[int(o.data_ptr()) for os_ in outs for o in os_])
    return count, arr, fac, out


def mttkrp_batch_autotune(layouts, R: int, factors, outs, candidates=None, reps: int = 3, stream=None):
    """Time the batched all-mode MTTKRP for each candidate parts_per_cu, leave
    the fastest set on the layouts and return ``(best, {candidate: ms})``.
    factors: per tensor, N fp32 device tensors; outs: per tensor, N outputs
    (tensor t's mode-n output of shape (I_n, R))."""
    count, arr, fac, out = _autotune_args(layouts, R, factors, outs)
    cands = list(candidates) if candidates is not None else [1, 2, 4, 8, 16]
    carr = (ctypes.c_int * len(cands))(*cands)
    times = (ctypes.c_float * len(cands))()
    best = ctypes.c_int()
    _check(_lib.mttkrp_batch_autotune(arr, count, int(R), carr, len(cands), fac, out, int(reps),
                                      ctypes.c_void_p(_stream(stream)), ctypes.byref(best), times))
    return int(best.value), {c: float(times[i]) for i, c in enumerate(cands)}


def mttkrp_batch_autotune_default_shapes(N: int):
    """The shape autotuner's default candidates for N-mode tensors, as
    (parts_per_cu, threads, gathers) tuples."""
    n = _lib.mttkrp_batch_autotune_default_shapes(int(N), None)
    arr = (mttkrp_part_shape * max(n, 1))()
    _lib.mttkrp_batch_autotune_default_shapes(int(N), arr)
    return [(arr[i].parts_per_cu, arr[i].threads, arr[i].gathers) for i in range(n)]


def mttkrp_batch_autotune_shape(layouts, R: int, factors, outs, candidates=None, reps: int = 3, stream=None):
    """Time the batched all-mode MTTKRP for each candidate launch shape
    (parts_per_cu, threads, gathers), leave the fastest set on the layouts and
    return ``(best, {shape: ms})``; candidates None = the library's defaults."""
    count, arr, fac, out = _autotune_args(layouts, R, factors, outs)
    cands = ([tuple(c) for c in candidates] if candidates is not None
             else mttkrp_batch_autotune_default_shapes(len(layouts[0].dims)))
    carr = (mttkrp_part_shape * len(cands))(*[mttkrp_part_shape(*c) for c in cands])
    times = (ctypes.c_float * len(cands))()
    best = mttkrp_part_shape()
    _check(_lib.mttkrp_batch_autotune_shape(arr, count, int(R), carr, len(cands), fac, out, int(reps),
                                            ctypes.c_void_p(_stream(stream)), ctypes.byref(best), times))
    return (best.parts_per_cu, best.threads, best.gathers), {c: float(times[i]) for i, c in enumerate(cands)}


def mttkrp_autotune_shape(h: Layout, R: int, factors, outs, candidates=None, reps: int = 3, stream=None):
    """Time mttkrp_run along every mode for each candidate launch shape
    (parts_per_cu, threads, gathers) on one layout, leave the fastest set and
    return ``(best, {shape: ms})``; candidates None = the library's defaults.
    factors, outs: N fp32 device tensors each (outs[n] of shape (I_n, R))."""
    count, arr, fac, out = _autotune_args([h], R, [factors], [outs])
    cands = ([tuple(c) for c in candidates] if candidates is not None
             else mttkrp_batch_autotune_default_shapes(len(h.dims)))
    carr = (mttkrp_part_shape * len(cands))(*[mttkrp_part_shape(*c) for c in cands])
    times = (ctypes.c_float * len(cands))()
    best = mttkrp_part_shape()
    _check(_lib.mttkrp_autotune_shape(ctypes.c_void_p(h.ptr), int(R), carr, len(cands), fac, out, int(reps),
                                      ctypes.c_void_p(_stream(stream)), ctypes.byref(best), times))
    return (best.parts_per_cu, best.threads, best.gathers), {c: float(times[i]) for i, c in enumerate(cands)}


def mttkrp_batch_run(b: Batch, mode: int, factors, outs, stream=None):
    """factors: list (per tensor) of lists of N fp32 device tensors; outs: list of outputs."""
    import torch
    N = len(b.layouts[0].dims)
    if len(factors) != len(b.layouts) or len(outs) != len(b.layouts):
        raise MttkrpError(MTTKRP_EINVAL, "need factors and outputs for every tensor of the batch")
    if not 0 <= int(mode) < N:
        raise MttkrpError(MTTKRP_EINVAL, "mode out of range")
    fp = (ctypes.c_void_p * (len(b.layouts) * N))()
    op = (ctypes.c_void_p * len(b.layouts))()
    for t, (h, fs, o) in enumerate(zip(b.layouts, factors, outs)):
        for m in range(N):
            if m != mode:
                _check_factor(fs[m], h.dims[m], b.R, "fp32", f"factor {m} of tensor {t}")
                fp[t * N + m] = int(fs[m].data_ptr())
        if o.dtype != torch.float32 or not o.is_cuda or not o.is_contiguous() or tuple(o.shape) != (h.dims[mode], b.R):
            raise MttkrpError(MTTKRP_EINVAL, f"output of tensor {t} must be ({h.dims[mode]}, {b.R}) float32")
        op[t] = int(o.data_ptr())
    _check(_lib.mttkrp_batch_run(ctypes.c_void_p(b.ptr), int(mode), fp, op, ctypes.c_void_p(_stream(stream))))


def mttkrp_batch_run_bf16(b: Batch, mode: int, factors, outs, stream=None):
    """As mttkrp_batch_run on a batch created with factor_dtype MTTKRP_BF16:
    factors are bfloat16 device tensors."""
    import torch
    N = len(b.layouts[0].dims)
    if len(factors) != len(b.layouts) or len(outs) != len(b.layouts):
        raise MttkrpError(MTTKRP_EINVAL, "need factors and outputs for every tensor of the batch")
    if not 0 <= int(mode) < N:
        raise MttkrpError(MTTKRP_EINVAL, "mode out of range")
    fp = (ctypes.c_void_p * (len(b.layouts) * N))()
    op = (ctypes.c_void_p * len(b.layouts))()
    for t, (h, fs, o) in enumerate(zip(b.layouts, factors, outs)):
        for m in range(N):
            if m != mode:
                _check_factor(fs[m], h.dims[m], b.R, "bf16", f"factor {m} of tensor {t}")
                fp[t * N + m] = int(fs[m].data_ptr())
        if o.dtype != torch.float32 or not o.is_cuda or not o.is_contiguous() or tuple(o.shape) != (h.dims[mode], b.R):
            raise MttkrpError(MTTKRP_EINVAL, f"output of tensor {t} must be ({h.dims[mode]}, {b.R}) float32")
        op[t] = int(o.data_ptr())
    _check(_lib.mttkrp_batch_run_bf16(ctypes.c_void_p(b.ptr), int(mode), fp, op, ctypes.c_void_p(_stream(stream))))


def mttkrp_batch_free(b: Batch):
    b.free()


def cpd_als_batch_iter_async(b: Batch, factors, lambdas, fits=None, stream=None):
    """One CP-ALS sweep for every tensor of the batch (enqueued only)."""
    import torch
    N = len(b.layouts[0].dims)
    C = len(b.layouts)
    fp = (ctypes.c_void_p * (C * N))()
    lp = (ctypes.c_void_p * C)()
    ftp = (ctypes.c_void_p * C)()
    for t, h in enumerate(b.layouts):
        for m in range(N):
            _check_factor(factors[t][m], h.dims[m], b.R, "fp32", f"factor {m} of tensor {t}")
            fp[t * N + m] = int(factors[t][m].data_ptr())
        if lambdas[t].dtype != torch.float64 or lambdas[t].numel() < b.R:
            raise MttkrpError(MTTKRP_EINVAL, "lambdas must be float64 device tensors with R entries")
        lp[t] = int(lambdas[t].data_ptr())
        ftp[t] = int(fits[t].data_ptr()) if fits is not None else None
    _check(_lib.cpd_als_batch_iter_async(ctypes.c_void_p(b.ptr), fp, lp, ftp if fits is not None else None,
                                         ctypes.c_void_p(_stream(stream))))
