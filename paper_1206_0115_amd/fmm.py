"""Python binding of ``libfmm.so`` (the C-ABI in ``include/fmm.h``).

Argument marshalling only: tensors are checked for device, dtype and shape
and their device pointers are passed to the library, whose HIP kernels do
every step of the computation.  There is no fallback: if the library is not
built the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm.so")

FMM_OK, FMM_ERR_ARG, FMM_ERR_OOM, FMM_ERR_HIP, FMM_ERR_STATE = 0, -1, -2, -3, -4
FMM_FP64, FMM_MIXED_FP32, FMM_MIXED_BF16, FMM_FP64_SVD, FMM_MIXED_SVD = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FMM_FP64, "mixed": FMM_MIXED_FP32, "mixed_fp32": FMM_MIXED_FP32,
              "mixed_bf16": FMM_MIXED_BF16,  # reserved; the library rejects it
              "fp64_svd": FMM_FP64_SVD, "mixed_svd": FMM_MIXED_SVD}
FMM_SCHEDULE_SERIAL, FMM_SCHEDULE_FORKED, FMM_SCHEDULE_PIPELINED = 0, 1, 2
SCHEDULES = {"serial": FMM_SCHEDULE_SERIAL, "forked": FMM_SCHEDULE_FORKED,
             "pipelined": FMM_SCHEDULE_PIPELINED}
FMM_KERNEL_INV_R, FMM_KERNEL_INV_R2 = 1, 2
KERNELS = {"inv_r": FMM_KERNEL_INV_R, "inv_r2": FMM_KERNEL_INV_R2}
FMM_NEAR_ONE_SIDED, FMM_NEAR_MUTUAL = 0, 1
NEAR_MODES = {"one_sided": FMM_NEAR_ONE_SIDED, "mutual": FMM_NEAR_MUTUAL}

EXPORT_KEYS, EXPORT_PERM, EXPORT_LEAF_START, EXPORT_CELL_KEYS = 0, 1, 2, 3
EXPORT_NEAR_OFF, EXPORT_NEAR_IDX, EXPORT_FAR_OFF, EXPORT_FAR_IDX = 4, 5, 6, 7
EXPORT_MUTUAL_OFF, EXPORT_MUTUAL_IDX = 8, 9


class FMMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class FmmInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("height", ctypes.c_int32), ("order", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("ld", ctypes.c_int32),
        ("n_leaf", ctypes.c_int64),
        ("ncell", ctypes.c_int64 * 21),
        ("lo", ctypes.c_double * 3), ("L", ctypes.c_double),
        ("near_pairs", ctypes.c_int64),
        ("far_pairs", ctypes.c_int64),
        ("far_pairs_level", ctypes.c_int64 * 21),
        ("m2l_tiles", ctypes.c_int64),
        ("m2l_active_slots", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("m2l_flops", ctypes.c_double),
        ("m2l_groups", ctypes.c_int64),
        ("m2l_groups_empty", ctypes.c_int64),
        ("m2l_group_skip", ctypes.c_int32),
    ]


class SvdInfo(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("rank", ctypes.c_int32 * 16),
        ("rmax_pad", ctypes.c_int32),
        ("weighted_rank", ctypes.c_double),
    ]


class RequestStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("done", ctypes.c_int32),
        ("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
        ("done_s", ctypes.c_double),
        ("batch", ctypes.c_int64), ("plan_bytes", ctypes.c_int64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "completed", "rejected", "batches", "graph_captures", "graph_replays",
        "max_batch_jobs", "max_active_seen", "peak_admitted_bytes")]


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1206_0115_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.fmm_plan.argtypes = [vp, i64, i32, i32]
    L.fmm_plan.restype = vp
    L.fmm_plan_stream.argtypes = [vp, i64, i32, i32, vp]
    L.fmm_plan_stream.restype = vp
    L.fmm_evaluate.argtypes = [vp, vp, vp, vp, vp]
    L.fmm_evaluate_parts.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.fmm_release.argtypes = [vp]
    L.fmm_release.restype = None
    L.fmm_last_error.restype = ctypes.c_char_p
    L.fmm_plan_set_precision.argtypes = [vp, i32]
    L.fmm_plan_set_schedule.argtypes = [vp, i32]
    L.fmm_plan_set_graph.argtypes = [vp, i32]
    L.fmm_plan_set_kernel.argtypes = [vp, i32]
    L.fmm_plan_set_near.argtypes = [vp, i32]
    L.fmm_plan_set_m2l_tolerance.argtypes = [vp, ctypes.c_double]
    L.fmm_plan_set_m2l_fold_interval.argtypes = [vp, i32]
    L.fmm_plan_set_m2l_split.argtypes = [vp, i32]
    L.fmm_plan_m2l_split.argtypes = [vp, ctypes.POINTER(i32)]
    L.fmm_plan_svd_info.argtypes = [vp, ctypes.POINTER(SvdInfo)]
    L.fmm_plan_info.argtypes = [vp, ctypes.POINTER(FmmInfo)]
    L.fmm_plan_export.argtypes = [vp, i32, i32, vp, sz]
    L.fmm_set_m2l_timing_events.argtypes = [vp, vp]
    L.fmm_set_step_timing_events.argtypes = [i32, vp, vp]
    L.fmm_trim_cache.restype = None
    L.fmm_direct_sampled.argtypes = [vp, vp, i64, vp, i64, i32, vp, vp, vp]
    L.fmm_direct_sampled_noalloc.argtypes = [vp, vp, i64, vp, i64, i32, vp, vp, vp]
    L.fmm_server_create.argtypes = [sz, i32]
    L.fmm_server_create.restype = vp
    L.fmm_server_submit.argtypes = [vp, vp, vp, i64, i32, i32, i32, vp, vp, vp]
    L.fmm_server_request_error.argtypes = [vp, i64, ctypes.c_char_p, sz]
    L.fmm_server_submit.restype = i64
    L.fmm_server_poll.argtypes = [vp, i64, ctypes.POINTER(RequestStats)]
    L.fmm_server_wait.argtypes = [vp, i64, ctypes.POINTER(RequestStats)]
    L.fmm_server_now.argtypes = [vp]
    L.fmm_server_now.restype = ctypes.c_double
    L.fmm_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.fmm_server_destroy.argtypes = [vp]
    L.fmm_server_destroy.restype = None
    _lib = L
    return L


def last_error() -> str:
    return lib().fmm_last_error().decode()


def _check(rc):
    if rc != FMM_OK:
        raise FMMError(rc, last_error())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_f64(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """An FMM plan over fixed particle positions (``fmm_plan``)."""

    def __init__(self, positions, height: int, order: int, precision="fp64", stream=None,
                 kernel="inv_r", m2l_tolerance=None):
        self.n = int(positions.shape[0])
        ptr = _dev_f64(positions, (self.n, 3), "positions")
        if stream is None:
            h = lib().fmm_plan(ptr, self.n, int(height), int(order))
        else:
            h = lib().fmm_plan_stream(ptr, self.n, int(height), int(order),
                                      _stream_handle(stream))
        if not h:
            raise FMMError(FMM_ERR_ARG, last_error())
        self._h = ctypes.c_void_p(h)
        self.height, self.order = int(height), int(order)
        self.kernel = FMM_KERNEL_INV_R
        if kernel not in ("inv_r", FMM_KERNEL_INV_R):
            self.set_kernel(kernel)
        if m2l_tolerance is not None:  # before the mode, so only these operators load
            self.set_m2l_tolerance(m2l_tolerance)
        self.set_precision(precision)

    @property
    def handle(self):
        return self._h

    def set_precision(self, precision):
        mode = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(lib().fmm_plan_set_precision(self._h, mode))
        self.precision = mode

    def set_schedule(self, schedule):
        """"serial" (every operator on the caller's stream) or "forked" (the
        near field on the plan's side stream, concurrently with the far
        chain; the default)."""
        code = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        _check(lib().fmm_plan_set_schedule(self._h, code))

    def set_graph(self, on: bool):
        """Replay evaluations from a captured hipGraph (``fmm_plan_set_graph``)."""
        _check(lib().fmm_plan_set_graph(self._h, 1 if on else 0))

    def set_near(self, mode):
        """"one_sided" (the default) or "mutual" (each pair of distinct
        neighbour leaves computed once, ``fmm_plan_set_near``)."""
        code = NEAR_MODES[mode] if isinstance(mode, str) else int(mode)
        _check(lib().fmm_plan_set_near(self._h, code))

    def set_kernel(self, kernel):
        """"inv_r" (1/r, the default) or "inv_r2" (1/r^2)."""
        code = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        _check(lib().fmm_plan_set_kernel(self._h, code))
        self.kernel = code

    def set_m2l_tolerance(self, eps: float):
        _check(lib().fmm_plan_set_m2l_tolerance(self._h, float(eps)))

    def set_m2l_fold_interval(self, offsets: int):
        """Far offsets between FP64 folds in the compressed mixed mode (0 =
        the default for the order)."""
        _check(lib().fmm_plan_set_m2l_fold_interval(self._h, int(offsets)))

    def set_m2l_split(self, parts: int):
        """Far-offset ranges per tile of the compressed M2L (1..4; 0 = chosen
        from the tile count and the device's resident workgroups)."""
        _check(lib().fmm_plan_set_m2l_split(self._h, int(parts)))

    def m2l_split(self) -> int:
        out = ctypes.c_int(0)
        _check(lib().fmm_plan_m2l_split(self._h, ctypes.byref(out)))
        return int(out.value)

    def svd_info(self) -> SvdInfo:
        out = SvdInfo()
        _check(lib().fmm_plan_svd_info(self._h, ctypes.byref(out)))
        return out

    def evaluate(self, charges, potential=None, forces=None, stream=None):
        import torch
        q = _dev_f64(charges, (self.n,), "charges")
        if potential is None:
            potential = torch.empty(self.n, dtype=torch.float64, device=charges.device)
        if forces is None:
            forces = torch.empty(self.n, 3, dtype=torch.float64, device=charges.device)
        _check(lib().fmm_evaluate(self._h, q, _dev_f64(potential, (self.n,), "potential"),
                                  _dev_f64(forces, (self.n, 3), "forces"),
                                  _stream_handle(stream)))
        return potential, forces

    def evaluate_parts(self, charges, stream=None):
        import torch
        q = _dev_f64(charges, (self.n,), "charges")
        dev = charges.device
        pn = torch.empty(self.n, dtype=torch.float64, device=dev)
        fn = torch.empty(self.n, 3, dtype=torch.float64, device=dev)
        pf = torch.empty(self.n, dtype=torch.float64, device=dev)
        ff = torch.empty(self.n, 3, dtype=torch.float64, device=dev)
        _check(lib().fmm_evaluate_parts(self._h, q, ctypes.c_void_p(pn.data_ptr()),
                                        ctypes.c_void_p(fn.data_ptr()),
                                        ctypes.c_void_p(pf.data_ptr()),
                                        ctypes.c_void_p(ff.data_ptr()),
                                        _stream_handle(stream)))
        return pn, fn, pf, ff

    def info(self) -> FmmInfo:
        out = FmmInfo()
        _check(lib().fmm_plan_info(self._h, ctypes.byref(out)))
        return out

    def export(self, what: int, level: int = 0) -> np.ndarray:
        inf = self.info()
        if what == EXPORT_KEYS:
            out = np.empty(self.n, dtype=np.uint64)
        elif what == EXPORT_PERM:
            out = np.empty(self.n, dtype=np.int64)
        elif what in (EXPORT_LEAF_START, EXPORT_NEAR_OFF):
            out = np.empty(inf.n_leaf + 1, dtype=np.int64)
        elif what == EXPORT_CELL_KEYS:
            out = np.empty(inf.ncell[level], dtype=np.uint64)
        elif what == EXPORT_NEAR_IDX:
            off = self.export(EXPORT_NEAR_OFF)
            out = np.empty(int(off[-1]), dtype=np.int64)
        elif what == EXPORT_FAR_OFF:
            out = np.empty(inf.ncell[level] + 1, dtype=np.int64)
        elif what == EXPORT_FAR_IDX:
            off = self.export(EXPORT_FAR_OFF, level)
            out = np.empty(int(off[-1]), dtype=np.int64)
        elif what == EXPORT_MUTUAL_OFF:
            out = np.empty(27, dtype=np.int64)
        elif what == EXPORT_MUTUAL_IDX:
            off = self.export(EXPORT_MUTUAL_OFF)
            out = np.empty(max(int(off[-1]), 1), dtype=np.int64)[:int(off[-1])]
        else:
            raise ValueError("unknown export item")
        _check(lib().fmm_plan_export(self._h, what, level,
                                     out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def release(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().fmm_release(h)
        self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


FMM_TIME_M2L, FMM_TIME_P2P, FMM_TIME_P2M, FMM_TIME_L2P = 0, 1, 2, 3
FMM_TIME_M2M, FMM_TIME_L2L, FMM_TIME_LOC_SUM = 4, 5, 6
TIMED_STEPS = {"m2l": FMM_TIME_M2L, "p2p": FMM_TIME_P2P, "p2m": FMM_TIME_P2M,
               "l2p": FMM_TIME_L2P, "m2m": FMM_TIME_M2M, "l2l": FMM_TIME_L2L,
               "loc_sum": FMM_TIME_LOC_SUM}


def set_step_timing_events(step, ev0, ev1):
    """Bracket one operator's kernel ("m2l", "p2p", "p2m", "l2p", "loc_sum",
    or all levels of "m2m" or "l2l") in later evaluations on this thread with
    two ``torch.cuda.Event`` objects (or None to stop)."""
    code = TIMED_STEPS[step] if isinstance(step, str) else int(step)
    if ev0 is None:
        _check(lib().fmm_set_step_timing_events(code, None, None))
        return
    _check(lib().fmm_set_step_timing_events(code, ctypes.c_void_p(ev0.cuda_event),
                                            ctypes.c_void_p(ev1.cuda_event)))


def set_m2l_timing_events(ev0, ev1):
    """Bracket the M2L kernel of later evaluations on this thread with two
    ``torch.cuda.Event`` objects (or None to stop)."""
    if ev0 is None:
        _check(lib().fmm_set_m2l_timing_events(None, None))
        return
    _check(lib().fmm_set_m2l_timing_events(ctypes.c_void_p(ev0.cuda_event),
                                           ctypes.c_void_p(ev1.cuda_event)))


def direct_sampled(positions, charges, targets, kernel="inv_r", stream=None):
    """Exact potentials and forces at the particles ``targets`` (int64
    device tensor of indices) over all sources (``fmm_direct_sampled``)."""
    import torch
    n = int(positions.shape[0])
    pos = _dev_f64(positions, (n, 3), "positions")
    q = _dev_f64(charges, (n,), "charges")
    if targets.dtype != torch.int64 or not targets.is_cuda or targets.dim() != 1:
        raise ValueError("targets must be a 1-D int64 device tensor")
    tg = targets.contiguous()
    nt = int(tg.shape[0])
    phi = torch.empty(nt, dtype=torch.float64, device=positions.device)
    f = torch.empty(nt, 3, dtype=torch.float64, device=positions.device)
    _check(lib().fmm_direct_sampled(pos, q, n, ctypes.c_void_p(tg.data_ptr()), nt,
                                    KERNELS[kernel], ctypes.c_void_p(phi.data_ptr()),
                                    ctypes.c_void_p(f.data_ptr()), _stream_handle(stream)))
    return phi, f


def trim_cache():
    lib().fmm_trim_cache()


class Request:
    """A queued evaluation; keeps its input and output tensors alive."""

    def __init__(self, server, ticket, tensors, potential, forces):
        self.server, self.ticket = server, ticket
        self._tensors = tensors
        self.potential, self.forces = potential, forces

    def poll(self):
        st = RequestStats()
        rc = lib().fmm_server_poll(self.server._h, self.ticket, ctypes.byref(st))
        if rc < 0:
            raise FMMError(rc, last_error())
        return st if rc == 1 else None

    def wait(self):
        st = RequestStats()
        lib().fmm_server_wait(self.server._h, self.ticket, ctypes.byref(st))
        return st

    def error(self) -> str:
        """Message of the request's failure ("" if none)."""
        buf = ctypes.create_string_buffer(1024)
        rc = lib().fmm_server_request_error(self.server._h, self.ticket, buf, len(buf))
        if rc < 0:
            raise FMMError(rc, last_error())
        return buf.value.decode()


class Server:
    """The serving loop (``fmm_server_*``): continuous batching of evaluations
    admitted by device-memory footprint."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 32):
        h = lib().fmm_server_create(int(hbm_budget_bytes), int(max_active))
        if not h:
            raise FMMError(FMM_ERR_ARG, last_error())
        self._h = ctypes.c_void_p(h)

    def submit(self, positions, charges, height, order, precision="fp64",
               potential=None, forces=None, stream=None) -> Request:
        """Queue one evaluation; the server starts on it after the work
        queued so far on `stream` (default: the current stream)."""
        import torch
        n = int(positions.shape[0])
        pp = _dev_f64(positions, (n, 3), "positions")
        qp = _dev_f64(charges, (n,), "charges")
        if potential is None:
            potential = torch.empty(n, dtype=torch.float64, device=positions.device)
        if forces is None:
            forces = torch.empty(n, 3, dtype=torch.float64, device=positions.device)
        mode = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        t = lib().fmm_server_submit(self._h, pp, qp, n, int(height), int(order), mode,
                                    _dev_f64(potential, (n,), "potential"),
                                    _dev_f64(forces, (n, 3), "forces"),
                                    _stream_handle(stream))
        if t < 0:
            raise FMMError(int(t), last_error())
        return Request(self, int(t), (positions, charges), potential, forces)

    def now(self) -> float:
        return float(lib().fmm_server_now(self._h))

    def stats(self) -> ServerStats:
        out = ServerStats()
        _check(lib().fmm_server_get_stats(self._h, ctypes.byref(out)))
        return out

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().fmm_server_destroy(h)
        self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
