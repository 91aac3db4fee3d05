"""Python binding of librecon: grayscale reconstruction by dilation and by
erosion, fill-holes, h-dome and regional maxima on uint8 tiles, hand-written HIP
for AMD MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``librecon.so``.  torch provides device memory (uint8 CUDA/HIP
tensors, whose ``data_ptr()`` is passed through) and streams
(``torch.cuda.Stream().cuda_stream``).  Importing this package without the
built library raises; there is no CPU fallback.

Low-level functions keep the C names (``recon_create``, ``recon_dilate``,
``recon_fill_holes``, ``recon_erode``, ``recon_hdome``, ``recon_regional_max``,
``recon_batch``, ``recon_submit``, ``recon_poll``, ``recon_wait``, ...);
``Recon`` wraps a context for convenience.  ``recon_pipeline_run`` runs the
co-scheduled per-tile pipeline over host tiles: its GPU variants are the HIP
operations; its CPU variants run in the library's own host code on the CPU
workers the scheduler is given (the paper's CPU + GPU execution), never as a
replacement for a missing GPU.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librecon.so")

RECON_OK, RECON_EINVAL, RECON_ENOMEM, RECON_EDEVICE, RECON_EAGAIN, RECON_ETIMEDOUT = 0, -1, -2, -3, -4, -5
RECON_OP_DILATE, RECON_OP_FILL_HOLES, RECON_OP_ERODE, RECON_OP_HDOME, RECON_OP_REGIONAL_MAX = 0, 1, 2, 3, 4
OPS = {"dilate": RECON_OP_DILATE, "fill_holes": RECON_OP_FILL_HOLES, "erode": RECON_OP_ERODE,
       "hdome": RECON_OP_HDOME, "regional_max": RECON_OP_REGIONAL_MAX}
TWO_PLANE_OPS = ("dilate", "erode")   # marker and mask are two images

# every symbol the C header declares
EXPORTED = (
    "recon_create", "recon_destroy", "recon_dilate", "recon_dilate_noalloc", "recon_fill_holes", "recon_erode",
    "recon_hdome", "recon_regional_max", "recon_label", "recon_area_threshold", "recon_distance",
    "recon_pre_watershed", "recon_batch",
    "recon_submit", "recon_poll", "recon_wait", "recon_serve_stop", "recon_serve_stats", "recon_last_stats",
    "recon_launch_times", "recon_last_error", "recon_pipeline_run", "recon_pipeline_error",
    "recon_pipeline_host_op", "recon_enqueue_status",
)


class ReconError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("librecon error %d: %s" % (code, msg))
        self.code = code


class ReconAgain(ReconError):
    """Serving admission is full (RECON_EAGAIN)."""


class ReconTimeout(ReconError):
    """recon_wait timed out (RECON_ETIMEDOUT)."""


class recon_image(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("pitch", ctypes.c_int64)]


class recon_task(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("conn", ctypes.c_int32), ("image", recon_image),
                ("mask", recon_image), ("scan_rounds", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("h", ctypes.c_int32), ("block_rows", ctypes.c_int32)]


class recon_config(ctypes.Structure):
    _fields_ = [("block_rows", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("scan_rounds", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("serve_mem_cap", ctypes.c_int64), ("serve_slots", ctypes.c_int32),
                ("stop_after_stage", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("drain_budget", ctypes.c_int32), ("binary_drain_budget", ctypes.c_int32),
                ("test_fault", ctypes.c_int32), ("component_route", ctypes.c_int32),
                ("spill_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class recon_stats(ctypes.Structure):
    _fields_ = [("dense_visits", ctypes.c_int64), ("revisits", ctypes.c_int64),
                ("reruns", ctypes.c_int64), ("queue_overflows", ctypes.c_int64),
                ("requests", ctypes.c_int64), ("aborted", ctypes.c_int64),
                ("dense_ms", ctypes.c_float), ("seed_ms", ctypes.c_float), ("drain_ms", ctypes.c_float),
                ("total_ms", ctypes.c_float), ("component_tasks", ctypes.c_int64),
                ("route_ms", ctypes.c_float), ("reserved_f", ctypes.c_float),
                ("queue_spills", ctypes.c_int64)]


class recon_serve_counters(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("requests", ctypes.c_int64), ("max_batch", ctypes.c_int64),
                ("max_busy_lanes", ctypes.c_int64), ("early_completions", ctypes.c_int64)]


# the co-scheduled tile pipeline (recon_pipeline_run)
PIPE_OPS = ("hdome", "fill_holes", "area_threshold", "markers", "label")
RECON_SCHED_FCFS, RECON_SCHED_PATS = 0, 1
POLICIES = {"fcfs": RECON_SCHED_FCFS, "pats": RECON_SCHED_PATS}


class recon_pipe_tile(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("pitch", ctypes.c_int64), ("objects", ctypes.c_void_p), ("markers", ctypes.c_void_p),
                ("labels", ctypes.c_void_p), ("label_pitch", ctypes.c_int64), ("count", ctypes.c_void_p)]


class recon_pipe_event(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("op", ctypes.c_int32), ("device", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double)]


class recon_pipe_config(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("cpu_workers", ctypes.c_int32), ("use_gpu", ctypes.c_int32),
                ("window", ctypes.c_int32), ("data_locality", ctypes.c_int32), ("conn", ctypes.c_int32),
                ("h", ctypes.c_int32), ("cpu_max_speedup", ctypes.c_float), ("area_min", ctypes.c_int64),
                ("area_max", ctypes.c_int64), ("speedup", ctypes.c_float * 5),
                ("transfer_impact", ctypes.c_float * 5), ("io_threads", ctypes.c_int32),
                ("cpu_guard", ctypes.c_int32), ("gpu_ms", ctypes.c_float * 5), ("prefetch", ctypes.c_int32),
                ("trace_cap", ctypes.c_int32),
                ("trace", ctypes.POINTER(recon_pipe_event)), ("gpu_inflight", ctypes.c_int32),
                ("gpu_batch", ctypes.c_int32)]


class recon_pipe_stats(ctypes.Structure):
    _fields_ = [("makespan_ms", ctypes.c_double), ("ops_cpu", ctypes.c_int64 * 5),
                ("ops_gpu", ctypes.c_int64 * 5), ("busy_cpu_ms", ctypes.c_double * 5),
                ("busy_gpu_ms", ctypes.c_double * 5), ("uploads", ctypes.c_int64), ("downloads", ctypes.c_int64),
                ("upload_bytes", ctypes.c_int64), ("download_bytes", ctypes.c_int64),
                ("transfer_ms", ctypes.c_double), ("io_ms", ctypes.c_double), ("trace_n", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librecon.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("librecon.so is not built (%s); run `python paper_1209_3332_amd/build.py`" % path)
    import torch  # noqa: F401  (load torch's HIP runtime first so one runtime serves both)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.recon_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(recon_config)]
    lib.recon_destroy.argtypes = [P]
    lib.recon_dilate.argtypes = [P, ctypes.POINTER(recon_image), ctypes.POINTER(recon_image), ctypes.c_int, P]
    lib.recon_dilate_noalloc.argtypes = [P, ctypes.POINTER(recon_image), ctypes.POINTER(recon_image),
                                         ctypes.c_int, P]
    lib.recon_fill_holes.argtypes = [P, ctypes.POINTER(recon_image), ctypes.c_int, P]
    lib.recon_erode.argtypes = [P, ctypes.POINTER(recon_image), ctypes.POINTER(recon_image), ctypes.c_int, P]
    lib.recon_hdome.argtypes = [P, ctypes.POINTER(recon_image), ctypes.c_int, ctypes.c_int, P]
    lib.recon_regional_max.argtypes = [P, ctypes.POINTER(recon_image), ctypes.c_int, P]
    lib.recon_label.argtypes = [P, ctypes.POINTER(recon_image), P, ctypes.c_int64, ctypes.c_int, P, P]
    lib.recon_area_threshold.argtypes = [P, ctypes.POINTER(recon_image), ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_int64, P]
    lib.recon_distance.argtypes = [P, ctypes.POINTER(recon_image), P, ctypes.c_int64, P]
    lib.recon_pre_watershed.argtypes = [P, ctypes.POINTER(recon_image), ctypes.c_int, P]
    lib.recon_batch.argtypes = [P, ctypes.POINTER(recon_task), ctypes.c_int32, P]
    lib.recon_submit.argtypes = [P, ctypes.POINTER(recon_task), ctypes.POINTER(ctypes.c_uint64)]
    lib.recon_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    lib.recon_wait.argtypes = [P, ctypes.c_uint64, ctypes.c_int64]
    lib.recon_serve_stop.argtypes = [P]
    lib.recon_serve_stats.argtypes = [P, ctypes.POINTER(recon_serve_counters)]
    lib.recon_last_stats.argtypes = [P, ctypes.POINTER(recon_stats)]
    lib.recon_enqueue_status.argtypes = [P, P, P]
    F = ctypes.POINTER(ctypes.c_float)
    lib.recon_launch_times.argtypes = [P, ctypes.c_int, F, F, F, F, F]
    lib.recon_last_error.argtypes = []
    lib.recon_last_error.restype = ctypes.c_char_p
    lib.recon_pipeline_run.argtypes = [P, ctypes.POINTER(recon_pipe_tile), ctypes.c_int32,
                                       ctypes.POINTER(recon_pipe_config), ctypes.POINTER(recon_pipe_stats)]
    lib.recon_pipeline_error.argtypes = []
    lib.recon_pipeline_error.restype = ctypes.c_char_p
    lib.recon_pipeline_host_op.argtypes = [ctypes.c_int, ctypes.POINTER(recon_image),
                                           ctypes.POINTER(recon_pipe_config), P, ctypes.c_int64, P]
    for name in EXPORTED:
        if name not in ("recon_last_error", "recon_pipeline_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc, msg=None):
    if rc == RECON_OK:
        return
    if msg is None:
        msg = _lib.recon_last_error().decode(errors="replace")
    if rc == RECON_EAGAIN:
        raise ReconAgain(rc, msg)
    if rc == RECON_ETIMEDOUT:
        raise ReconTimeout(rc, msg)
    raise ReconError(rc, msg)


def image_of(t) -> recon_image:
    """recon_image view of a 2-D uint8 device tensor (rows may be padded)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.dim() != 2:
        raise TypeError("expected a 2-D torch.uint8 tensor")
    if not t.is_cuda:
        raise TypeError("image tensors must live on the GPU")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError("image rows must be contiguous (stride(1) == 1)")
    return recon_image(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- low-level functions with the C names --------------------------------------------

def recon_create(device: int = 0, **cfg) -> int:
    lib = load_library()
    c = recon_config()
    for k, v in cfg.items():
        setattr(c, k, int(v))
    h = ctypes.c_void_p()
    _check(lib.recon_create(ctypes.byref(h), int(device), ctypes.byref(c)))
    return h.value


def recon_destroy(ctx: int) -> None:
    _check(load_library().recon_destroy(ctx))


def recon_dilate(ctx: int, marker, mask, conn: int = 8, stream=None) -> None:
    m, k = image_of(marker), image_of(mask)
    _check(load_library().recon_dilate(ctx, ctypes.byref(m), ctypes.byref(k), int(conn), _stream_ptr(stream)))


def recon_dilate_noalloc(ctx: int, marker, mask, conn: int = 8, stream=None) -> None:
    m, k = image_of(marker), image_of(mask)
    _check(load_library().recon_dilate_noalloc(ctx, ctypes.byref(m), ctypes.byref(k), int(conn),
                                               _stream_ptr(stream)))


def recon_fill_holes(ctx: int, img, conn: int = 8, stream=None) -> None:
    m = image_of(img)
    _check(load_library().recon_fill_holes(ctx, ctypes.byref(m), int(conn), _stream_ptr(stream)))


def recon_erode(ctx: int, marker, mask, conn: int = 8, stream=None) -> None:
    m, k = image_of(marker), image_of(mask)
    _check(load_library().recon_erode(ctx, ctypes.byref(m), ctypes.byref(k), int(conn), _stream_ptr(stream)))


def recon_hdome(ctx: int, img, h: int, conn: int = 8, stream=None) -> None:
    m = image_of(img)
    _check(load_library().recon_hdome(ctx, ctypes.byref(m), int(h), int(conn), _stream_ptr(stream)))


def recon_regional_max(ctx: int, img, conn: int = 8, stream=None) -> None:
    m = image_of(img)
    _check(load_library().recon_regional_max(ctx, ctypes.byref(m), int(conn), _stream_ptr(stream)))


def recon_label(ctx: int, img, labels, conn: int = 8, count=None, stream=None) -> None:
    """labels: 2-D torch.int32 device tensor of img's shape (rows may be padded);
    count: optional 1-element torch.int32 device tensor receiving the number of labels."""
    import torch
    m = image_of(img)
    if not isinstance(labels, torch.Tensor) or labels.dtype != torch.int32 or labels.dim() != 2 or \
            not labels.is_cuda or tuple(labels.shape) != tuple(img.shape) or labels.stride(1) != 1:
        raise TypeError("labels must be a 2-D int32 device tensor of the image's shape with contiguous rows")
    if count is not None and (count.dtype != torch.int32 or not count.is_cuda or count.numel() < 1):
        raise TypeError("count must be an int32 device tensor")
    _check(load_library().recon_label(ctx, ctypes.byref(m), labels.data_ptr(), labels.stride(0), int(conn),
                                      count.data_ptr() if count is not None else None, _stream_ptr(stream)))


def recon_area_threshold(ctx: int, img, min_area: int, max_area: int, conn: int = 8, stream=None) -> None:
    m = image_of(img)
    _check(load_library().recon_area_threshold(ctx, ctypes.byref(m), int(conn), int(min_area), int(max_area),
                                               _stream_ptr(stream)))


def recon_distance(ctx: int, img, dist2, stream=None) -> None:
    """dist2: 2-D torch.int32 device tensor of img's shape (rows may be padded)."""
    import torch
    m = image_of(img)
    if not isinstance(dist2, torch.Tensor) or dist2.dtype != torch.int32 or dist2.dim() != 2 or \
            not dist2.is_cuda or tuple(dist2.shape) != tuple(img.shape) or dist2.stride(1) != 1:
        raise TypeError("dist2 must be a 2-D int32 device tensor of the image's shape with contiguous rows")
    _check(load_library().recon_distance(ctx, ctypes.byref(m), dist2.data_ptr(), dist2.stride(0),
                                         _stream_ptr(stream)))


def recon_pre_watershed(ctx: int, img, conn: int = 8, stream=None) -> None:
    m = image_of(img)
    _check(load_library().recon_pre_watershed(ctx, ctypes.byref(m), int(conn), _stream_ptr(stream)))


def make_task(op: str, image, mask=None, conn: int = 8, scan_rounds: int = 0, queue_capacity: int = 0,
              h: int = 0, block_rows: int = 0) -> recon_task:
    """recon_task for op in OPS; `mask` for dilate / erode, `h` for hdome;
    block_rows 0 = the context's."""
    if op not in OPS:
        raise ValueError("op must be one of %s" % ", ".join(OPS))
    t = recon_task()
    t.op = OPS[op]
    t.scan_rounds = int(scan_rounds)
    t.queue_capacity = int(queue_capacity)
    t.conn = int(conn)
    t.h = int(h)
    t.block_rows = int(block_rows)
    t.image = image_of(image)
    if op in TWO_PLANE_OPS:
        t.mask = image_of(mask)
    return t


def recon_batch(ctx: int, tasks, stream=None) -> None:
    """tasks: sequence of recon_task (see make_task)."""
    arr = (recon_task * len(tasks))(*tasks)
    _check(load_library().recon_batch(ctx, arr, len(tasks), _stream_ptr(stream)))


def recon_submit(ctx: int, task: recon_task) -> int:
    tk = ctypes.c_uint64()
    _check(load_library().recon_submit(ctx, ctypes.byref(task), ctypes.byref(tk)))
    return tk.value


def recon_poll(ctx: int, ticket: int) -> bool:
    d = ctypes.c_int()
    _check(load_library().recon_poll(ctx, ticket, ctypes.byref(d)))
    return bool(d.value)


def recon_wait(ctx: int, ticket: int, timeout_us: int = -1) -> None:
    _check(load_library().recon_wait(ctx, ticket, int(timeout_us)))


def recon_serve_stop(ctx: int) -> None:
    _check(load_library().recon_serve_stop(ctx))


def recon_serve_stats(ctx: int) -> dict:
    s = recon_serve_counters()
    _check(load_library().recon_serve_stats(ctx, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in recon_serve_counters._fields_}


def recon_launch_times(ctx: int, back: int = 0) -> dict:
    """Kernel durations (ms) of a recent launch: back = 0 the last, up to 63."""
    t = [ctypes.c_float() for _ in range(5)]
    _check(load_library().recon_launch_times(ctx, int(back), *[ctypes.byref(x) for x in t]))
    return dict(zip(("dense_ms", "seed_ms", "drain_ms", "total_ms", "route_ms"), (x.value for x in t)))


def recon_last_stats(ctx: int) -> dict:
    s = recon_stats()
    _check(load_library().recon_last_stats(ctx, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in recon_stats._fields_}


def recon_enqueue_status(ctx: int, host_flag: int, stream=None) -> None:
    """Enqueue a write of the last launch's outcome (0 converged, 1 given up)
    into the pinned host word at address host_flag, on `stream`."""
    _check(load_library().recon_enqueue_status(ctx, ctypes.c_void_p(int(host_flag)), _stream_ptr(stream)))


def recon_last_error() -> str:
    return load_library().recon_last_error().decode(errors="replace")


def pipe_config(policy: str = "pats", cpu_workers: int = 0, use_gpu: bool = True, window: int = 8,
                data_locality: bool = True, conn: int = 8, h: int = 20, area_min: int = 20, area_max: int = 1000,
                speedup=None, transfer_impact=None, cpu_max_speedup: float = 0.0,
                io_threads: int = 2, gpu_ms=None, cpu_guard: bool = False,
                prefetch: bool = False, gpu_inflight: int = 1, gpu_batch: int = 1) -> recon_pipe_config:
    """recon_pipe_config; speedup / transfer_impact: dicts or sequences over PIPE_OPS."""
    c = recon_pipe_config()
    if policy not in POLICIES:
        raise ValueError("policy must be one of %s" % ", ".join(POLICIES))
    c.policy = POLICIES[policy]
    c.cpu_workers, c.use_gpu, c.window = int(cpu_workers), int(bool(use_gpu)), int(window)
    c.data_locality, c.conn, c.h = int(bool(data_locality)), int(conn), int(h)
    c.area_min, c.area_max = int(area_min), int(area_max)
    c.cpu_max_speedup = float(cpu_max_speedup)
    c.io_threads = int(io_threads)
    c.cpu_guard = int(bool(cpu_guard))
    c.prefetch = int(bool(prefetch))
    c.gpu_inflight = int(gpu_inflight)
    c.gpu_batch = int(gpu_batch)

    def seq(v, default):
        if v is None:
            return [default] * 5
        if isinstance(v, dict):
            return [float(v.get(k, default)) for k in PIPE_OPS]
        return [float(x) for x in v]
    for i, x in enumerate(seq(speedup, 1.0)):
        c.speedup[i] = x
    for i, x in enumerate(seq(transfer_impact, 0.0)):
        c.transfer_impact[i] = x
    for i, x in enumerate(seq(gpu_ms, 0.0)):
        c.gpu_ms[i] = x
    return c


def pipe_outputs(images):
    """Output buffers for recon_pipeline_run (reusable across runs)."""
    import numpy as np
    return [{"objects": np.empty(im.shape, np.uint8), "markers": np.empty(im.shape, np.uint8),
             "labels": np.empty(im.shape, np.int32)} for im in images]


def recon_pipeline_run(ctx, images, cfg: recon_pipe_config, trace: bool = False, outputs=None):
    """Run the tile pipeline on host uint8 numpy images (ctx may be None
    without the GPU).  Returns (outputs, stats): per tile a dict of `objects`,
    `markers` (uint8) and `labels` (int32) numpy arrays and `count` (the
    caller's `outputs`, from pipe_outputs, when given: buffers reused across
    runs); stats as a dict, with `trace` (a list of (tile, op name, device,
    start_ms, end_ms) in the order the devices took the instances; device 0 is
    the GPU, 1 + k CPU worker k) when asked for."""
    import numpy as np
    lib = load_library()
    n = len(images)
    imgs = [np.ascontiguousarray(im, dtype=np.uint8) for im in images]
    if outputs is None:
        outputs = pipe_outputs(imgs)
    if len(outputs) != n:
        raise ValueError("one output dict per image")
    outs = []
    arr = (recon_pipe_tile * max(n, 1))()
    counts = (ctypes.c_int32 * max(n, 1))()
    for i, im in enumerate(imgs):
        if im.ndim != 2:
            raise ValueError("images must be 2-D")
        o = outputs[i]
        for k, dt in (("objects", np.uint8), ("markers", np.uint8), ("labels", np.int32)):
            a = o[k]
            if a.shape != im.shape or a.dtype != dt or not a.flags.c_contiguous:
                raise ValueError("output %s of tile %d must be a C-contiguous %s array of the image's shape"
                                 % (k, i, np.dtype(dt).name))
        outs.append(o)
        t = arr[i]
        t.image = im.ctypes.data
        t.height, t.width = im.shape
        t.pitch = im.strides[0]
        t.objects, t.markers, t.labels = o["objects"].ctypes.data, o["markers"].ctypes.data, o["labels"].ctypes.data
        t.label_pitch = im.shape[1]
        t.count = ctypes.addressof(counts) + 4 * i
    st = recon_pipe_stats()
    events = None
    if trace:
        cap = 5 * max(n, 1)
        events = (recon_pipe_event * cap)()
        cfg = recon_pipe_config.from_buffer_copy(cfg)
        cfg.trace_cap = cap
        cfg.trace = ctypes.cast(events, ctypes.POINTER(recon_pipe_event))
    rc = lib.recon_pipeline_run(ctx, arr, n, ctypes.byref(cfg), ctypes.byref(st))
    _check(rc, lib.recon_pipeline_error().decode(errors="replace"))
    for i, o in enumerate(outs):
        o["count"] = int(counts[i])
    stats = {}
    for f, _ in recon_pipe_stats._fields_:
        v = getattr(st, f)
        stats[f] = list(v) if not isinstance(v, (int, float)) else v
    if trace:
        stats["trace"] = [(e.tile, PIPE_OPS[e.op], e.device, e.start_ms, e.end_ms)
                          for e in events[:st.trace_n]]
    return outs, stats


def recon_pipeline_error() -> str:
    """Message of the calling thread's last failed pipeline call."""
    return load_library().recon_pipeline_error().decode(errors="replace")


def recon_pipeline_host_op(op: str, image, cfg: recon_pipe_config):
    """One operation's CPU variant on a host uint8 numpy image (a copy is
    returned); for "label" returns (labels, count)."""
    import numpy as np
    lib = load_library()
    if op not in PIPE_OPS:
        raise ValueError("op must be one of %s" % ", ".join(PIPE_OPS))
    im = np.array(image, dtype=np.uint8, copy=True, order="C")
    if im.ndim != 2:
        raise ValueError("image must be 2-D")
    ri = recon_image(im.ctypes.data, im.shape[0], im.shape[1], im.strides[0])
    labels = np.empty(im.shape, dtype=np.int32) if op == "label" else None
    cnt = ctypes.c_int32(0)
    rc = lib.recon_pipeline_host_op(PIPE_OPS.index(op), ctypes.byref(ri), ctypes.byref(cfg),
                                    labels.ctypes.data if labels is not None else None,
                                    im.shape[1], ctypes.byref(cnt))
    _check(rc, lib.recon_pipeline_error().decode(errors="replace"))
    return (labels, int(cnt.value)) if op == "label" else im


class Recon:
    """A librecon context on one GPU."""

    def __init__(self, device: int = 0, **cfg):
        self.ctx = recon_create(device, **cfg)
        self.cfg = dict(cfg)
        self._keep = {}

    def close(self):
        if self.ctx:
            recon_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dilate(self, marker, mask, conn: int = 8, stream=None):
        """In place: marker <- reconstruction by dilation of mask from marker."""
        recon_dilate(self.ctx, marker, mask, conn, stream)
        return marker

    def dilate_noalloc(self, marker, mask, conn: int = 8, stream=None):
        """recon_dilate with the library's fixed device workspace (no allocation)."""
        recon_dilate_noalloc(self.ctx, marker, mask, conn, stream)
        return marker

    def fill_holes(self, img, conn: int = 8, stream=None):
        """In place: img <- fill-holes(img) with background connectivity conn."""
        recon_fill_holes(self.ctx, img, conn, stream)
        return img

    def erode(self, marker, mask, conn: int = 8, stream=None):
        """In place: marker <- reconstruction by erosion of mask from marker."""
        recon_erode(self.ctx, marker, mask, conn, stream)
        return marker

    def hdome(self, img, h: int, conn: int = 8, stream=None):
        """In place: img <- img - rho_img(max(img - h, 0))."""
        recon_hdome(self.ctx, img, h, conn, stream)
        return img

    def regional_max(self, img, conn: int = 8, stream=None):
        """In place: img <- 255 on the regional maxima of img, 0 elsewhere."""
        recon_regional_max(self.ctx, img, conn, stream)
        return img

    def label(self, img, labels=None, conn: int = 8, count=None, stream=None):
        """Connected components of img's nonzero pixels into an int32 device plane (allocated if None)."""
        import torch
        if labels is None:
            labels = torch.empty(tuple(img.shape), dtype=torch.int32, device=img.device)
        recon_label(self.ctx, img, labels, conn, count, stream)
        return labels

    def area_threshold(self, img, min_area: int, max_area: int, conn: int = 8, stream=None):
        """In place: img <- 255 on the components with min_area <= area <= max_area, else 0."""
        recon_area_threshold(self.ctx, img, min_area, max_area, conn, stream)
        return img

    def distance(self, img, dist2=None, stream=None):
        """Exact squared Euclidean distance to the nearest 0 pixel, into an int32 plane (allocated if None)."""
        import torch
        if dist2 is None:
            dist2 = torch.empty(tuple(img.shape), dtype=torch.int32, device=img.device)
        recon_distance(self.ctx, img, dist2, stream)
        return dist2

    def pre_watershed(self, img, conn: int = 8, stream=None):
        """In place: img <- 255 on the regional maxima of min(floor(sqrt(dist2)), 255), else 0."""
        recon_pre_watershed(self.ctx, img, conn, stream)
        return img

    def batch(self, tasks, stream=None):
        """tasks: list of dicts {op, image, mask?, conn, h?, scan_rounds?, queue_capacity?,
        block_rows?} of device tensors (results in place)."""
        recon_batch(self.ctx, [make_task(t["op"], t["image"], t.get("mask"), t.get("conn", 8),
                                         t.get("scan_rounds", 0), t.get("queue_capacity", 0), t.get("h", 0),
                                         t.get("block_rows", 0))
                               for t in tasks], stream)

    def submit(self, op, image, mask=None, conn: int = 8, scan_rounds: int = 0, queue_capacity: int = 0,
               h: int = 0) -> int:
        tk = recon_submit(self.ctx, make_task(op, image, mask, conn, scan_rounds, queue_capacity, h))
        self._keep[tk] = (image, mask)
        return tk

    def poll(self, ticket: int) -> bool:
        done = recon_poll(self.ctx, ticket)
        if done:
            self._keep.pop(ticket, None)
        return done

    def wait(self, ticket: int, timeout_us: int = -1):
        recon_wait(self.ctx, ticket, timeout_us)
        self._keep.pop(ticket, None)

    def serve_stop(self):
        recon_serve_stop(self.ctx)

    def serve_stats(self) -> dict:
        return recon_serve_stats(self.ctx)

    def last_stats(self) -> dict:
        return recon_last_stats(self.ctx)

    def launch_times(self, back: int = 0) -> dict:
        """Kernel durations of the launch `back` launches ago (timing contexts)."""
        return recon_launch_times(self.ctx, back)


# Fail loudly at import when the native library is missing.
load_library()
