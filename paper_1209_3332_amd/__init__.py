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
``Recon`` wraps a context for convenience.
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
    "recon_launch_times", "recon_last_error",
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
                ("h", ctypes.c_int32)]


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
    F = ctypes.POINTER(ctypes.c_float)
    lib.recon_launch_times.argtypes = [P, ctypes.c_int, F, F, F, F, F]
    lib.recon_last_error.argtypes = []
    lib.recon_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "recon_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc == RECON_OK:
        return
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
              h: int = 0) -> recon_task:
    """recon_task for op in OPS; `mask` for dilate / erode, `h` for hdome."""
    if op not in OPS:
        raise ValueError("op must be one of %s" % ", ".join(OPS))
    t = recon_task()
    t.op = OPS[op]
    t.scan_rounds = int(scan_rounds)
    t.queue_capacity = int(queue_capacity)
    t.conn = int(conn)
    t.h = int(h)
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


def recon_last_error() -> str:
    return load_library().recon_last_error().decode(errors="replace")


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
        """tasks: list of dicts {op, image, mask?, conn, h?} of device tensors (results in place)."""
        recon_batch(self.ctx, [make_task(t["op"], t["image"], t.get("mask"), t.get("conn", 8),
                                         t.get("scan_rounds", 0), t.get("queue_capacity", 0), t.get("h", 0))
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
