"""ctypes binding of liblbl.so: the C ABI declared in include/lbl.h, with the
same names and argument marshalling only.  Every step of the labeling path
runs in the HIP library; nothing here computes labels.

Buffers may be torch tensors (their data_ptr is passed), numpy arrays (host
memory) or raw integer addresses.  Streams may be torch streams, raw
hipStream_t integers or None (the current torch stream when torch is loaded,
else the default stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbl.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUSY, ETIMEDOUT, ECLOSED = range(7)
STATUS_NAMES = {0: "LBL_OK", 1: "LBL_EINVAL", 2: "LBL_ENOMEM", 3: "LBL_EDEVICE", 4: "LBL_EBUSY",
                5: "LBL_ETIMEDOUT", 6: "LBL_ECLOSED"}

ROW_MAJOR = 0
MORTON = 1
LOAD_KEEP_INT8 = 0x1
LOAD_INPUT_DEVICE = 0x2
LOAD_NO_SPARSE = 0x4
LOAD_SPARSE_ONLY = 0x8
HOST_PTRS = 0x1
KERNEL_AUTO = 0x00
KERNEL_BITS = 0x10
KERNEL_MFMA = 0x20
KERNEL_MFMA_I8 = 0x40
KERNEL_SPARSE = 0x80
BATCH_MAX_PROPS = 1024

EXPORTS = (
    "lbl_load_abstraction", "lbl_load_abstraction_dense", "lbl_free_abstraction", "lbl_abstraction_info",
    "lbl_label_frame", "lbl_label_batch", "lbl_tune", "lbl_tune_batch", "lbl_tune_save", "lbl_tune_load", "lbl_tune_describe",
    "lbl_serve_start", "lbl_serve_submit", "lbl_serve_wait", "lbl_serve_stats_get", "lbl_serve_stop",
    "lbl_cell_position", "lbl_last_error", "lbl_version", "lbl_profile_enable", "lbl_profile_read",
    "lbl_raster_frame", "lbl_product_shortest_paths", "lbl_tune_batch_describe", "lbl_label_frame_noalloc",
)


class LblError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("cell_m", ctypes.c_float),
                ("cell_order", ctypes.c_uint32)]


class AbsInfo(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_uint64), ("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32),
                ("n_words", ctypes.c_uint32), ("row_stride", ctypes.c_uint32), ("bits_bytes", ctypes.c_uint64),
                ("int8_bytes", ctypes.c_uint64), ("nonzero_words", ctypes.c_uint64), ("set_cells", ctypes.c_uint64),
                ("sparse_entries", ctypes.c_uint64), ("sparse_bytes", ctypes.c_uint64),
                ("sparse_frame_bytes", ctypes.c_uint64), ("sparse_tiles", ctypes.c_uint32),
                ("sparse_row_block", ctypes.c_uint32), ("sparse_frame_bytes_narrow", ctypes.c_uint64),
                ("sparse_tiles_narrow", ctypes.c_uint32), ("sparse_tiles_direct", ctypes.c_uint32),
                ("sparse_frame_bytes_direct", ctypes.c_uint64)]


class Job(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("O", ctypes.c_void_p), ("n_props", ctypes.c_uint32),
                ("L", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [("pack_launches", ctypes.c_uint64), ("label_launches", ctypes.c_uint64),
                ("batch_launches", ctypes.c_uint64), ("emit_launches", ctypes.c_uint64),
                ("pack_ms", ctypes.c_double), ("label_ms", ctypes.c_double),
                ("batch_ms", ctypes.c_double), ("emit_ms", ctypes.c_double)]


class ServeCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_batch_frames", ctypes.c_uint32),
                ("max_wait_us", ctypes.c_uint32), ("max_queue", ctypes.c_uint32), ("n_streams", ctypes.c_uint32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("pairs", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double), ("pairs_per_s", ctypes.c_double),
                ("max_in_flight", ctypes.c_uint64), ("budget_high_water", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def library_path() -> str:
    return LIB_PATH


def lib():
    """The loaded library.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1810_02612_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    sig = {
        "lbl_load_abstraction": [ctypes.POINTER(Grid), u64, vp, vp, u32, ctypes.POINTER(vp)],
        "lbl_load_abstraction_dense": [ctypes.POINTER(Grid), u64, vp, u32, ctypes.POINTER(vp)],
        "lbl_free_abstraction": [vp],
        "lbl_abstraction_info": [vp, ctypes.POINTER(AbsInfo)],
        "lbl_label_frame": [vp, vp, u32, vp, u32, vp],
        "lbl_label_frame_noalloc": [vp, vp, u32, vp, vp],
        "lbl_label_batch": [ctypes.POINTER(Job), ctypes.c_size_t, u32, vp],
        "lbl_tune": [vp, vp, u32, u32, vp],
        "lbl_tune_batch": [ctypes.POINTER(Job), ctypes.c_size_t, vp],
        "lbl_tune_save": [ctypes.c_char_p],
        "lbl_tune_load": [ctypes.c_char_p],
        "lbl_tune_describe": [vp, u32, ctypes.c_char_p, ctypes.c_size_t],
        "lbl_tune_batch_describe": [ctypes.POINTER(Job), ctypes.c_size_t, vp, ctypes.c_char_p, ctypes.c_size_t],
        "lbl_serve_start": [ctypes.POINTER(ServeCfg), ctypes.POINTER(vp)],
        "lbl_serve_submit": [vp, vp, vp, u32, vp, ctypes.POINTER(u64)],
        "lbl_serve_wait": [vp, u64, i64],
        "lbl_serve_stats_get": [vp, ctypes.POINTER(ServeStats)],
        "lbl_serve_stop": [vp],
        "lbl_cell_position": [ctypes.POINTER(Grid), u32, ctypes.POINTER(u32), ctypes.POINTER(u32)],
        "lbl_profile_enable": [ctypes.c_int],
        "lbl_profile_read": [ctypes.POINTER(Profile)],
        "lbl_raster_frame": [ctypes.POINTER(Grid), ctypes.c_double, vp, u64, u32, vp, vp],
        "lbl_product_shortest_paths": [u64, u64, vp, vp, vp, vp, u32, u32, u32, vp, u32, u32, vp, vp,
                                       ctypes.POINTER(ctypes.c_uint32), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.lbl_last_error.restype = ctypes.c_char_p
    L.lbl_last_error.argtypes = []
    L.lbl_version.restype = ctypes.c_char_p
    L.lbl_version.argtypes = []
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise LblError(status, lib().lbl_last_error().decode())


def _addr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("numpy buffers must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if hasattr(x, "is_contiguous") and not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr()
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s) -> int | None:
    if s is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def version() -> str:
    return lib().lbl_version().decode()


def last_error() -> str:
    return lib().lbl_last_error().decode()


def _grid(nx, ny, cell_m=0.0, cell_order=ROW_MAJOR):
    return Grid(int(nx), int(ny), float(cell_m), int(cell_order))


def load_abstraction(nx: int, ny: int, row_ptr, col_idx, flags: int = 0, cell_m: float = 0.0,
                     cell_order: int = ROW_MAJOR) -> int:
    """Returns an lbl_abs_t handle (int).  row_ptr/col_idx: numpy (host) or,
    with LOAD_INPUT_DEVICE, device tensors.  cell_order: how col_idx (and
    later the rows of O) number the cells, ROW_MAJOR or MORTON."""
    if isinstance(row_ptr, np.ndarray):
        row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
        col_idx = np.ascontiguousarray(col_idx, np.uint32)
        n_traj = len(row_ptr) - 1
    else:
        n_traj = row_ptr.numel() - 1
    h = ctypes.c_void_p()
    g = _grid(nx, ny, cell_m, cell_order)
    _check(lib().lbl_load_abstraction(ctypes.byref(g), n_traj, _addr(row_ptr), _addr(col_idx), flags,
                                      ctypes.byref(h)))
    return h.value


def load_abstraction_dense(nx: int, ny: int, T, flags: int = 0, cell_m: float = 0.0,
                           cell_order: int = ROW_MAJOR) -> int:
    if isinstance(T, np.ndarray):
        T = np.ascontiguousarray(T, np.uint8)
    n_traj = T.shape[0]
    h = ctypes.c_void_p()
    g = _grid(nx, ny, cell_m, cell_order)
    _check(lib().lbl_load_abstraction_dense(ctypes.byref(g), n_traj, _addr(T), flags, ctypes.byref(h)))
    return h.value


def free_abstraction(a: int) -> None:
    _check(lib().lbl_free_abstraction(a))


def abstraction_info(a: int) -> dict:
    info = AbsInfo()
    _check(lib().lbl_abstraction_info(a, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in AbsInfo._fields_}


def label_frame(a: int, O, n_props: int, L, flags: int = 0, stream=None) -> None:
    _check(lib().lbl_label_frame(a, _addr(O), n_props, _addr(L), flags, _stream(stream)))


def label_frame_noalloc(a: int, O, n_props: int, L, stream=None) -> None:
    """lbl_label_frame_noalloc: device O and L; intermediates in the library's
    static device array (no allocation)."""
    _check(lib().lbl_label_frame_noalloc(a, _addr(O), n_props, _addr(L), _stream(stream)))


SHAPE_RECT, SHAPE_DISC = 0, 1
# lbl_shape: kind, prop, cx, cy, a, b (40 bytes, no padding)
SHAPE_DTYPE = np.dtype([("kind", "<u4"), ("prop", "<u4"), ("cx", "<f8"), ("cy", "<f8"), ("a", "<f8"), ("b", "<f8")])


def shapes_array(kind, prop, cx, cy, a, b) -> np.ndarray:
    """Host lbl_shape records from parallel arrays."""
    n = len(kind)
    out = np.zeros(n, SHAPE_DTYPE)
    for name, v in (("kind", kind), ("prop", prop), ("cx", cx), ("cy", cy), ("a", a), ("b", b)):
        out[name] = np.asarray(v)
    return out


def raster_frame(nx: int, ny: int, cell_m: float, shapes: np.ndarray, n_props: int, O, stream=None,
                 cell_order: int = ROW_MAJOR) -> None:
    """Rasterize proposition shapes (a SHAPE_DTYPE host array) into the device
    frame O (n_cells x n_props bytes, cells numbered in cell_order)."""
    shapes = np.ascontiguousarray(shapes, SHAPE_DTYPE)
    g = _grid(nx, ny, cell_m, cell_order)
    ptr = shapes.ctypes.data if len(shapes) else None
    _check(lib().lbl_raster_frame(ctypes.byref(g), float(cell_m), ptr, len(shapes), n_props, _addr(O),
                                  _stream(stream)))


MONITOR_REJECT = 0xFF


def product_shortest_paths(n_vertices: int, src, dst, cost, L, n_props: int, delta, v0: int, q0: int, dist, pred,
                           stream=None, l_stride: int | None = None) -> int:
    """Least-cost paths on the product of the transition system (device
    src/dst/cost/L arrays; L rows of l_stride bytes, default n_props, of
    which the first n_props are read) and a monitor (host delta table,
    n_states << n_props bytes) into device dist/pred arrays (n_vertices *
    n_states uint32); returns the number of relaxation sweeps."""
    delta = np.ascontiguousarray(delta, np.uint8)
    n_states = len(delta) >> n_props
    sweeps = ctypes.c_uint32(0)
    n_edges = src.numel() if hasattr(src, "numel") else len(src)
    _check(lib().lbl_product_shortest_paths(n_vertices, n_edges, _addr(src), _addr(dst), _addr(cost), _addr(L),
                                            n_props if l_stride is None else l_stride, n_props, n_states,
                                            delta.ctypes.data, v0, q0, _addr(dist), _addr(pred),
                                            ctypes.byref(sweeps), _stream(stream)))
    return sweeps.value


def label_batch(jobs, flags: int = 0, stream=None) -> None:
    """jobs: sequence of (abstraction, O, n_props, L)."""
    _check(lib().lbl_label_batch(_jobs(jobs), len(jobs), flags, _stream(stream)))


def tune(a: int, O_sample, n_props: int, density_pct: int = 10, stream=None) -> None:
    _check(lib().lbl_tune(a, _addr(O_sample), n_props, density_pct, _stream(stream)))


def _jobs(jobs):
    arr = (Job * len(jobs))()
    for i, (a, O, n_props, L) in enumerate(jobs):
        arr[i] = Job(a, _addr(O), int(n_props), _addr(L))
    return arr


def tune_batch(jobs, stream=None) -> None:
    _check(lib().lbl_tune_batch(_jobs(jobs), len(jobs), _stream(stream)))


def tune_batch_describe(jobs, stream=None) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().lbl_tune_batch_describe(_jobs(jobs), len(jobs), _stream(stream), buf, len(buf)))
    return buf.value.decode()


def tune_save(path: str) -> None:
    _check(lib().lbl_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _check(lib().lbl_tune_load(path.encode()))


def tune_describe(a: int, n_props: int) -> str:
    buf = ctypes.create_string_buffer(256)
    _check(lib().lbl_tune_describe(a, n_props, buf, len(buf)))
    return buf.value.decode()


def serve_start(hbm_budget_bytes: int = 2 << 30, max_batch_frames: int = 16, max_wait_us: int = 200,
                max_queue: int = 4096, n_streams: int = 2) -> int:
    cfg = ServeCfg(hbm_budget_bytes, max_batch_frames, max_wait_us, max_queue, n_streams)
    h = ctypes.c_void_p()
    _check(lib().lbl_serve_start(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def serve_submit(s: int, a: int, O, n_props: int, L) -> int:
    t = ctypes.c_uint64()
    _check(lib().lbl_serve_submit(s, a, _addr(O), n_props, _addr(L), ctypes.byref(t)))
    return t.value


def serve_wait(s: int, ticket: int, timeout_us: int = -1) -> int:
    """Returns the status (OK, ETIMEDOUT, or the request's error)."""
    return lib().lbl_serve_wait(s, ticket, timeout_us)


def serve_stats(s: int) -> dict:
    st = ServeStats()
    _check(lib().lbl_serve_stats_get(s, ctypes.byref(st)))
    return st.as_dict()


def serve_stop(s: int) -> None:
    _check(lib().lbl_serve_stop(s))


def cell_position(nx: int, ny: int, cell: int, cell_order: int = ROW_MAJOR) -> tuple[int, int]:
    w, b = ctypes.c_uint32(), ctypes.c_uint32()
    g = _grid(nx, ny, 0.0, cell_order)
    _check(lib().lbl_cell_position(ctypes.byref(g), cell, ctypes.byref(w), ctypes.byref(b)))
    return w.value, b.value


def profile_enable(on: bool = True) -> None:
    _check(lib().lbl_profile_enable(1 if on else 0))


def profile_read() -> dict:
    p = Profile()
    _check(lib().lbl_profile_read(ctypes.byref(p)))
    return {k: getattr(p, k) for k, _ in Profile._fields_}
