"""ORACLE -- test infrastructure, not part of the product.

Plain CPU reference for the labeling path (Sec. 4.2, Eq. bool_dot and
Eq. approx; Sec. 4.3, Alg. mat_mul over CSR rows; Sec. 4.1, Alg. zcurve).
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library; the only thing
both sides consume is the input produced by the seeded generator.

Pins (what ties each function to something other than itself) live in
tests/test_oracle_pins.py:
  label_csr    CSR worked example of Sec. 4.3; numpy integer matmul special
               case; dense brute force; algebraic invariants; geometric brute
               force from the footprint and region shapes on tiny grids.
  label_dense  the same pins (it is Eq. bool_dot written out).
  zorder       bit interleaving, exhaustively on 2^1..2^6-sided grids.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the oracle with gcc (plain -O2; no vectorisation pragmas)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-o", _LIB_PATH + ".tmp",
           os.path.join(_HERE, "lbl_oracle.c"), "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    global _lib
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    _lib = _bind(_LIB_PATH)
    return _lib


def _bind(path: str):
    """Load a compiled oracle and declare its C signatures."""
    lib = ctypes.CDLL(path)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    u32 = ctypes.POINTER(ctypes.c_uint32)
    u64 = ctypes.POINTER(ctypes.c_uint64)
    d = ctypes.POINTER(ctypes.c_double)
    lib.oracle_label_csr.restype = ctypes.c_int
    lib.oracle_label_csr.argtypes = [u64, u32, ctypes.c_uint64, u8, ctypes.c_uint32, u64,
                                     ctypes.c_uint64, u8, ctypes.c_int]
    lib.oracle_label_dense.restype = None
    lib.oracle_label_dense.argtypes = [u8, ctypes.c_uint64, ctypes.c_uint64, u8, ctypes.c_uint32, u8]
    lib.oracle_zorder.restype = ctypes.c_uint64
    lib.oracle_zorder.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d]
    lib.oracle_raster_shapes.restype = ctypes.c_int
    lib.oracle_raster_shapes.argtypes = [u32, u32, d, d, d, d, ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32, u8]
    lib.oracle_product_paths.restype = ctypes.c_int
    lib.oracle_product_paths.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u32, u32, u32, u8, ctypes.c_uint32,
                                         ctypes.c_uint32, u8, ctypes.c_uint32, ctypes.c_uint32, u32, u32]
    lib.oracle_scan_lengths.restype = ctypes.c_int
    lib.oracle_scan_lengths.argtypes = [u64, u32, ctypes.c_uint64, u8, ctypes.c_uint32, ctypes.c_uint32,
                                        u64, ctypes.c_uint64, u64]
    return lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def label_csr(row_ptr, col_idx, n_cells: int, O, rows=None, threads: int = 1) -> np.ndarray:
    """L (uint8, len(rows) x n_props) for CSR rows of M against O (n_cells x n_props)."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
    col_idx = np.ascontiguousarray(col_idx, np.uint32)
    O = np.ascontiguousarray(O, np.uint8)
    if O.ndim != 2 or O.shape[0] != n_cells:
        raise ValueError("O must be n_cells x n_props")
    n_traj = len(row_ptr) - 1
    if rows is None:
        rows = np.arange(n_traj, dtype=np.uint64)
    rows = np.ascontiguousarray(rows, np.uint64)
    if len(rows) and int(rows.max()) >= n_traj:
        raise ValueError("row out of range")
    n_props = O.shape[1]
    L = np.empty((len(rows), n_props), np.uint8)
    if len(col_idx) == 0:
        col_idx = np.zeros(1, np.uint32)
    rc = lib.oracle_label_csr(_p(row_ptr, ctypes.c_uint64), _p(col_idx, ctypes.c_uint32), n_cells,
                              _p(O, ctypes.c_uint8), n_props, _p(rows, ctypes.c_uint64), len(rows),
                              _p(L, ctypes.c_uint8), int(threads))
    if rc == -1:
        raise ValueError("column index out of range")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return L


def label_dense(M, O) -> np.ndarray:
    """L for a dense M (n_traj x n_cells) by the triple loop of Eq. bool_dot."""
    lib = _load()
    M = np.ascontiguousarray(M, np.uint8)
    O = np.ascontiguousarray(O, np.uint8)
    n_traj, n_cells = M.shape
    if O.shape[0] != n_cells:
        raise ValueError("shape mismatch")
    L = np.empty((n_traj, O.shape[1]), np.uint8)
    lib.oracle_label_dense(_p(M, ctypes.c_uint8), n_traj, n_cells, _p(O, ctypes.c_uint8),
                           O.shape[1], _p(L, ctypes.c_uint8))
    return L


def zorder(x, lo, hi, d: int) -> int:
    """z-order index of point x in the box [lo, hi] at depth d (Alg. zcurve as read)."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float64)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    k = len(x)
    return int(lib.oracle_zorder(k, d, _p(x, ctypes.c_double), _p(lo, ctypes.c_double),
                                 _p(hi, ctypes.c_double)))


def raster_shapes(kind, prop, cx, cy, a, b, nx: int, ny: int, cell: float, n_props: int) -> np.ndarray:
    """O (n_cells x n_props, row-major cells, 0/1) of proposition shapes by the
    Sec. 4.1 encoding read as positive-area overlap (every cell x every shape)."""
    lib = _load()
    kind = np.ascontiguousarray(kind, np.uint32)
    prop = np.ascontiguousarray(prop, np.uint32)
    cx, cy, a, b = (np.ascontiguousarray(x, np.float64) for x in (cx, cy, a, b))
    n = len(kind)
    if not all(len(x) == n for x in (prop, cx, cy, a, b)):
        raise ValueError("shape arrays differ in length")
    O = np.empty((nx * ny, n_props), np.uint8)
    rc = lib.oracle_raster_shapes(_p(kind, ctypes.c_uint32), _p(prop, ctypes.c_uint32), _p(cx, ctypes.c_double),
                                  _p(cy, ctypes.c_double), _p(a, ctypes.c_double), _p(b, ctypes.c_double), n,
                                  nx, ny, float(cell), n_props, _p(O, ctypes.c_uint8))
    if rc != 0:
        raise ValueError("invalid shape kind or proposition index")
    return O


def scan_lengths(row_ptr, col_idx, n_cells: int, O, prop: int, rows=None) -> np.ndarray:
    """Cells the early-terminating serial scan compares per row (Sec. 5.1):
    first cell shared by the row and proposition prop, plus one; n_cells if
    none is shared."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
    col_idx = np.ascontiguousarray(col_idx, np.uint32)
    O = np.ascontiguousarray(O, np.uint8)
    if O.ndim != 2 or O.shape[0] != n_cells or not 0 <= prop < O.shape[1]:
        raise ValueError("O must be n_cells x n_props and prop one of its columns")
    n_traj = len(row_ptr) - 1
    rows = np.arange(n_traj, dtype=np.uint64) if rows is None else np.ascontiguousarray(rows, np.uint64)
    if len(rows) and int(rows.max()) >= n_traj:
        raise ValueError("row out of range")
    if len(col_idx) == 0:
        col_idx = np.zeros(1, np.uint32)
    out = np.empty(len(rows), np.uint64)
    rc = lib.oracle_scan_lengths(_p(row_ptr, ctypes.c_uint64), _p(col_idx, ctypes.c_uint32), n_cells,
                                 _p(O, ctypes.c_uint8), O.shape[1], prop, _p(rows, ctypes.c_uint64), len(rows),
                                 _p(out, ctypes.c_uint64))
    if rc == -1:
        raise ValueError("column index out of range")
    if rc == -2:
        raise ValueError("column ids must ascend within a row")
    return out


def product_paths(n_vertices: int, src, dst, cost, L, delta, v0: int, q0: int):
    """(dist, pred) on the product of a transition system and a monitor
    (Sec. 3.2), each n_vertices * n_states uint32, index v * n_states + q.
    L: n_edges x n_props labels; delta: n_states << n_props next states
    (>= n_states: no move)."""
    lib = _load()
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    cost = np.ascontiguousarray(cost, np.uint32)
    L = np.ascontiguousarray(L, np.uint8)
    delta = np.ascontiguousarray(delta, np.uint8)
    n_edges = len(src)
    n_props = L.shape[1] if L.ndim == 2 else 1
    n_states = len(delta) >> n_props
    if n_states < 1 or len(delta) != n_states << n_props:
        raise ValueError("delta must hold n_states << n_props entries")
    dist = np.empty(n_vertices * n_states, np.uint32)
    pred = np.empty(n_vertices * n_states, np.uint32)
    keep = [a if len(a) else np.zeros(1, a.dtype) for a in (src, dst, cost)]
    Lk = L if L.size else np.zeros((1, n_props), np.uint8)
    rc = lib.oracle_product_paths(n_vertices, n_edges, _p(keep[0], ctypes.c_uint32), _p(keep[1], ctypes.c_uint32),
                                  _p(keep[2], ctypes.c_uint32), _p(Lk, ctypes.c_uint8), n_props, n_states,
                                  _p(delta, ctypes.c_uint8), v0, q0, _p(dist, ctypes.c_uint32),
                                  _p(pred, ctypes.c_uint32))
    if rc == -1:
        raise ValueError("edge vertex out of range or zero cost")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return dist, pred
