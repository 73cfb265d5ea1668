"""Seeded synthetic inputs for the labeling path.

This module makes inputs only: the trajectory-by-cell matrix T (CSR, cell ids
row-major) and per-frame cell-by-proposition maps O (uint8).  It holds none of
the labeling arithmetic (no product of T with O), so both the oracle and the
GPU library can consume what it produces.

The paper's roadmap and freeway scenario are not available; these are
stand-ins with the shapes of its workload (Sec. 5): a fixed set of
trajectories in the agent's body frame, swept by a car footprint and encoded
as binary vectors over an occupancy grid (Sec. 4.1), and proposition regions
encoded the same way.

Recipe (every draw comes from numpy's default_rng seeded with a list that
starts with 181002612):
  T   seed [181002612, cfg, abstraction, 1, 0]
      start (x0, y0) ~ U(extent), heading ~ U[-pi, pi), arcs with curvature
      ~ U[-0.2, 0.2] 1/m, clothoids with end curvatures ~ U[-0.2, 0.2] 1/m,
      length ~ U[len_lo, len_hi]; poses every res/4 plus the endpoint; a
      4.5 m x 2.0 m footprint centred on each pose; conservative raster.
  O   seed [181002612, cfg, abstraction, 2, frame]
      every proposition is a union of n_s ~ U{1..10} shapes, each an
      axis-aligned rectangle (aspect ~ U[0.5, 2]) or a disc with probability
      1/2, centred ~ U(extent), of area -ln(1 - rho) * A / n_s for target
      cell density rho.
  Time-augmented workload (Sec. 5: the plane and time, 2^21 cells)
      grid 128 x 128 cells of 0.5 m and 128 layers of 0.1 s, flattened to a
      128 x 16384 grid (cell id = (layer * 128 + iy) * 128 + ix); a circular
      road of centre radius 20 m and half width 2 m around the grid centre.
  T   seed [181002612, 300, 1, 0]; roadmap vertices on the road (angle
      ~ U[0, 2 pi), radius 20 + U(-0.75, 0.75) m, heading along the road
      + N(0, 0.05), start layer ~ U{0..116}), 8 transitions per vertex
      (speed ~ U[4, 12] m/s, curvature 1/radius + U(-0.02, 0.02) 1/m,
      duration 6 + Binomial(6, 0.455) layers), vertices in order of start layer, then
      angle; the car footprint at each layer's pose.
  O   seed [181002612, 300, 2, frame]; proposition 0 (moving vehicle): three
      other cars circling the road (radius 20 + U(-0.75, 0.75) m, speed
      ~ U[5, 12] m/s, either direction) over all layers; proposition 1 (not
      nominal lane): every cell meeting the plane outside the road, in every
      layer.
  Bernoulli T and O (Sec. 5.1's random subsets): each cell of each row, and
      each (cell, proposition), set independently with the given bias.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None

SEED0 = 181002612
FOOT_LEN = 4.5
FOOT_WID = 2.0


def build() -> str:
    """Compile the C geometry helper in place (gcc, -O2)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-o", _LIB_PATH + ".tmp",
           os.path.join(_HERE, "raster.c"), "-lm", "-lpthread"]
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
    lib = ctypes.CDLL(_LIB_PATH)
    d = ctypes.POINTER(ctypes.c_double)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    u32 = ctypes.POINTER(ctypes.c_uint32)
    u64 = ctypes.POINTER(ctypes.c_uint64)
    lib.gen_raster.restype = ctypes.c_void_p
    lib.gen_raster.argtypes = [d, d, d, d, d, d, u8, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, u64, u64]
    lib.gen_raster_fill.restype = None
    lib.gen_raster_fill.argtypes = [ctypes.c_void_p, u32]
    lib.gen_raster_free.restype = None
    lib.gen_raster_free.argtypes = [ctypes.c_void_p]
    lib.gen_traj_poses.restype = ctypes.c_uint64
    lib.gen_traj_poses.argtypes = [d, d, d, d, d, d, u8, ctypes.c_uint64, ctypes.c_double,
                                   d, ctypes.c_uint64]
    lib.gen_spacetime.restype = ctypes.c_void_p
    lib.gen_spacetime.argtypes = [d, d, d, d, d, u32, u32, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, u64, u64]
    lib.gen_raster_shapes.restype = None
    lib.gen_raster_shapes.argtypes = [u8, d, d, d, d, u32, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_double, ctypes.c_uint32, u8]
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


@dataclasses.dataclass
class Trajectories:
    """Parameters of N_t trajectories (one per row of T)."""
    x0: np.ndarray
    y0: np.ndarray
    th0: np.ndarray
    k0: np.ndarray
    k1: np.ndarray
    length: np.ndarray
    kind: np.ndarray  # uint8: 0 arc, 1 clothoid

    def __len__(self):
        return len(self.x0)


@dataclasses.dataclass
class Grid:
    n: int          # cells per side (nx == ny == n)
    res: float      # cell side in metres

    @property
    def n_cells(self) -> int:
        return self.n * self.n

    @property
    def extent(self) -> float:
        return self.n * self.res


@dataclasses.dataclass
class Abstraction:
    """T in CSR form over row-major cell ids, plus what made it."""
    grid: Grid
    row_ptr: np.ndarray   # uint64, N_t + 1
    col_idx: np.ndarray   # uint32, row_ptr[-1]; ascending within a row
    traj: Trajectories | None = None

    @property
    def n_traj(self) -> int:
        return len(self.row_ptr) - 1

    def dense(self) -> np.ndarray:
        """uint8 N_t x N_c matrix (small cases only)."""
        T = np.zeros((self.n_traj, self.grid.n_cells), np.uint8)
        rows = np.repeat(np.arange(self.n_traj), np.diff(self.row_ptr).astype(np.int64))
        T[rows, self.col_idx.astype(np.int64)] = 1
        return T


def draw_trajectories(rng, n_traj: int, grid: Grid, len_lo: float, len_hi: float,
                      clothoid_frac: float) -> Trajectories:
    ext = grid.extent
    x0 = rng.uniform(0.0, ext, n_traj)
    y0 = rng.uniform(0.0, ext, n_traj)
    th0 = rng.uniform(-math.pi, math.pi, n_traj)
    k0 = rng.uniform(-0.2, 0.2, n_traj)
    k1 = rng.uniform(-0.2, 0.2, n_traj)
    length = rng.uniform(len_lo, len_hi, n_traj)
    kind = (rng.random(n_traj) < clothoid_frac).astype(np.uint8)
    return Trajectories(x0, y0, th0, k0, k1, length, kind)


def raster_trajectories(tr: Trajectories, grid: Grid, threads: int | None = None) -> Abstraction:
    lib = _load()
    n_traj = len(tr)
    cols = [np.ascontiguousarray(a, np.float64) for a in (tr.x0, tr.y0, tr.th0, tr.k0, tr.k1, tr.length)]
    kind = np.ascontiguousarray(tr.kind, np.uint8)
    counts = np.zeros(n_traj, np.uint64)
    total = np.zeros(1, np.uint64)
    h = lib.gen_raster(*[_ptr(c, ctypes.c_double) for c in cols], _ptr(kind, ctypes.c_uint8),
                       n_traj, grid.n, grid.res, grid.res / 4.0, FOOT_LEN, FOOT_WID,
                       threads or _threads(), _ptr(counts, ctypes.c_uint64),
                       _ptr(total, ctypes.c_uint64))
    if not h:
        raise MemoryError("rasterizer failed")
    try:
        col_idx = np.empty(int(total[0]), np.uint32)
        lib.gen_raster_fill(h, _ptr(col_idx, ctypes.c_uint32))
    finally:
        lib.gen_raster_free(h)
    row_ptr = np.zeros(n_traj + 1, np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return Abstraction(grid, row_ptr, col_idx, tr)


def trajectory_poses(tr: Trajectories, t: int, grid: Grid) -> np.ndarray:
    """Sampled poses (x, y, heading) of trajectory t, shape (n, 3)."""
    lib = _load()
    cols = [np.ascontiguousarray(a, np.float64) for a in (tr.x0, tr.y0, tr.th0, tr.k0, tr.k1, tr.length)]
    kind = np.ascontiguousarray(tr.kind, np.uint8)
    ds = grid.res / 4.0
    cap = int(tr.length[t] / ds) + 4
    out = np.empty((cap, 3), np.float64)
    n = lib.gen_traj_poses(*[_ptr(c, ctypes.c_double) for c in cols], _ptr(kind, ctypes.c_uint8),
                           t, ds, _ptr(out, ctypes.c_double), cap)
    assert n <= cap
    return out[:n].copy()


@dataclasses.dataclass
class Shapes:
    """Proposition regions: kind 0 rectangle (half sizes a, b), 1 disc (radius a)."""
    kind: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    a: np.ndarray
    b: np.ndarray
    prop: np.ndarray


def draw_shapes(rng, grid: Grid, rhos) -> Shapes:
    """One union of 1..10 shapes per proposition; rhos gives each target density."""
    A = grid.extent ** 2
    kinds, cxs, cys, As, Bs, props = [], [], [], [], [], []
    for p, rho in enumerate(rhos):
        n_s = int(rng.integers(1, 11))
        area = -math.log1p(-float(rho)) * A / n_s
        for _ in range(n_s):
            disc = rng.random() < 0.5
            cx = rng.uniform(0.0, grid.extent)
            cy = rng.uniform(0.0, grid.extent)
            if disc:
                r = math.sqrt(area / math.pi)
                kinds.append(1); As.append(r); Bs.append(r)
            else:
                aspect = rng.uniform(0.5, 2.0)
                h = math.sqrt(area / aspect)
                w = aspect * h
                kinds.append(0); As.append(0.5 * w); Bs.append(0.5 * h)
            cxs.append(cx); cys.append(cy); props.append(p)
    return Shapes(np.array(kinds, np.uint8), np.array(cxs), np.array(cys), np.array(As),
                  np.array(Bs), np.array(props, np.uint32))


def raster_shapes(sh: Shapes, grid: Grid, n_props: int) -> np.ndarray:
    """uint8 O of shape (N_c, n_props), cell-major, values 0/1."""
    lib = _load()
    O = np.zeros((grid.n_cells, n_props), np.uint8)
    args = [np.ascontiguousarray(x) for x in (sh.kind, sh.cx, sh.cy, sh.a, sh.b, sh.prop)]
    lib.gen_raster_shapes(_ptr(args[0], ctypes.c_uint8), _ptr(args[1], ctypes.c_double),
                          _ptr(args[2], ctypes.c_double), _ptr(args[3], ctypes.c_double),
                          _ptr(args[4], ctypes.c_double), _ptr(args[5], ctypes.c_uint32),
                          len(sh.kind), grid.n, grid.res, n_props, _ptr(O, ctypes.c_uint8))
    return O


# --------------------------------------------------------------------------
# Workload configurations (sizes of the paper-shaped stand-ins)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Config:
    cfg: int
    n_traj: int
    n: int
    res: float
    n_props: int
    len_lo: float
    len_hi: float
    clothoid_frac: float
    rho_lo: float
    rho_hi: float


CONFIGS = {
    # 1k arcs on 64x64 (0.5 m), 8 propositions
    1: Config(1, 1000, 64, 0.5, 8, 5.0, 30.0, 0.0, 0.05, 0.20),
    # 50k arcs + clothoids on 256x256 (0.25 m), 32 propositions
    2: Config(2, 50000, 256, 0.25, 32, 2.0, 60.0, 0.5, 0.05, 0.20),
    # 200k arcs + clothoids on 512x512 (0.2 m), 64 propositions, fixed rho per run
    3: Config(3, 200000, 512, 0.2, 64, 2.0, 60.0, 0.5, 0.01, 0.01),
}

# six uneven abstractions, each side paired with a resolution covering ~102.4 m
BATCH_ROWS = (10000, 25000, 50000, 100000, 150000, 200000)
BATCH_SIDES = (128, 128, 256, 256, 512, 512)
BATCH_RES = {128: 0.8, 256: 0.4, 512: 0.2}


def make_abstraction(cfg: int, abstraction: int = 0, n_traj: int | None = None,
                     n: int | None = None, res: float | None = None,
                     threads: int | None = None) -> Abstraction:
    """T of a configuration; n_traj/n/res override the configuration's sizes."""
    c = CONFIGS[cfg if cfg in CONFIGS else 2]
    grid = Grid(n or c.n, res or c.res)
    rng = np.random.default_rng([SEED0, cfg, abstraction, 1, 0])
    tr = draw_trajectories(rng, n_traj or c.n_traj, grid, c.len_lo, c.len_hi, c.clothoid_frac)
    return raster_trajectories(tr, grid, threads)


def make_frame(cfg: int, grid: Grid, n_props: int, frame: int, abstraction: int = 0,
               rho: float | None = None, rho_lo: float = 0.05, rho_hi: float = 0.20) -> np.ndarray:
    """O of one frame.  rho fixes every proposition's target density, else
    each is drawn from U[rho_lo, rho_hi]."""
    rng = np.random.default_rng([SEED0, cfg, abstraction, 2, frame])
    if rho is None:
        rhos = rng.uniform(rho_lo, rho_hi, n_props)
    else:
        rhos = np.full(n_props, float(rho))
    sh = draw_shapes(rng, grid, rhos)
    return raster_shapes(sh, grid, n_props)


def frame_shapes(cfg: int, grid: Grid, n_props: int, frame: int, abstraction: int = 0,
                 rho: float | None = None, rho_lo: float = 0.05, rho_hi: float = 0.20) -> Shapes:
    rng = np.random.default_rng([SEED0, cfg, abstraction, 2, frame])
    if rho is None:
        rhos = rng.uniform(rho_lo, rho_hi, n_props)
    else:
        rhos = np.full(n_props, float(rho))
    return draw_shapes(rng, grid, rhos)


def batch_layout(cfg: int = 4):
    """(n_traj, side, res) of the six uneven abstractions, seeded permutation."""
    rng = np.random.default_rng([SEED0, cfg, 0, 0, 0])
    rows = rng.permutation(np.array(BATCH_ROWS))
    sides = rng.permutation(np.array(BATCH_SIDES))
    return [(int(r), int(s), BATCH_RES[int(s)]) for r, s in zip(rows, sides)]


def make_batch_abstraction(i: int, cfg: int = 4, scale: float = 1.0,
                           threads: int | None = None) -> Abstraction:
    n_traj, side, res = batch_layout(cfg)[i]
    n_traj = max(1, int(round(n_traj * scale)))
    grid = Grid(side, res)
    c = CONFIGS[2]
    rng = np.random.default_rng([SEED0, cfg, i, 1, 0])
    tr = draw_trajectories(rng, n_traj, grid, c.len_lo, c.len_hi, c.clothoid_frac)
    return raster_trajectories(tr, grid, threads)


def batch_frame_props(cfg: int, abstraction: int, frame: int, lo: int = 4, hi: int = 64) -> int:
    rng = np.random.default_rng([SEED0, cfg, abstraction, 3, frame])
    return int(rng.integers(lo, hi + 1))


# ---------------------------------------------------------------- time-augmented workload

@dataclasses.dataclass
class SpaceTimeGrid:
    """The plane (n x n cells of side res) times n_tau layers of dt seconds,
    flattened to an nx x ny grid with ny = n * n_tau."""
    n: int = 128
    n_tau: int = 128
    res: float = 0.5
    dt: float = 0.1

    @property
    def nx(self) -> int:
        return self.n

    @property
    def ny(self) -> int:
        return self.n * self.n_tau

    @property
    def n_cells(self) -> int:
        return self.n * self.n * self.n_tau

    @property
    def extent(self) -> float:
        return self.n * self.res


ROAD_RADIUS = 20.0      # m, centre line of the circular road (grid of 64 m)
ROAD_HALF_WIDTH = 2.0   # m
TRANSITIONS_PER_VERTEX = 8
ST_SEED = 300


def _road_centre(g: SpaceTimeGrid):
    return 0.5 * g.extent, 0.5 * g.extent


def _spacetime_cells(g: SpaceTimeGrid, x0, y0, th0, k, v, tau0, dur, threads=None):
    lib = _load()
    n = len(x0)
    arrs = [np.ascontiguousarray(a, np.float64) for a in (x0, y0, th0, k, v)]
    t0 = np.ascontiguousarray(tau0, np.uint32)
    du = np.ascontiguousarray(dur, np.uint32)
    counts = np.zeros(n, np.uint64)
    total = ctypes.c_uint64(0)
    h = lib.gen_spacetime(*[_ptr(a, ctypes.c_double) for a in arrs], _ptr(t0, ctypes.c_uint32),
                          _ptr(du, ctypes.c_uint32), n, g.n, g.n_tau, g.res, g.dt, FOOT_LEN, FOOT_WID,
                          threads or _threads(), _ptr(counts, ctypes.c_uint64), ctypes.byref(total))
    if not h:
        raise MemoryError("gen_spacetime failed")
    try:
        col = np.empty(int(total.value), np.uint32)
        lib.gen_raster_fill(h, _ptr(col, ctypes.c_uint32))
    finally:
        lib.gen_raster_free(h)
    row_ptr = np.zeros(n + 1, np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, col


def draw_transitions(rng, n_traj: int, g: SpaceTimeGrid) -> dict:
    """Roadmap transitions on the circular road, ordered by source vertex."""
    per = TRANSITIONS_PER_VERTEX
    n_v = -(-n_traj // per)
    cx, cy = _road_centre(g)
    phi = rng.uniform(0.0, 2 * math.pi, n_v)
    r = ROAD_RADIUS + rng.uniform(-0.75, 0.75, n_v)
    head = phi + 0.5 * math.pi + rng.normal(0.0, 0.05, n_v)
    tau_v = rng.integers(0, max(1, g.n_tau - 12 + 1), n_v)  # layers past the grid are dropped
    order = np.lexsort((phi, tau_v))
    phi, r, head, tau_v = phi[order], r[order], head[order], tau_v[order]
    n = n_v * per
    v = rng.uniform(4.0, 12.0, n)
    k = np.repeat(1.0 / r, per) + rng.uniform(-0.02, 0.02, n)
    dur = 6 + rng.binomial(6, 0.455, n)
    tr = dict(x0=np.repeat(cx + r * np.cos(phi), per), y0=np.repeat(cy + r * np.sin(phi), per),
              th0=np.repeat(head, per), k=k, v=v, tau0=np.repeat(tau_v, per), dur=dur)
    return {key: a[:n_traj] for key, a in tr.items()}


def spacetime_abstraction(n_traj: int, g: SpaceTimeGrid | None = None, threads: int | None = None,
                          shuffle_rows: bool = False) -> Abstraction:
    """T of n_traj roadmap transitions in the time-augmented workspace, rows
    in order of source vertex, or in a seeded random order."""
    g = g or SpaceTimeGrid()
    rng = np.random.default_rng([SEED0, ST_SEED, 1, 0])
    tr = draw_transitions(rng, n_traj, g)
    if shuffle_rows:
        perm = np.random.default_rng([SEED0, ST_SEED, 5, 0]).permutation(n_traj)
        tr = {key: a[perm] for key, a in tr.items()}
    row_ptr, col = _spacetime_cells(g, tr["x0"], tr["y0"], tr["th0"], tr["k"], tr["v"], tr["tau0"], tr["dur"],
                                    threads)
    return Abstraction(grid=g, row_ptr=row_ptr, col_idx=col)


def off_road_mask(g: SpaceTimeGrid) -> np.ndarray:
    """n x n bool: plane cells meeting the region outside the road with
    positive area (nearest point inside the inner circle, or farthest point
    outside the outer one)."""
    cx, cy = _road_centre(g)
    lo = np.arange(g.n) * g.res
    X0, Y0 = np.meshgrid(lo, lo)  # [iy, ix]
    X1, Y1 = X0 + g.res, Y0 + g.res
    near = np.hypot(np.maximum(np.maximum(X0 - cx, cx - X1), 0.0), np.maximum(np.maximum(Y0 - cy, cy - Y1), 0.0))
    far = np.hypot(np.maximum(abs(X0 - cx), abs(X1 - cx)), np.maximum(abs(Y0 - cy), abs(Y1 - cy)))
    return (near < ROAD_RADIUS - ROAD_HALF_WIDTH) | (far > ROAD_RADIUS + ROAD_HALF_WIDTH)


def spacetime_frame(g: SpaceTimeGrid | None = None, frame: int = 0, n_agents: int = 3) -> np.ndarray:
    """O (n_cells x 2 uint8): proposition 0 moving vehicle, 1 not nominal lane."""
    g = g or SpaceTimeGrid()
    rng = np.random.default_rng([SEED0, ST_SEED, 2, frame])
    cx, cy = _road_centre(g)
    phi = rng.uniform(0.0, 2 * math.pi, n_agents)
    r = ROAD_RADIUS + rng.uniform(-0.75, 0.75, n_agents)
    sgn = np.where(rng.uniform(size=n_agents) < 0.5, -1.0, 1.0)
    v = rng.uniform(5.0, 12.0, n_agents)
    _, cells = _spacetime_cells(g, cx + r * np.cos(phi), cy + r * np.sin(phi), phi + sgn * 0.5 * math.pi,
                                sgn / r, v, np.zeros(n_agents), np.full(n_agents, g.n_tau), threads=1)
    O = np.zeros((g.n_cells, 2), np.uint8)
    O[cells.astype(np.int64), 0] = 1
    O[:, 1] = np.tile(off_road_mask(g).reshape(-1), g.n_tau)
    return O


def bernoulli_abstraction(n_traj: int, n_cells: int, p: float, seed: int = 0) -> Abstraction:
    """Rows with every cell set independently with probability p (sorted ids)."""
    rng = np.random.default_rng([SEED0, ST_SEED, 3, seed])
    counts = rng.binomial(n_cells, p, n_traj)
    rows = []
    for c in counts:
        ids = np.unique(rng.integers(0, n_cells, int(c)))
        while len(ids) < c:  # redraw collisions
            ids = np.unique(np.concatenate([ids, rng.integers(0, n_cells, int(c) - len(ids))]))
        rows.append(ids.astype(np.uint32))
    row_ptr = np.zeros(n_traj + 1, np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate(rows) if rows else np.zeros(0, np.uint32)
    return Abstraction(grid=SpaceTimeGrid(), row_ptr=row_ptr, col_idx=col)


def bernoulli_frame(n_cells: int, n_props: int, q: float, seed: int = 0) -> np.ndarray:
    """O with every (cell, proposition) set independently with probability q."""
    rng = np.random.default_rng([SEED0, ST_SEED, 4, seed])
    return (rng.uniform(size=(n_cells, n_props)) < q).astype(np.uint8)


def spacetime_roadmap(n_traj: int, g: SpaceTimeGrid | None = None):
    """The transition system behind spacetime_abstraction's rows: transition
    t leaves vertex t // 8 and ends at the vertex whose start layer is the
    first at or after its end layer and whose angle along the road is
    nearest its end point's (a sink vertex, id n_v, when no vertex starts
    that late); cost = 1 + its length in millimetres.  Returns (n_vertices,
    src, dst, cost) as numpy arrays of uint32."""
    g = g or SpaceTimeGrid()
    rng = np.random.default_rng([SEED0, ST_SEED, 1, 0])
    tr = draw_transitions(rng, n_traj, g)
    per = TRANSITIONS_PER_VERTEX
    n_v = -(-n_traj // per)
    cx, cy = _road_centre(g)
    vx, vy = tr["x0"][::per], tr["y0"][::per]
    v_layer = tr["tau0"][::per].astype(np.int64)
    v_phi = np.arctan2(vy - cy, vx - cx)
    src = (np.arange(n_traj) // per).astype(np.uint32)
    s = tr["v"] * (tr["dur"] - 1) * g.dt
    half = 0.5 * tr["k"] * s
    f = s * np.sinc(half / math.pi)  # sin(half) / half, numpy's sinc is normalised
    mid = tr["th0"] + half
    ex, ey = tr["x0"] + f * np.cos(mid), tr["y0"] + f * np.sin(mid)
    e_phi = np.arctan2(ey - cy, ex - cx)
    e_layer = tr["tau0"].astype(np.int64) + tr["dur"].astype(np.int64)
    # vertices are sorted by (layer, angle); the first layer at or after the end
    layers = np.unique(v_layer)
    li = np.searchsorted(layers, e_layer)
    dst = np.full(n_traj, n_v, np.uint32)
    ok = li < len(layers)
    two_pi = 2 * math.pi
    vp = np.mod(v_phi, two_pi)  # ascending within each layer (vertices were sorted by angle)
    ep = np.mod(e_phi, two_pi)
    for layer in np.unique(layers[li[ok]]):
        ts = np.nonzero(ok & (layers[np.minimum(li, len(layers) - 1)] == layer))[0]
        a = int(np.searchsorted(v_layer, layer, side="left"))
        b = int(np.searchsorted(v_layer, layer, side="right"))
        ang = vp[a:b]
        k = np.searchsorted(ang, ep[ts])
        cand = np.stack([(k - 1) % (b - a), k % (b - a)])  # neighbours on the circle
        gap = np.abs(np.angle(np.exp(1j * (ang[cand] - ep[ts][None, :]))))
        dst[ts] = (a + cand[np.argmin(gap, axis=0), np.arange(len(ts))]).astype(np.uint32)
    cost = (1 + np.round(1000.0 * s)).astype(np.uint32)
    return n_v + 1, src, dst, cost
