"""GPU parity of the proposition rasterizer (lbl_raster_frame) against the
oracle's encoding of the same shapes, byte for byte, and the rasterized frame
labeled end to end."""
import sys

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
from paper_1810_02612_amd import lbl  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def gpu_raster(nx, ny, cell, shapes, n_props):
    O = torch.full((nx * ny, n_props), 7, dtype=torch.uint8, device="cuda")  # every byte must be written
    lbl.raster_frame(nx, ny, cell, shapes, n_props, O)
    torch.cuda.synchronize()
    return O.cpu().numpy()


def oracle_raster(nx, ny, cell, shapes, n_props):
    return oracle.raster_shapes(shapes["kind"], shapes["prop"], shapes["cx"], shapes["cy"], shapes["a"], shapes["b"],
                                nx, ny, cell, n_props)


def arr(shape_list):
    kind, prop, cx, cy, a, b = (np.array([s[i] for s in shape_list]) for i in range(6))
    return lbl.shapes_array(kind, prop, cx, cy, a, b)


@pytest.mark.parametrize("cfg,n,res,n_props,frame,rho", [(1, 64, 0.5, 8, 0, None), (2, 256, 0.25, 32, 1, None),
                                                         (3, 512, 0.2, 64, 2, 0.01), (3, 512, 0.2, 64, 3, 0.4),
                                                         (4, 128, 0.8, 37, 4, None)])
def test_matches_oracle(cfg, n, res, n_props, frame, rho):
    g = gen.Grid(n, res)
    sh = gen.frame_shapes(cfg, g, n_props, frame, rho=rho)
    shapes = lbl.shapes_array(sh.kind, sh.prop, sh.cx, sh.cy, sh.a, sh.b)
    say(f"raster cfg{cfg} {n}^2 x {n_props}, {len(shapes)} shapes")
    got = gpu_raster(n, n, res, shapes, n_props)
    want = oracle_raster(n, n, res, shapes, n_props)
    assert np.array_equal(got, want), f"{(got != want).sum()} bytes differ"
    # the generator's frames are the same encoding
    assert np.array_equal(got, gen.make_frame(cfg, g, n_props, frame, rho=rho))


def test_edge_cases():
    say("raster edge cases")
    # no shapes: every byte cleared
    assert gpu_raster(16, 16, 0.5, lbl.shapes_array([], [], [], [], [], []), 5).sum() == 0
    cases = [
        [(1, 0, -5.0, -5.0, 1.0, 0.0), (0, 0, 100.0, 1.0, 3.0, 3.0)],           # outside the workspace
        [(0, 0, 1.5, 1.5, 0.5, 0.5), (0, 1, 1.0, 1.5, 0.0, 0.5), (1, 2, 0.25, 0.25, 0.0, 0.0)],  # touching only
        [(1, 0, 1.75, 1.25, 0.25, 0.0), (1, 1, 2.0, 1.5, 0.25, 0.0)],           # disc reaching edges, on a corner
        [(0, 0, 0.0, 0.0, 0.75, 0.75), (0, 2, 8.0, 4.0, 100.0, 0.1)],           # straddling the border, very long
        [(0, 0, 3.3, 2.7, 1e-12, 1e-12), (1, 1, 3.3, 2.7, 1e-12, 0.0)],        # tiny
    ]
    for k, c in enumerate(cases):
        shapes = arr(c)
        for nx, ny in ((16, 16), (16, 32), (64, 8)):
            got = gpu_raster(nx, ny, 0.5, shapes, 3)
            want = oracle_raster(nx, ny, 0.5, shapes, 3)
            assert np.array_equal(got, want), (k, nx, ny)


@pytest.mark.parametrize("n_props", [1, 64])
def test_proposition_counts(n_props):
    rng = np.random.default_rng(n_props)
    shapes = arr([(int(rng.integers(0, 2)), int(rng.integers(0, n_props)), rng.uniform(-2, 34), rng.uniform(-2, 34),
                   rng.uniform(0, 6), rng.uniform(0, 6)) for _ in range(200)])
    got = gpu_raster(64, 64, 0.5, shapes, n_props)
    assert np.array_equal(got, oracle_raster(64, 64, 0.5, shapes, n_props))


def test_rejects_bad_input():
    O = torch.zeros((256, 4), dtype=torch.uint8, device="cuda")
    bad = [
        [(2, 0, 1.0, 1.0, 1.0, 1.0)],            # unknown kind
        [(0, 4, 1.0, 1.0, 1.0, 1.0)],            # prop >= n_props
        [(0, 0, float("nan"), 1.0, 1.0, 1.0)],  # not finite
        [(1, 0, 1.0, 1.0, -1.0, 0.0)],           # negative radius
        [(0, 0, 1.0, 1.0, 1.0, -0.5)],           # negative half size
    ]
    for c in bad:
        with pytest.raises(lbl.LblError) as e:
            lbl.raster_frame(16, 16, 0.5, arr(c), 4, O)
        assert e.value.status == lbl.EINVAL
    ok = arr([(0, 0, 1.0, 1.0, 1.0, 1.0)])
    for nx, cell, n_props in ((12, 0.5, 4), (16, 0.0, 4), (16, float("inf"), 4), (16, 0.5, 0), (16, 0.5, 65)):
        with pytest.raises(lbl.LblError) as e:
            lbl.raster_frame(nx, 16, cell, ok, n_props, O)
        assert e.value.status == lbl.EINVAL


def test_shapes_to_labels():
    g = gen.Grid(64, 0.5)
    a = gen.make_abstraction(1)
    h = lbl.load_abstraction(64, 64, a.row_ptr, a.col_idx)
    try:
        sh = gen.frame_shapes(1, g, 8, 11)
        shapes = lbl.shapes_array(sh.kind, sh.prop, sh.cx, sh.cy, sh.a, sh.b)
        O = torch.empty((g.n_cells, 8), dtype=torch.uint8, device="cuda")
        L = torch.full((a.n_traj, 8), 9, dtype=torch.uint8, device="cuda")
        lbl.raster_frame(64, 64, 0.5, shapes, 8, O)
        lbl.label_frame(h, O, 8, L)
        torch.cuda.synchronize()
        want = oracle.label_csr(a.row_ptr, a.col_idx, g.n_cells, oracle_raster(64, 64, 0.5, shapes, 8))
        assert np.array_equal(L.cpu().numpy(), want)
    finally:
        lbl.free_abstraction(h)
