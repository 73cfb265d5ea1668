// Proposition regions of a frame rasterized into O on the device (Sec. 4.1
// encoding: a cell's entry is 1 iff the region intersects the cell, read as
// an overlap of positive area with the closed cell square).
//
// k_zero clears O; k_raster_shapes then gives every shape workgroups that
// walk the cells of its bounding box (widened by one cell on each side, so
// that rounding in the division cannot drop a cell, and clamped to the grid)
// and test each cell exactly:
//   rectangle: on both axes the overlap length, min of the upper ends minus
//              max of the lower ends, is positive;
//   disc:      the squared distance from the centre to the square's nearest
//              point is below the squared radius.
// Cell bounds are ix * cell and ix * cell + cell in double precision, and
// products are not fused with sums, so every decision is the one the
// definition gives in IEEE double arithmetic.  Shapes of one proposition may
// write the same byte; they all write 1.
#include <algorithm>
#include <cmath>

#include "lbl_internal.h"

namespace lbl {
namespace {

constexpr uint32_t kRasterSlices = 8;  // workgroups per shape

unsigned zero_blocks(uint64_t n_bytes)
{
    const uint64_t b = (n_bytes / 16 + 255) / 256;
    return (unsigned)std::min<uint64_t>(std::max<uint64_t>(b, 1), 4096);
}

// z-order index of cell (ix, iy): bits of ix at the odd positions, of iy at
// the even ones (x the more significant bit of each pair).
__device__ __forceinline__ uint32_t z_index(uint32_t ix, uint32_t iy)
{
    uint32_t z = 0;
    for (int b = 0; b < 16; ++b) z |= ((ix >> b) & 1u) << (2 * b + 1) | ((iy >> b) & 1u) << (2 * b);
    return z;
}

__global__ void __launch_bounds__(256) k_zero_bytes(uint8_t *__restrict__ O, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((reinterpret_cast<uintptr_t>(O) & 15u) == 0) {
        uint4 *o = reinterpret_cast<uint4 *>(O);
        for (uint64_t i = i0; i < n / 16; i += stride) o[i] = make_uint4(0u, 0u, 0u, 0u);
        for (uint64_t i = (n / 16) * 16 + i0; i < n; i += stride) O[i] = 0;
    } else {
        for (uint64_t i = i0; i < n; i += stride) O[i] = 0;
    }
}

__global__ void __launch_bounds__(256)
k_raster_shapes(const lbl_shape *__restrict__ shapes, uint32_t nx, uint32_t ny, double cell, uint32_t n_props,
                uint32_t morton, uint8_t *__restrict__ O)
{
#pragma clang fp contract(off)
    const lbl_shape sh = shapes[blockIdx.x];
    const bool rect = sh.kind == LBL_SHAPE_RECT;
    const double hx = sh.a, hy = rect ? sh.b : sh.a;
    // bounding box in cells, widened by one and clamped (in double, so that
    // far-away shapes do not overflow an integer)
    const double fx0 = fmax(floor((sh.cx - hx) / cell) - 1.0, 0.0), fx1 = fmin(floor((sh.cx + hx) / cell) + 1.0, nx - 1.0);
    const double fy0 = fmax(floor((sh.cy - hy) / cell) - 1.0, 0.0), fy1 = fmin(floor((sh.cy + hy) / cell) + 1.0, ny - 1.0);
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    const uint32_t ix0 = (uint32_t)fx0, iy0 = (uint32_t)fy0;
    const uint32_t wx = (uint32_t)fx1 - ix0 + 1, wy = (uint32_t)fy1 - iy0 + 1;
    const uint64_t n_box = (uint64_t)wx * wy;
    for (uint64_t k = (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; k < n_box;
         k += (uint64_t)gridDim.y * blockDim.x) {
        const uint32_t ix = ix0 + (uint32_t)(k % wx), iy = iy0 + (uint32_t)(k / wx);
        const double x0 = (double)ix * cell, x1 = x0 + cell;
        const double y0 = (double)iy * cell, y1 = y0 + cell;
        bool hit;
        if (rect) {
            const double ox = fmin(x1, sh.cx + sh.a) - fmax(x0, sh.cx - sh.a);
            const double oy = fmin(y1, sh.cy + sh.b) - fmax(y0, sh.cy - sh.b);
            hit = ox > 0.0 && oy > 0.0;
        } else {
            const double qx = fmin(fmax(sh.cx, x0), x1), qy = fmin(fmax(sh.cy, y0), y1);
            const double ex = sh.cx - qx, ey = sh.cy - qy;
            hit = ex * ex + ey * ey < sh.a * sh.a;
        }
        if (hit) O[(morton ? (uint64_t)z_index(ix, iy) : (uint64_t)iy * nx + ix) * n_props + sh.prop] = 1;
    }
}

}  // namespace
}  // namespace lbl

using namespace lbl;

lbl_status lbl_raster_frame(const lbl_grid *g, double cell_m, const lbl_shape *shapes, uint64_t n_shapes,
                            uint32_t n_props, uint8_t *O, void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(g != nullptr && O != nullptr, "grid or O is null");
    LBL_REQUIRE(n_shapes == 0 || shapes != nullptr, "shapes is null");
    {
        const lbl_status gst = check_grid(g);
        if (gst != LBL_OK) return gst;
    }
    LBL_REQUIRE(n_props >= 1 && n_props <= 64, "n_props must be in [1, 64]");
    LBL_REQUIRE(std::isfinite(cell_m) && cell_m > 0.0, "cell_m must be finite and positive");
    LBL_REQUIRE(n_shapes < (1ull << 31), "too many shapes");
    for (uint64_t i = 0; i < n_shapes; ++i) {
        const lbl_shape &s = shapes[i];
        LBL_REQUIRE(s.kind == LBL_SHAPE_RECT || s.kind == LBL_SHAPE_DISC, "unknown shape kind");
        LBL_REQUIRE(s.prop < n_props, "shape prop >= n_props");
        LBL_REQUIRE(std::isfinite(s.cx) && std::isfinite(s.cy) && std::isfinite(s.a) && std::isfinite(s.b),
                    "shape coordinates and sizes must be finite");
        LBL_REQUIRE(s.a >= 0.0 && (s.kind == LBL_SHAPE_DISC || s.b >= 0.0), "shape sizes must be non-negative");
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const uint64_t n_bytes = (uint64_t)g->nx * g->ny * n_props;
    hipLaunchKernelGGL(k_zero_bytes, dim3(zero_blocks(n_bytes)), dim3(256), 0, st, O, n_bytes);
    LBL_HIP_TRY(hipGetLastError());
    if (n_shapes == 0) return LBL_OK;
    void *ws = nullptr;
    lbl_status rc = workspace(st, n_shapes * sizeof(lbl_shape), &ws);
    if (rc != LBL_OK) return rc;
    lbl_shape *d_shapes = static_cast<lbl_shape *>(ws);
    LBL_HIP_TRY(hipMemcpyAsync(d_shapes, shapes, n_shapes * sizeof(lbl_shape), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_raster_shapes, dim3((unsigned)n_shapes, kRasterSlices), dim3(256), 0, st, d_shapes, g->nx,
                       g->ny, cell_m, n_props, (uint32_t)(g->cell_order == LBL_MORTON), O);
    LBL_HIP_TRY(hipGetLastError());
    return LBL_OK;
}
