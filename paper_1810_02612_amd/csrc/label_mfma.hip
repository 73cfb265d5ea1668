// int8 MFMA labeling kernel: S = T * O with int32 accumulation on the matrix
// cores, then L = (S > 0).  Exact, because every count is an integer no larger
// than the number of cells (< 2^31).
//
// Instruction: v_mfma_i32_16x16x64_i8 (gfx950), D[16x16] += A[16x64] B[64x16].
// A wavefront owns MT tiles of 16 trajectory rows and every proposition
// (ceil(n_props / 16) tiles of 16 columns).  The K dimension is walked 8 words
// (512 cells) at a time.  Lane (g, i) (g = lane / 16, i = lane % 16) loads 16
// bytes of row i: words w0 + 2g and w0 + 2g + 1.  Step q (0..7) of the block
// feeds the MFMA with the 16 cells [16 (q % 4), 16 (q % 4) + 16) of word
// w0 + 2g + q / 4 from every lane; the B operand of lane (g, j) carries the
// same 16 cells for proposition j, so A and B agree on which cell each byte
// is, and the 64 products of one MFMA cover 64 distinct cells.  Bits become
// bytes with the nibble spread (n * 0x00204081) & 0x01010101.
//
// The A operand comes from the bitpacked T (expanded in registers) or, for
// the comparison variant, from the int8 copy of T read straight from HBM.
// A block of 8 words that is zero in every row of the wavefront is skipped.
#include "lbl_internal.h"
#include "mfma.h"
#include "tune.h"

namespace lbl {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t spread_nib(uint32_t x) { return (x * 0x00204081u) & 0x01010101u; }

__device__ __forceinline__ v4i expand16(uint32_t x)
{
    v4i r;
    r[0] = (int)spread_nib(x & 0xFu);
    r[1] = (int)spread_nib((x >> 4) & 0xFu);
    r[2] = (int)spread_nib((x >> 8) & 0xFu);
    r[3] = (int)spread_nib((x >> 12) & 0xFu);
    return r;
}

__device__ __forceinline__ uint32_t slice16(const u64x2 &v, int q)
{
    const uint64_t w = (q < 4) ? v.x : v.y;
    return (uint32_t)(w >> (16 * (q & 3))) & 0xFFFFu;
}

template <int MT, int NT, bool I8>
__global__ void __launch_bounds__(256)
k_label_mfma(const uint64_t *__restrict__ T, uint32_t row_stride, const int8_t *__restrict__ T8,
             uint32_t n_words, uint64_t n_traj, const uint64_t *__restrict__ Ow, uint32_t n_props,
             uint8_t *__restrict__ L)
{
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, i = lane & 15;
    const uint64_t row0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (16 * MT);
    if (row0 >= n_traj) return;
    const uint32_t row_cells = n_words * 64;

    v4i acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = v4i{0, 0, 0, 0};

    bool row_ok[MT];
    const uint64_t *Trow[MT];
    const int8_t *T8row[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const uint64_t r = row0 + 16 * m + i;
        row_ok[m] = r < n_traj;
        Trow[m] = T + (row_ok[m] ? r : 0) * (uint64_t)row_stride;
        T8row[m] = I8 ? T8 + (row_ok[m] ? r : 0) * (uint64_t)row_cells : nullptr;
    }

    for (uint32_t w0 = 0; w0 < n_words; w0 += 8) {
        const uint32_t wa = w0 + 2 * g;  // this lane's first word of the block
        u64x2 a[MT];
        bool any = false;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            a[m].x = (row_ok[m] && wa < n_words) ? Trow[m][wa] : 0ull;
            a[m].y = (row_ok[m] && wa + 1 < n_words) ? Trow[m][wa + 1] : 0ull;
            any |= (a[m].x | a[m].y) != 0ull;
        }
        if (__ballot(any) == 0ull) continue;  // uniform skip of an all-zero block

        u64x2 b[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const uint32_t p = 16 * n + i;
            b[n].x = (wa < n_words) ? Ow[(uint64_t)wa * 64 + p] : 0ull;
            b[n].y = (wa + 1 < n_words) ? Ow[(uint64_t)(wa + 1) * 64 + p] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            v4i bo[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) bo[n] = expand16(slice16(b[n], q));
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                v4i ao;
                if (I8) {
                    const uint32_t wq = wa + (q >> 2);
                    const bool ok = row_ok[m] && wq < n_words;
                    ao = ok ? *reinterpret_cast<const v4i *>(T8row[m] + (uint64_t)wq * 64 + 16 * (q & 3))
                            : v4i{0, 0, 0, 0};
                } else {
                    ao = expand16(slice16(a[m], q));
                }
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[m][n] = mfma_i32_16x16x64_i8(ao, bo[n], acc[m][n]);
            }
        }
    }

    // D layout: lane (g, i) holds rows 4g..4g+3 of column i of each 16x16 tile
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const uint32_t p = 16 * n + i;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t row = row0 + 16 * m + 4 * g + r;
                if (row < n_traj && p < n_props) L[row * n_props + p] = acc[m][n][r] > 0 ? 1 : 0;
            }
        }
}

template <int MT, int NT, bool I8>
hipError_t launch_t(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L, int wpb, hipStream_t s)
{
    const uint64_t rows_per_block = 16ull * MT * wpb;
    const uint64_t blocks = (a->n_traj + rows_per_block - 1) / rows_per_block;
    hipLaunchKernelGGL((k_label_mfma<MT, NT, I8>), dim3((unsigned)blocks), dim3(64 * wpb), 0, s, a->T_bits,
                       a->row_stride, a->T_i8, a->n_words, a->n_traj, Ow, n_props, L);
    return hipGetLastError();
}

template <int MT, bool I8>
hipError_t launch_nt(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L, int wpb, hipStream_t s)
{
    switch ((n_props + 15) / 16) {
    case 1: return launch_t<MT, 1, I8>(a, Ow, n_props, L, wpb, s);
    case 2: return launch_t<MT, 2, I8>(a, Ow, n_props, L, wpb, s);
    case 3: return launch_t<MT, 3, I8>(a, Ow, n_props, L, wpb, s);
    default: return launch_t<MT, 4, I8>(a, Ow, n_props, L, wpb, s);
    }
}

// Layout probe: one wavefront multiplies lane-indexed operands exactly as the
// labeling kernel feeds them and stores the four accumulators of every lane.
__global__ void k_mfma_probe(const v4i *A, const v4i *B, v4i *D)
{
    const int lane = threadIdx.x & 63;
    D[lane] = mfma_i32_16x16x64_i8(A[lane], B[lane], v4i{0, 0, 0, 0});
}

}  // namespace

hipError_t launch_label_mfma(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L,
                             const MfmaTile &tile, bool from_i8, hipStream_t s)
{
    const int wpb = tile.waves_per_block;
    if (wpb < 1 || wpb > 4) return hipErrorInvalidValue;
    if (from_i8) {
        switch (tile.m_tiles) {
        case 1: return launch_nt<1, true>(a, Ow, n_props, L, wpb, s);
        case 2: return launch_nt<2, true>(a, Ow, n_props, L, wpb, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (tile.m_tiles) {
    case 1: return launch_nt<1, false>(a, Ow, n_props, L, wpb, s);
    case 2: return launch_nt<2, false>(a, Ow, n_props, L, wpb, s);
    case 4: return launch_nt<4, false>(a, Ow, n_props, L, wpb, s);
    default: return hipErrorInvalidValue;
    }
}

// Check on the device that the MFMA pairs A byte b of lane (g, i) with B byte
// b of lane (g, j) into D[i][j], and returns row 4g + r of column i in
// accumulator r of lane (g, i).  Random 0/1 operands; compared on the host.
lbl_status mfma_layout_selftest()
{
    static std::once_flag once;
    static lbl_status result = LBL_OK;
    static std::string msg;
    std::call_once(once, [] {
        int8_t hA[64 * 16], hB[64 * 16];
        uint32_t x = 12345u;
        for (int k = 0; k < 64 * 16; ++k) {
            x = x * 1664525u + 1013904223u;
            hA[k] = (int8_t)((x >> 13) & 1u);
            x = x * 1664525u + 1013904223u;
            hB[k] = (int8_t)((x >> 17) & 1u);
        }
        int32_t want[16][16] = {};
        for (int gg = 0; gg < 4; ++gg)
            for (int ii = 0; ii < 16; ++ii)
                for (int jj = 0; jj < 16; ++jj)
                    for (int bb = 0; bb < 16; ++bb)
                        want[ii][jj] += hA[(gg * 16 + ii) * 16 + bb] * hB[(gg * 16 + jj) * 16 + bb];
        void *dA = nullptr, *dB = nullptr, *dD = nullptr;
        int32_t hD[64 * 4];
        hipError_t e = hipMalloc(&dA, sizeof(hA));
        if (e == hipSuccess) e = hipMalloc(&dB, sizeof(hB));
        if (e == hipSuccess) e = hipMalloc(&dD, sizeof(hD));
        if (e == hipSuccess) e = hipMemcpy(dA, hA, sizeof(hA), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dB, hB, sizeof(hB), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, nullptr, (const v4i *)dA, (const v4i *)dB,
                               (v4i *)dD);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpy(hD, dD, sizeof(hD), hipMemcpyDeviceToHost);
        (void)hipFree(dA);
        (void)hipFree(dB);
        (void)hipFree(dD);
        if (e != hipSuccess) {
            result = e == hipErrorOutOfMemory ? LBL_ENOMEM : LBL_EDEVICE;
            msg = std::string("MFMA layout self-test: ") + hipGetErrorString(e);
            return;
        }
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r)
                if (hD[l * 4 + r] != want[4 * (l >> 4) + r][l & 15]) {
                    result = LBL_EDEVICE;
                    msg = "MFMA layout self-test: accumulator layout differs from the kernel's assumption";
                    return;
                }
    });
    if (result != LBL_OK) set_error(msg);
    return result;
}

}  // namespace lbl
