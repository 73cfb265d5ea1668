// Matrix-core intrinsic used by the int8 labeling kernel (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace lbl {

typedef int mfma_v4i __attribute__((ext_vector_type(4)));

// D[16x16] (int32) = A[16x64] (int8) * B[64x16] (int8) + C
__device__ __forceinline__ mfma_v4i mfma_i32_16x16x64_i8(mfma_v4i a, mfma_v4i b, mfma_v4i c)
{
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

}  // namespace lbl
