// Event spans around library kernels, active only while profiling is enabled.
#pragma once

#include "lbl_internal.h"

namespace lbl {

bool profiling();
// Record a start event on s (returns a token, or nullptr when not profiling).
void *span_begin(hipStream_t s);
// Record the end event; kind 0 = O packing, 1 = labeling, 2 = whole batch.
void span_end(void *begin, hipStream_t s, int kind);

}  // namespace lbl
