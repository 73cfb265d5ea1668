// Entry points not yet implemented.
#include "lbl_internal.h"

using namespace lbl;

extern "C" {
lbl_status lbl_label_batch(const lbl_job *, size_t, uint32_t, void *) { set_error("lbl_label_batch: not implemented"); return LBL_EINVAL; }
lbl_status lbl_serve_start(const lbl_serve_cfg *, lbl_server_t *) { set_error("not implemented"); return LBL_EINVAL; }
lbl_status lbl_serve_submit(lbl_server_t, lbl_abs_t, const uint8_t *, uint32_t, uint8_t *, uint64_t *) { set_error("not implemented"); return LBL_EINVAL; }
lbl_status lbl_serve_wait(lbl_server_t, uint64_t, int64_t) { set_error("not implemented"); return LBL_EINVAL; }
lbl_status lbl_serve_stats_get(lbl_server_t, lbl_serve_stats *) { set_error("not implemented"); return LBL_EINVAL; }
lbl_status lbl_serve_stop(lbl_server_t) { set_error("not implemented"); return LBL_EINVAL; }
}
