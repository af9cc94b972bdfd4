// Batched persistent launch (placeholder until the persistent kernel lands).
#include "batch.hpp"

namespace lbm {

struct BatchCtx {};

#define NOT_YET return set_error(LBM_E_INVAL, "batched contexts are not available in this build")
lbm_status batch_required_bytes(const std::vector<DomainGeo>&, const lbm_params&, int64_t*) { NOT_YET; }
lbm_status batch_init(const std::vector<DomainGeo>&, const lbm_params&, double, double, char*, int64_t, hipStream_t,
                      BatchCtx**) { NOT_YET; }
lbm_status batch_step(BatchCtx*, int64_t) { NOT_YET; }
lbm_status batch_run_to_steady(BatchCtx*, double, int64_t, int64_t, int64_t*) { NOT_YET; }
lbm_status batch_profile(BatchCtx*, int, int, int, double*, double*, double*) { NOT_YET; }
lbm_status batch_permeability(BatchCtx*, int, int, int, int, double*) { NOT_YET; }
lbm_status batch_fields(BatchCtx*, int, double*, double*) { NOT_YET; }
lbm_status batch_totals(BatchCtx*, int, double*, double*) { NOT_YET; }
lbm_status batch_state_bytes(BatchCtx*, int64_t*) { NOT_YET; }
lbm_status batch_save(BatchCtx*, void*, int64_t, int64_t) { NOT_YET; }
lbm_status batch_load(BatchCtx*, const void*, int64_t) { NOT_YET; }
lbm_status batch_autotune(BatchCtx*, int32_t) { NOT_YET; }
void batch_destroy(BatchCtx* b) { delete b; }

}  // namespace lbm
