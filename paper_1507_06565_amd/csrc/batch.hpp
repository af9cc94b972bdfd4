// Batched pore-scale runs: many independent domains advanced together; in the
// AA layout by one persistent kernel (batch.hip), in the brick layout by the
// brick sweep over one brick array (brick_batch.cpp).  Internal; reached through the C ABI when a
// geometry holds more than one domain.
#pragma once
#include <vector>

#include "internal.hpp"

namespace lbm {

struct BatchCtx;

lbm_status batch_required_bytes(const std::vector<DomainGeo>& doms, const lbm_params& p, int64_t* bytes);
lbm_status batch_init(const std::vector<DomainGeo>& doms, const lbm_params& p, double wp, double wm, char* buf,
                      int64_t bytes, hipStream_t s, BatchCtx** out);
lbm_status batch_step(BatchCtx* b, int64_t n);
lbm_status batch_run_to_steady(BatchCtx* b, double rel_tol, int64_t check_every, int64_t max_steps,
                               int64_t* steps_done);
lbm_status batch_profile(BatchCtx* b, int dom, int axis, int comp, double* u_sup, double* u_int, double* por);
lbm_status batch_permeability(BatchCtx* b, int dom, int fa, int z0, int z1, double* k);
lbm_status batch_fields(BatchCtx* b, int dom, double* rho, double* u);
lbm_status batch_totals(BatchCtx* b, int dom, double* mass, double* mom);
lbm_status batch_state_bytes(BatchCtx* b, int64_t* bytes);
lbm_status batch_save(BatchCtx* b, void* host, int64_t bytes, int64_t steps);
lbm_status batch_load(BatchCtx* b, const void* host, int64_t bytes);
lbm_status batch_autotune(BatchCtx* b, int32_t steps_per_trial);
lbm_status batch_set_launch(BatchCtx* b, int32_t block, int32_t W);
lbm_status batch_get_launch(BatchCtx* b, int32_t* block, int32_t* W);
void batch_destroy(BatchCtx* b);

// Batches in the brick layout (brick_batch.cpp): every domain's stored bricks
// in one brick array, stepped by the brick sweep over a list of the bricks of
// the running domains; same calls as above.
struct BrickBatch;
lbm_status bbatch_required_bytes(const std::vector<DomainGeo>& doms, const lbm_params& p, int64_t* bytes);
lbm_status bbatch_init(const std::vector<DomainGeo>& doms, const lbm_params& p, double wp, double wm, char* buf,
                       int64_t bytes, hipStream_t s, BrickBatch** out);
lbm_status bbatch_step(BrickBatch* b, int64_t n);
lbm_status bbatch_run_to_steady(BrickBatch* b, double rel_tol, int64_t check_every, int64_t max_steps,
                                int64_t* steps_done);
lbm_status bbatch_profile(BrickBatch* b, int dom, int axis, int comp, double* u_sup, double* u_int, double* por);
lbm_status bbatch_permeability(BrickBatch* b, int dom, int fa, int z0, int z1, double* k);
lbm_status bbatch_fields(BrickBatch* b, int dom, double* rho, double* u);
lbm_status bbatch_totals(BrickBatch* b, int dom, double* mass, double* mom);
lbm_status bbatch_state_bytes(BrickBatch* b, int64_t* bytes);
lbm_status bbatch_save(BrickBatch* b, void* host, int64_t bytes, int64_t steps);
lbm_status bbatch_load(BrickBatch* b, const void* host, int64_t bytes);
lbm_status bbatch_autotune(BrickBatch* b, int32_t steps_per_trial);
lbm_status bbatch_set_launch(BrickBatch* b, int32_t block, int32_t W);
lbm_status bbatch_get_launch(BrickBatch* b, int32_t* block, int32_t* W);
void bbatch_destroy(BrickBatch* b);

}  // namespace lbm
