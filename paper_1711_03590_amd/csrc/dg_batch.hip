// dg_batch.hip -- continuous batching of solve requests.
#include "dg_internal.hpp"

using namespace dgk;

extern "C" {
dg_status dg_batch_create(int, const dg_allocator *, dg_batch **) { return fail(DG_ERR_UNSUPPORTED, "batch: not built yet"); }
dg_status dg_batch_admit(dg_batch *, dg_op *, dg_vec, dg_vec, const dg_solve_params *, int *, void *) { return fail(DG_ERR_UNSUPPORTED, "batch: not built yet"); }
dg_status dg_batch_run(dg_batch *, int, void *) { return fail(DG_ERR_UNSUPPORTED, "batch: not built yet"); }
dg_status dg_batch_poll(dg_batch *, int *, dg_solve_stats *, int, int *) { return fail(DG_ERR_UNSUPPORTED, "batch: not built yet"); }
int dg_batch_active(const dg_batch *) { return 0; }
dg_status dg_batch_destroy(dg_batch *) { return DG_OK; }
}
