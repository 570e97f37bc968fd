// Tiled fused search (dedispersion + boxcar detection) for uint8 data with unit
// weights.  Placeholder until the tiled kernel lands: the general path is used.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dd {

struct TiledTables {};

void free_tiled(TiledTables *t) { delete t; }

bool search_supported(const dedisp_plan_s *, const WidthList &) { return false; }

size_t search_work_bytes(const dedisp_plan_s *, int32_t, int64_t) { return 0; }

dedisp_status run_search_tiled(dedisp_plan, const uint8_t *, int64_t, int64_t, int64_t,
                               const WidthList &, const double *, const double *, double *,
                               int32_t *, int32_t *, void *, hipStream_t) {
  return fail(DEDISP_ERR_UNSUPPORTED, "tiled search not built");
}

}  // namespace dd

extern "C" {

dedisp_status dedisp_batch_create(dedisp_batch *, int32_t, const dedisp_plan *, const int64_t *,
                                  const int32_t *, int32_t) {
  return dd::fail(DEDISP_ERR_UNSUPPORTED, "batched search not built");
}
dedisp_status dedisp_batch_destroy(dedisp_batch) {
  return dd::fail(DEDISP_ERR_UNSUPPORTED, "batched search not built");
}
dedisp_status dedisp_batch_work_bytes(dedisp_batch, size_t *) {
  return dd::fail(DEDISP_ERR_UNSUPPORTED, "batched search not built");
}
dedisp_status dedisp_batch_run(dedisp_batch, const void *const *, const int64_t *, const double *,
                               const double *, double *, int32_t *, int32_t *, void *, size_t,
                               int32_t, void *) {
  return dd::fail(DEDISP_ERR_UNSUPPORTED, "batched search not built");
}
dedisp_status dedisp_batch_info(dedisp_batch, int64_t *, int64_t *) {
  return dd::fail(DEDISP_ERR_UNSUPPORTED, "batched search not built");
}
dedisp_status dedisp_autotune(dedisp_plan, const void *, int64_t, int64_t, const int32_t *, int32_t,
                              const double *, const double *, void *, size_t, void *, int32_t *) {
  return dd::fail(DEDISP_ERR_UNSUPPORTED, "autotuner not built");
}
dedisp_status dedisp_set_tile(dedisp_plan p, int32_t tile) {
  if (!p) return dd::fail(DEDISP_ERR_INVALID_ARG, "null plan");
  p->tile_choice = tile;
  return DEDISP_OK;
}

}  // extern "C"
