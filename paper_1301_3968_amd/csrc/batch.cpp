// Batched persistent search across beams and the tile autotuner.
#include "internal.h"

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

}  // extern "C"
