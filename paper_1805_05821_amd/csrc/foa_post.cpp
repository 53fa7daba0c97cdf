// Host FP64 post-processing of the FOA state (filled in with the host linear
// algebra): rank truncation, eigenpairs, indicators and modes.
#include "foa.h"
#include "foa_ctx.h"

using namespace foa;

extern "C" {

foa_status foa_truncate(foa_ctx c, double, int32_t, int32_t *, double *) {
  if (!c) return FOA_E_ARG;
  return set_err(c, FOA_E_STATE, "truncation not available in this build");
}

foa_status foa_modes(foa_ctx c, int32_t, double *, int8_t *, double *, double *, void *, int64_t, int32_t,
                     foa_dtype, int32_t *) {
  if (!c) return FOA_E_ARG;
  return set_err(c, FOA_E_STATE, "modes not available in this build");
}

foa_status foa_indicators(foa_ctx c, int32_t, double *, double *, int32_t *) {
  if (!c) return FOA_E_ARG;
  return set_err(c, FOA_E_STATE, "indicators not available in this build");
}

foa_status foa_batch_workspace_bytes(int32_t, const int64_t *, const int32_t *, foa_prec, size_t *) {
  return FOA_E_STATE;
}
foa_status foa_batch_init(foa_batch *, int32_t, const int64_t *, const int32_t *, foa_prec, void *, size_t, void *,
                          double, const char *) {
  return FOA_E_STATE;
}
foa_status foa_batch_push(foa_batch b, const void *const *, foa_dtype) { return b ? FOA_E_STATE : FOA_E_ARG; }
foa_status foa_batch_sync(foa_batch, int32_t *, int32_t *) { return FOA_E_STATE; }
foa_status foa_batch_view(foa_batch, int32_t, foa_ctx *) { return FOA_E_STATE; }
foa_status foa_batch_destroy(foa_batch b) { return b ? FOA_E_STATE : FOA_E_ARG; }

}  // extern "C"
