// Batched form entry points (argument checks only until the batched kernels land).
#include "foa.h"

extern "C" {

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
