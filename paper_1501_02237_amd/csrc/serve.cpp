// Serving engine (placeholder until the continuous-batching engine lands).
#include "api_internal.hpp"

extern "C" {
int bdeg_serve_open(size_t, bdeg_server **) { return BDEG_E_STATE; }
int bdeg_serve_submit(bdeg_server *, const int64_t *, int32_t, int32_t, uint64_t, int32_t, uint64_t *) {
  return BDEG_E_STATE;
}
int bdeg_serve_poll(bdeg_server *, uint64_t, bdeg_result *) { return BDEG_E_STATE; }
int bdeg_serve_wait(bdeg_server *, uint64_t, bdeg_result *) { return BDEG_E_STATE; }
int bdeg_serve_close(bdeg_server *) { return BDEG_E_STATE; }
}
