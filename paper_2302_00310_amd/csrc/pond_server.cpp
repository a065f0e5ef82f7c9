// Serving loop of libpond.so (continuous batching of independent solves).
#include <hip/hip_runtime.h>

#include "../../include/pond.h"
#include "pond_state.h"

using namespace pond;

extern "C" {

int pond_server_create(void*, size_t, void*, int, pond_server** out) {
  if (out) *out = nullptr;
  return fail(POND_ERR_UNSUPPORTED, "serving is not built yet");
}
int pond_submit(pond_server*, const pond_request*, uint64_t*) {
  return fail(POND_ERR_UNSUPPORTED, "serving is not built yet");
}
int pond_poll(pond_server*, uint64_t, pond_result*) {
  return fail(POND_ERR_UNSUPPORTED, "serving is not built yet");
}
int pond_server_destroy(pond_server*) { return POND_OK; }

}  // extern "C"
