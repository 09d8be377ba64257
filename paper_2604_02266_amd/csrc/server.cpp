// Serving entry points (continuous batching).  Implemented in a later step.
#include "otfs_internal.h"
#include "plan_internal.h"

using namespace otfs;

extern "C" otfs_status otfs_server_create(int, void*, size_t, const otfs_cg_opts*, int32_t,
                                          otfs_server_t** out) {
  if (out) *out = nullptr;
  return fail(OTFS_E_UNSUPPORTED, "serving is not built yet");
}
extern "C" otfs_status otfs_submit(otfs_server_t*, const otfs_frame_desc*, const void*, uint64_t*) {
  return fail(OTFS_E_UNSUPPORTED, "serving is not built yet");
}
extern "C" otfs_status otfs_poll(otfs_server_t*, uint64_t, void*, uint8_t*, otfs_frame_stats*,
                                 uint64_t*) {
  return fail(OTFS_E_UNSUPPORTED, "serving is not built yet");
}
extern "C" otfs_status otfs_server_stats(otfs_server_t*, otfs_server_stats_t*) {
  return fail(OTFS_E_UNSUPPORTED, "serving is not built yet");
}
extern "C" otfs_status otfs_server_free(otfs_server_t*) { return OTFS_OK; }
