// Entry points whose implementation is not in this build yet.
#include "internal.h"

using namespace binimpl;

extern "C" {
int bin_particles_batched(const bin_request*, int32_t, void*) {
  clear_error();
  return fail(BIN_ERR_UNSUPPORTED, "bin_particles_batched not implemented yet");
}
int bin_graph_create(const bin_request*, int32_t, bin_graph**) {
  clear_error();
  return fail(BIN_ERR_UNSUPPORTED, "graphs not implemented yet");
}
int bin_graph_launch(bin_graph*, void*) { return fail(BIN_ERR_UNSUPPORTED, "graphs not implemented yet"); }
int bin_graph_destroy(bin_graph*) { return fail(BIN_ERR_UNSUPPORTED, "graphs not implemented yet"); }
int bin_autotune(const bin_request*, int32_t) { return fail(BIN_ERR_UNSUPPORTED, "autotune not implemented yet"); }
int binsrv_create(const binsrv_config*, binsrv**) { return fail(BIN_ERR_UNSUPPORTED, "server not implemented yet"); }
int binsrv_submit(binsrv*, const binsrv_request*, uint64_t*) { return fail(BIN_ERR_UNSUPPORTED, "server"); }
int binsrv_wait(binsrv*, uint64_t, int64_t, bin_result*) { return fail(BIN_ERR_UNSUPPORTED, "server"); }
int binsrv_release(binsrv*, uint64_t) { return fail(BIN_ERR_UNSUPPORTED, "server"); }
int binsrv_get_stats(binsrv*, binsrv_stats*) { return fail(BIN_ERR_UNSUPPORTED, "server"); }
int binsrv_destroy(binsrv*) { return fail(BIN_ERR_UNSUPPORTED, "server"); }
}
