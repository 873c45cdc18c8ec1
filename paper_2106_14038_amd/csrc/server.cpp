// Served form: placeholder until the request loop lands.
#include "engine.hpp"
#include "gsmart.h"

namespace gs {
int server_start(Engine *, const gs_server_options *, gs_server **out) {
  *out = nullptr;
  set_error("server not built yet");
  return GS_EUNSUPPORTED;
}
int server_submit(gs_server *, const gs_query *, uint32_t, uint64_t *) { return GS_EUNSUPPORTED; }
int server_poll(gs_server *, uint64_t, gs_result **) { return GS_EUNSUPPORTED; }
int server_stop(gs_server *, gs_server_stats *) { return GS_EUNSUPPORTED; }
}  // namespace gs
