// Serving loop: placeholder until the batching executor lands.
#include "gcdf_serve.h"

namespace gcdf {

struct Server {};

gcdf_status server_start(gcdf_ctx*, size_t, int, Server**) {
  return set_error(GCDF_EINVAL, "serving is not available in this build");
}
void server_stop(Server*) {}
gcdf_status server_submit(Server*, const gcdf_request*, uint64_t*) {
  return set_error(GCDF_EINVAL, "serving is not available in this build");
}
gcdf_status server_poll(Server*, uint64_t) { return set_error(GCDF_EINVAL, "serving is not available in this build"); }

}  // namespace gcdf
