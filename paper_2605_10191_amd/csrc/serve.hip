// Placeholder for the continuous-batching server.
#include "internal.hpp"

namespace polfed {

polfed_status serve_start(polfed_ctx*, size_t, int) {
  fail(POLFED_ERR_INVALID, "serving not available yet");
}
polfed_status serve_submit(polfed_ctx*, const polfed_op*, const polfed_params*, const double*,
                           double*, double*, double*, polfed_req**) {
  fail(POLFED_ERR_INVALID, "serving not available yet");
}
polfed_status req_poll(polfed_req*, int*) { fail(POLFED_ERR_INVALID, "serving not available yet"); }
polfed_status req_wait(polfed_req*, int*, polfed_report*) {
  fail(POLFED_ERR_INVALID, "serving not available yet");
}
polfed_status req_destroy(polfed_req*) { return POLFED_OK; }
polfed_status serve_stop(polfed_ctx*) { return POLFED_OK; }

}  // namespace polfed
