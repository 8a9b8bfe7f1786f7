// Mapping-trace analysis (placeholder until the kernels land).
#include "internal.h"
namespace odp {
int analyze_reserve(Workspace*, size_t) { return ODP_OK; }
void analyze_release(Workspace*) {}
}  // namespace odp
extern "C" int odp_analyze_trace(const odp_event*, size_t, uint8_t*, odp_report*, odp_stream_t) {
  return odp::set_error(ODP_EINVAL, "odp_analyze_trace: not built yet");
}
