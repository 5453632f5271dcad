// Multi-source BFS and closeness centrality (placeholder until the kernels land).
#include "msbfs.h"

namespace blest {

hipError_t ms_run(const DevGraph&, MsDev*, const int32_t*, int32_t, int, int16_t*, int64_t*, int64_t*, double*,
                  hipStream_t) {
  return hipErrorNotSupported;
}
void ms_release(MsDev*) {}
void ms_reset(MsDev*) {}

}  // namespace blest
