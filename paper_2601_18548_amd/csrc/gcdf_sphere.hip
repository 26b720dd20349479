// Query kernels for sphere obstacles (x, y, z, r): the primitive-aware network
// input [p', r, a] of the closing discussion (Sec. VII), one more input column
// than the point query; the same tile engine (gcdf_tile.h) with SPH set.
#include "gcdf_tile.h"

namespace gcdf {

hipError_t launch_fused_sphere(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu,
                               hipStream_t s) {
  if (job.dumpH || job.seed) return hipErrorInvalidValue;  // training takes point networks only
  if (net.width == 256) return launch_w<256, true>(net, job, pairs, want_grad, num_cu, s);
  return launch_w<512, true>(net, job, pairs, want_grad, num_cu, s);
}

}  // namespace gcdf
