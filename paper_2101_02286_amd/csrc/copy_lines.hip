// Copy-only line-kernel instances: the loads, LDS staging, tile order and
// stores of a one-partition launch with the stencil and the solve left out,
// so that the solve's own memory access pattern can be timed alone.
#include "line.h"

namespace cb {

#define CB_COPY_INST(M, MODE, UNI) \
  {1, M, 0, MODE, 0, UNI, false, line_max_threads<1, M, double, MODE, UNI>(), \
   (const void *)&k_line<1, M, double, MODE, 0, UNI, false, true>}
#define CB_COPY_MODE(M, UNI) CB_COPY_INST(M, MODE_X, UNI), CB_COPY_INST(M, MODE_S, UNI)
static const LineKernel kCopy[] = {
    CB_COPY_MODE(4, true),  CB_COPY_MODE(4, false),  CB_COPY_MODE(6, true),  CB_COPY_MODE(6, false),
    CB_COPY_MODE(8, true),  CB_COPY_MODE(8, false),  CB_COPY_MODE(12, true), CB_COPY_MODE(12, false),
    CB_COPY_MODE(16, true), CB_COPY_MODE(16, false), CB_COPY_MODE(32, true),
};

const LineKernel *find_copy_kernel(int M, int mode, bool uni) {
  for (const auto &k : kCopy)
    if (k.M == M && k.mode == mode && k.uni == uni) return &k;
  return nullptr;
}

}  // namespace cb
