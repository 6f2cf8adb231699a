// FP32 + FP64-refinement instances of the partitioned (P > 1) kernels with
// 8 register rows per lane: the interior solve of phase C in FP32, phases
// A and B in FP64, and the residual forms of phases A and C that the
// refinement iterations run.
#include "wg.h"

namespace cb {

// FP32 phase C on whole partitions (full-block plans): tridiagonal
// unit-stride lines only (the refinement form of wider bands, and of strided
// 16-row lanes at their 1024-thread bound, spills registers)
template <int R, int M, int MODE, int Q, bool ILU, bool RES>
const void *wg32_fb() {
  if constexpr (MODE == MODE_X && ILU && R == 1)
    return (const void *)&k_wg_c<R, M, MODE, Q, true, float, RES, true>;
  else
    return nullptr;
}

#define CB_WG32_INST(R, M, MODE, Q, ILU)                                                               \
  {R, M, MODE, Q, ILU, wg_max_threads<M, MODE>(), (const void *)&k_wg_a<R, MODE, Q, false>,            \
   (const void *)&k_wg_b<R>, nullptr, (const void *)&k_wg_a<R, MODE, Q, true>,                        \
   (const void *)&k_wg_c<R, M, MODE, Q, ILU, float, false>, (const void *)&k_wg_c<R, M, MODE, Q, ILU, float, true>, \
   nullptr, wg32_fb<R, M, MODE, Q, ILU, false>(), wg32_fb<R, M, MODE, Q, ILU, true>()}
#define CB_WG32_I(R, M, MODE, Q) CB_WG32_INST(R, M, MODE, Q, false), CB_WG32_INST(R, M, MODE, Q, true)
#define CB_WG32_Q(R, M, MODE) CB_WG32_I(R, M, MODE, 0), CB_WG32_I(R, M, MODE, 2), CB_WG32_I(R, M, MODE, 3)
#define CB_WG32_R(R) CB_WG32_Q(R, 8, MODE_X), CB_WG32_Q(R, 8, MODE_S)
static const WgKernel kWg32Kernels[] = {CB_WG32_R(1), CB_WG32_R(2), CB_WG32_R(3)};

const WgKernel *wg32_table_m8(int *count) {
  *count = (int)(sizeof(kWg32Kernels) / sizeof(kWg32Kernels[0]));
  return kWg32Kernels;
}

}  // namespace cb
