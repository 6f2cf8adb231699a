// Heptadiagonal (r = 3) line-kernel instances with 16 register rows per lane.
#include "line.h"

namespace cb {

static const LineKernel kTable[] = {CB_LINE_T(3, 16, true, false), CB_LINE_T(3, 16, false, false),
                                    CB_LINE_T(3, 16, true, true), CB_LINE_T(3, 16, false, true)};

const LineKernel *line_table_r3_m16(int *count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

static const BatchKernel kBatch[] = {CB_BATCH_T(3, 16, true, false), CB_BATCH_T(3, 16, false, false),
                                     CB_BATCH_T(3, 16, true, true), CB_BATCH_T(3, 16, false, true)};

const BatchKernel *batch_table_r3_m16(int *count) {
  *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
  return kBatch;
}

}  // namespace cb
