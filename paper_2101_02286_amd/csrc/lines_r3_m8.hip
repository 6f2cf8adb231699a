// Heptadiagonal (r = 3) line-kernel instances with 8 register rows per lane.
#include "line.h"

namespace cb {

static const LineKernel kTable[] = {CB_LINE_T(3, 8, true, false), CB_LINE_T(3, 8, false, false),
                                    CB_LINE_T(3, 8, true, true), CB_LINE_T(3, 8, false, true)};

const LineKernel *line_table_r3_m8(int *count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

static const BatchKernel kBatch[] = {CB_BATCH_T(3, 8, true, false), CB_BATCH_T(3, 8, false, false),
                                     CB_BATCH_T(3, 8, true, true), CB_BATCH_T(3, 8, false, true)};

const BatchKernel *batch_table_r3_m8(int *count) {
  *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
  return kBatch;
}

}  // namespace cb
