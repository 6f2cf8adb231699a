// Line-kernel instances with 6 register rows per lane.
#include "line.h"

namespace cb {

static const LineKernel kTable[] = {CB_LINE_R(6, true, false)};

const LineKernel *line_table_m6(int *count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

static const BatchKernel kBatch[] = {CB_BATCH_R(6, true, false)};

const BatchKernel *batch_table_m6(int *count) {
  *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
  return kBatch;
}

}  // namespace cb
