// Line-kernel instances with 12 register rows per lane.
#include "line.h"

namespace cb {

static const LineKernel kTable[] = {CB_LINE_R(12, true, false), CB_LINE_R(12, true, true)};

const LineKernel *line_table_m12(int *count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

static const BatchKernel kBatch[] = {CB_BATCH_R(12, true, false), CB_BATCH_R(12, true, true)};

const BatchKernel *batch_table_m12(int *count) {
  *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
  return kBatch;
}

}  // namespace cb
