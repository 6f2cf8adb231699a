// Line-kernel instances with 32 register rows per lane (uniform FP64 lanes,
// interiors by elimination): fewer lanes per line, so more adjacent lines
// share a workgroup.
#include "line.h"

namespace cb {

static const LineKernel kTable[] = {CB_LINE_Q(1, 32, double, MODE_X, true, true),
                                    CB_LINE_Q(1, 32, double, MODE_S, true, true),
                                    CB_LINE_Q(2, 32, double, MODE_X, true, true),
                                    CB_LINE_Q(2, 32, double, MODE_S, true, true)};

const LineKernel *line_table_m32(int *count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

static const BatchKernel kBatch[] = {CB_BATCH_MODE(1, 32, double, true, true), CB_BATCH_MODE(2, 32, double, true, true)};

const BatchKernel *batch_table_m32(int *count) {
  *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
  return kBatch;
}

}  // namespace cb
