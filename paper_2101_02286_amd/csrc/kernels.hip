// HIP kernels of libcb for gfx950 (MI355X): the FP64 instances of the
// two-level (P > 1) kernels (wg.h), the standalone stencil, and the dispatch
// to the line and batched kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "device.h"
#include "launch.h"
#include "line.h"
#include "wg.h"

namespace cb {

// ------------------------------------------------------------------------
// Standalone periodic stencil b = sum_q c_q f_{j+q} along one axis.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stencil(const StencilArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.total) return;
  // consecutive threads touch consecutive addresses: along the line when it
  // is unit-stride (idx = (v, u, j)), else across lines (idx = (v, j, u))
  int64_t u, j, vv;
  if (a.rs == 1) {
    j = idx % a.n;
    const int64_t rest = idx / a.n;
    u = rest % a.nu;
    vv = rest / a.nu;
  } else {
    u = idx % a.nu;
    const int64_t rest = idx / a.nu;
    j = rest % a.n;
    vv = rest / a.n;
  }
  const int64_t base = u * a.su + vv * a.sv;
  double acc = 0.0;
  for (int q = a.lo; q <= a.hi; ++q) {
    int64_t jj = j + q;
    jj = jj < 0 ? jj + a.n : (jj >= a.n ? jj - a.n : jj);
    acc += a.c[q - a.lo] * a.f[base + jj * a.rs];
  }
  a.b[base + j * a.rs] = acc;
}

// ------------------------------------------------------------------------
// Dispatch tables
// ------------------------------------------------------------------------
const LineKernel *find_line_kernel(int R, int M, int fp32, int mode, int Q, bool uni, bool ilu) {
  int cnt = 0;
  const LineKernel *t = nullptr;
  if (R == 3) {
    if (M == 8) t = line_table_r3_m8(&cnt);
    else if (M == 16) t = line_table_r3_m16(&cnt);
    else return nullptr;
  } else switch (M) {
    case 4: t = line_table_m4(&cnt); break;
    case 6: t = line_table_m6(&cnt); break;
    case 8: t = line_table_m8(&cnt); break;
    case 12: t = line_table_m12(&cnt); break;
    case 16: t = line_table_m16(&cnt); break;
    case 32: t = line_table_m32(&cnt); break;
    default: return nullptr;
  }
  for (int i = 0; i < cnt; ++i)
    if (t[i].R == R && t[i].M == M && t[i].fp32 == fp32 && t[i].mode == mode && t[i].Q == Q && t[i].uni == uni &&
        t[i].ilu == ilu)
      return &t[i];
  return nullptr;
}

#define CB_WG_INST(R, M, MODE, Q, ILU)                                                                 \
  {R, M, MODE, Q, ILU, wg_max_threads<M, MODE>(), (const void *)&k_wg_a<R, MODE, Q>,                      \
   (const void *)&k_wg_b<R>, (const void *)&k_wg_c<R, M, MODE, Q, ILU>, nullptr, nullptr, nullptr,        \
   ILU ? (const void *)&k_wg_c<R, M, MODE, Q, true, double, false, true> : nullptr}
#define CB_WG_I(R, M, MODE, Q) CB_WG_INST(R, M, MODE, Q, false), CB_WG_INST(R, M, MODE, Q, true)
#define CB_WG_Q(R, M, MODE) CB_WG_I(R, M, MODE, 0), CB_WG_I(R, M, MODE, 2), CB_WG_I(R, M, MODE, 3)
static const WgKernel kWgKernels[] = {
    CB_WG_Q(1, 8, MODE_X), CB_WG_Q(1, 8, MODE_S), CB_WG_Q(2, 8, MODE_X), CB_WG_Q(2, 8, MODE_S),
    CB_WG_Q(1, 16, MODE_X), CB_WG_Q(1, 16, MODE_S), CB_WG_Q(2, 16, MODE_X), CB_WG_Q(2, 16, MODE_S),
    CB_WG_Q(3, 8, MODE_X),  CB_WG_Q(3, 8, MODE_S),  CB_WG_Q(3, 16, MODE_X), CB_WG_Q(3, 16, MODE_S),
};

const WgKernel *find_wg_kernel(int R, int M, int mode, int Q, bool ilu) {
  for (const auto &k : kWgKernels)
    if (k.R == R && k.M == M && k.mode == mode && k.Q == Q && k.ilu == ilu) return &k;
  return nullptr;
}

const WgKernel *wg32_table_m8(int *count);
const WgKernel *wg32_table_m16(int *count);

const WgKernel *find_wg32_kernel(int R, int M, int mode, int Q, bool ilu) {
  int cnt = 0;
  const WgKernel *t = M == 8 ? wg32_table_m8(&cnt) : (M == 16 ? wg32_table_m16(&cnt) : nullptr);
  for (int i = 0; i < cnt; ++i)
    if (t[i].R == R && t[i].M == M && t[i].mode == mode && t[i].Q == Q && t[i].ilu == ilu) return &t[i];
  return nullptr;
}

const void *stencil_kernel() { return (const void *)&k_stencil; }

const BatchKernel *find_batch_kernel(int R, int M, int fp32, bool uni, bool ilu, int mode, int Q) {
  int cnt = 0;
  const BatchKernel *t = nullptr;
  if (R == 3) {
    if (M == 8) t = batch_table_r3_m8(&cnt);
    else if (M == 16) t = batch_table_r3_m16(&cnt);
    else return nullptr;
  } else switch (M) {
    case 4: t = batch_table_m4(&cnt); break;
    case 6: t = batch_table_m6(&cnt); break;
    case 8: t = batch_table_m8(&cnt); break;
    case 12: t = batch_table_m12(&cnt); break;
    case 16: t = batch_table_m16(&cnt); break;
    case 32: t = batch_table_m32(&cnt); break;
    default: return nullptr;
  }
  for (int i = 0; i < cnt; ++i)
    if (t[i].R == R && t[i].M == M && t[i].fp32 == fp32 && t[i].uni == uni && t[i].ilu == ilu && t[i].mode == mode &&
        t[i].Q == Q)
      return &t[i];
  return nullptr;
}

}  // namespace cb
