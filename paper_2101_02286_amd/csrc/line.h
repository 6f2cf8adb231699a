// Line-solver kernel template (one-partition lines) shared by the per-M
// translation units lines_m*.hip and by the batched launch in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "launch.h"

namespace cb {

// Workgroup size bound of a line-kernel instance.  FP64 instances fit 128
// VGPRs and allow 1024 threads, except general-layout unit-stride ones (LDS
// tile plus per-lane coefficients); FP32 instances carry the FP64
// refinement state beside the FP32 reduction and get up to 256 VGPRs by
// allowing at most 512 threads.
template <int R, int M, typename T, int MODE, bool UNI>
constexpr int line_max_threads() {
  return sizeof(T) == 4 ? ((R == 1 && M <= 8 && MODE == 1) ? 1024 : 512) : ((UNI || MODE == 1) ? 1024 : 512);
}

// Exchange region size (doubles per thread and region): the halo exchange
// carries 2Q values, the refinement residual and the lane reduction 2r.
// Staged unit-stride launches use 2r (their halo comes from the LDS tile).
template <int R, int Q, int MODE>
constexpr int line_region() {
  return 2 * Q > 2 * R ? 2 * Q : 2 * R;
}

// ------------------------------------------------------------------------
// Line solver for one-partition lines (P = 1): load -> [stencil] -> solve
// [-> FP64 residual refinement] -> store, all on chip.  One workgroup per
// tile of W lines; the L lanes of a line hold its rows in registers.
// MODE_X: rows of a line are contiguous (unit stride); a line's lanes are
//         adjacent threads.  MODE_S: strided rows; threads of equal lane
//         index cover W adjacent lines so each row access is one contiguous
//         W*8-byte segment.
// ------------------------------------------------------------------------
// COPY: the same loads, tile and stores with the stencil and the solve left
// out (x = b), the access pattern's own ceiling for the roofline.
template <int R, int M, typename T, int MODE, int Q, bool UNI, bool ILU = false, bool COPY = false>
__device__ __forceinline__ void line_tile(const LineArgs &a, int64_t tile, double *smem) {
  constexpr int RS = line_region<R, Q, MODE>();
  LanePos p;
  p.tid = threadIdx.x;
  p.lgL = a.lgL;
  p.lgW = a.lgW;
  p.L = 1 << a.lgL;
  p.W = 1 << a.lgW;
  p.mode = MODE;
  if (MODE == MODE_X) {
    p.li = p.tid >> p.lgL;
    p.l = p.tid & (p.L - 1);
  } else {
    p.l = p.tid >> p.lgW;
    p.li = p.tid & (p.W - 1);
  }
  // staged unit-stride lines take their stencil halo from the tile, so their
  // exchange regions only carry the 2r values of the lane reduction
  const bool staged = MODE == MODE_X && a.stage_x;
  const int RSr = staged ? 2 * R : RS;
  Xchg xc{smem, RSr, (int)blockDim.x, 0, a.block_sync != 0};
  const SegDev &sg = a.seg;
  const int nrow = sg.S;  // line length (the whole line is this plan's one segment)
  const int64_t line = tile * p.W + p.li;
  const bool active = line < a.nlines;
  const FastDiv fd{a.nudiv.d, a.nudiv.mul, a.nudiv.s1, a.nudiv.s2};
  const uint32_t line32 = active ? (uint32_t)line : 0u;
  const uint32_t lv = fd.div(line32), lu = line32 - lv * a.nudiv.d;
  const int64_t base = (int64_t)lu * a.su + (int64_t)lv * a.sv;
  int start, m, type = 0;
  if (UNI) {
    m = M;
    start = p.l * M;
  } else {
    lane_rows(sg.S, p.lgL, p.l, start, m);
    type = sg.lane_type[p.l];
  }
  const int64_t rs = MODE == MODE_X ? 1 : a.rs;
  const double *in = a.in + base + start * rs;
  // 32-row strided lanes: the output row as a uniform distance from the input
  // row, so only one address stays live through the solve (that instance
  // otherwise spills two 8-byte values per thread; the others spill more
  // with this form)
  double *out = (MODE == MODE_S && M == 32) ? const_cast<double *>(in) + (a.out - a.in)
                                            : a.out + base + start * rs;

  // MODE_X: a lane's rows are one contiguous 8M-byte run, so one vector load
  // instruction touches many cache lines partially; these loads go through
  // the caches (a streaming hint would drop the lines between the partial
  // accesses).  MODE_S: every row access is a whole 128- or 256-byte segment
  // of W adjacent lines, read once, so the loads are marked streaming.
  // Staged unit-stride path: the line's L lanes read it with consecutive
  // 8-byte words (whole cache lines per instruction) into an LDS tile where
  // one pad word follows every M words, so each lane's M contiguous rows are
  // read back without bank conflicts.
  double *tb = nullptr;
  if (staged) tb = smem + a.stage_off + (size_t)p.li * a.stage_pitch;
  double b64[M];
  if (staged) {
    const double *lin = a.in + base;
    if (a.stage_vec) {  // 16-byte pairs: rows 2e, 2e+1 share a pad group (M even)
      const dbl2 *lin2 = reinterpret_cast<const dbl2 *>(lin);
      dbl2 t2[M / 2];
#pragma unroll
      for (int k = 0; k < M / 2; ++k) {
        const int e2 = p.l + k * p.L;
        t2[k] = (active && 2 * e2 < nrow) ? __builtin_nontemporal_load(lin2 + e2) : dbl2{0.0, 0.0};
      }
#pragma unroll
      for (int k = 0; k < M / 2; ++k) {
        const int e = 2 * (p.l + k * p.L);
        if (e < nrow) {
          tb[e + e / M] = t2[k].x;
          tb[e + e / M + 1] = t2[k].y;
        }
      }
    } else {
      double t[M];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int e = p.l + k * p.L;
        t[k] = (active && e < nrow) ? __builtin_nontemporal_load(lin + e) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int e = p.l + k * p.L;
        if (e < nrow) tb[e + e / M] = t[k];
      }
    }
    xc.sync();
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int e = start + k;
      b64[k] = (UNI || k < m) ? tb[e + e / M] : 0.0;
    }
  } else if (MODE == MODE_X && UNI && (M % 2 == 0)) {
    const dbl2 *in2 = reinterpret_cast<const dbl2 *>(in);
#pragma unroll
    for (int k = 0; k < M / 2; ++k) {
      dbl2 t = active ? in2[k] : dbl2{0.0, 0.0};
      b64[2 * k] = t.x;
      b64[2 * k + 1] = t.y;
    }
  } else if (MODE == MODE_X) {
#pragma unroll
    for (int k = 0; k < M; ++k) b64[k] = (active && (UNI || k < m)) ? in[k] : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < M; ++k) b64[k] = (active && (UNI || k < m)) ? __builtin_nontemporal_load(in + k * rs) : 0.0;
  }

  if (Q > 0 && !COPY) {  // fused right-hand-side stencil (Eq. (1)/(2)), periodic
    constexpr int QQ = Q > 0 ? Q : 1;
    double fp[QQ], fn[QQ];
    if (staged) {  // the neighbouring rows are in the LDS tile
#pragma unroll
      for (int i = 0; i < QQ; ++i) {
        int e = start - QQ + i;
        e = e < 0 ? e + nrow : e;
        fp[i] = tb[e + e / M];
        e = start + m + i;
        e = e >= nrow ? e - nrow : e;
        fn[i] = tb[e + e / M];
      }
    } else {
      halo<QQ, M>(b64, m, UNI, p, xc, fp, fn);
    }
    double bb[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int q = -Q; q <= Q; ++q) acc += a.stc[q + 3] * row_at<(Q > 0 ? Q : 1), M>(b64, fp, fn, k + q, m, UNI);
      bb[k] = (UNI || k < m) ? acc : 0.0;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) b64[k] = bb[k];
  }

  // general layouts: the lanes read different coefficient blocks, staged in LDS
  T *cl = nullptr;
  if (!UNI && a.coef_lds && !COPY) {
    cl = reinterpret_cast<T *>(smem + (size_t)2 * RSr * blockDim.x);
    stage_coef<T>(sg, cl, p.tid, blockDim.x);
  }
  auto solve = [&](T(&v)[M]) {
    if (!UNI && a.coef_lds)
      solve_segment<R, M, T, UNI, CSRC_LDS, ILU>(v, sg, p, type, m, xc, cl);
    else
      solve_segment<R, M, T, UNI, CSRC_GLOBAL, ILU>(v, sg, p, type, m, xc);
  };

  double x64[M];
  if (COPY) {
#pragma unroll
    for (int k = 0; k < M; ++k) x64[k] = b64[k];
  } else if (sizeof(T) == 8) {
    T v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = (T)b64[k];
    solve(v);
#pragma unroll
    for (int k = 0; k < M; ++k) x64[k] = (double)v[k];
  } else {
    // FP32 reduction with FP64 residual refinement: x <- x + A32^{-1}(b - A x)
#pragma unroll
    for (int k = 0; k < M; ++k) x64[k] = 0.0;
    for (int it = 0; it <= a.refine_iters; ++it) {
      T v[M];
      if (it == 0) {
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (T)b64[k];
      } else {
        double xp[R], xn[R];
        halo<R, M>(x64, m, UNI, p, xc, xp, xn);
#pragma unroll
        for (int k = 0; k < M; ++k) {
          v[k] = (T)0;
          if (UNI || k < m) {  // padding slots (k >= m) have no row
            double ax = 0.0;
            const double *bd = a.bands_row ? a.bands_row + (int64_t)(start + k) * (2 * R + 1) : a.bands;
#pragma unroll
            for (int o = -R; o <= R; ++o) ax += bd[o + R] * row_at<R, M>(x64, xp, xn, k + o, m, UNI);
            v[k] = (T)(b64[k] - ax);
          }
        }
      }
      solve(v);
#pragma unroll
      for (int k = 0; k < M; ++k) x64[k] += (double)v[k];
    }
  }

  if (staged) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int e = start + k;
      if (UNI || k < m) tb[e + e / M] = x64[k];
    }
    xc.sync();
    if (!active) return;
    double *lout = a.out + base;
    if (a.stage_vec) {
      dbl2 *lout2 = reinterpret_cast<dbl2 *>(lout);
#pragma unroll
      for (int k = 0; k < M / 2; ++k) {
        const int e = 2 * (p.l + k * p.L);
        if (e < nrow) __builtin_nontemporal_store(dbl2{tb[e + e / M], tb[e + e / M + 1]}, lout2 + e / 2);
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int e = p.l + k * p.L;
        if (e < nrow) __builtin_nontemporal_store(tb[e + e / M], lout + e);
      }
    }
    return;
  }
  if (!active) return;
  if (MODE == MODE_X && UNI && (M % 2 == 0)) {
    dbl2 *out2 = reinterpret_cast<dbl2 *>(out);
#pragma unroll
    for (int k = 0; k < M / 2; ++k) out2[k] = dbl2{x64[2 * k], x64[2 * k + 1]};
  } else if (MODE == MODE_X) {
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (UNI || k < m) out[k] = x64[k];
  } else {
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (UNI || k < m) __builtin_nontemporal_store(x64[k], out + k * rs);
  }
}

template <int R, int M, typename T, int MODE, int Q, bool UNI, bool ILU, bool COPY = false>
__global__ __launch_bounds__((line_max_threads<R, M, T, MODE, UNI>())) void k_line(const LineArgs a) {
  extern __shared__ double smem[];
  uint32_t tile = blockIdx.x;
  if (a.xcds > 1) {
    // workgroup b runs on XCD b mod X; XCD j takes the j-th contiguous range
    // of tiles (the first G mod X ranges one tile longer), in order
    const uint32_t X = (uint32_t)a.xcds, G = gridDim.x, q = G / X, rem = G % X;
    const uint32_t j = tile % X, s = tile / X;
    tile = j * q + (j < rem ? j : rem) + s;
  }
  if constexpr (sizeof(T) == 4 && UNI && M >= 8 && (M >= 12 || R >= 2)) {
    // FP32 uniform lanes of 12 or more rows (8 or more for r >= 2): the
    // arguments are read from the kernel argument segment (where `a`, the
    // only explicit argument, sits at offset 0) through a pointer the
    // compiler cannot trace back to it, so each field is loaded (a scalar
    // load) where it is used instead of all being loaded at entry and held
    // in SGPRs for the whole kernel, which next to the FP32 reduction and the
    // FP64 refinement state spills SGPRs into VGPR lanes (16-row lanes:
    // 194-256 VGPRs and 2 waves per SIMD, against 121-134 and 3-4 this way).
    // Where nothing spills (8-row tridiagonal lanes, general layouts) the
    // loads at the point of use only add latency, so those keep the plain
    // form.  (Taking the address of `a` instead would make the compiler copy
    // it to private memory.)
    using ArgsC = __attribute__((address_space(4))) const LineArgs;
    ArgsC *ap = (ArgsC *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(ap));
    line_tile<R, M, T, MODE, Q, UNI, ILU, COPY>(*(const LineArgs *)ap, (int64_t)tile, smem);
  } else {
    line_tile<R, M, T, MODE, Q, UNI, ILU, COPY>(a, (int64_t)tile, smem);
  }
}


// ------------------------------------------------------------------------
// Batched launch over the lines of many (grid, axis, plan) items of uneven
// sizes, all of one kernel class (r, rows per lane, arithmetic, lane layout,
// interior solve, unit-stride or strided rows, stencil half-width Q).  Every
// item runs with the fused stencil (an identity stencil for plain solves)
// and its own tile shape.  One workgroup per tile, or persistent: the grid
// takes tiles from a device work queue; a workgroup leaves when the queue is
// exhausted, and the last one to leave resets the queue so the launch can be
// replayed (e.g. from a captured graph) without a memset.
// ------------------------------------------------------------------------
template <int R, int M, typename T, bool UNI, bool ILU, int MODE, int Q>
__global__ __launch_bounds__((line_max_threads<R, M, T, MODE, UNI>())) void k_batched(BatchHdr *hdr,
                                                                               const BatchItemDev *__restrict__ items,
                                                                               int per_tile) {
  extern __shared__ double smem[];
  __shared__ int64_t s_tile;
  const int64_t total = hdr->total_tiles;
  const int nitems = hdr->n_items;
  if (per_tile) {
    // one workgroup per tile (no queue); within an item whose tile order is
    // XCD-grouped (as a single launch of it would take), the workgroups of
    // one XCD (every X-th) take one contiguous range of its tiles
    const int64_t t = blockIdx.x;
    if (t >= total) return;
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const BatchItemDev &it = items[lo];
    int64_t local = t - it.tile_begin;
    if (it.a.xcds > 1) {
      const int64_t G = (lo + 1 < nitems ? items[lo + 1].tile_begin : total) - it.tile_begin;
      const int64_t X = it.a.xcds, q = G / X, rem = G % X, j = local % X, s = local / X;
      local = j * q + (j < rem ? j : rem) + s;
    }
    line_tile<R, M, T, MODE, Q, UNI, ILU>(it.a, local, smem);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(&hdr->next_tile, 1ull);
    __syncthreads();
    const int64_t t = s_tile;
    __syncthreads();
    if (t >= total) break;
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const BatchItemDev &it = items[lo];
    line_tile<R, M, T, MODE, Q, UNI, ILU>(it.a, t - it.tile_begin, smem);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(&hdr->done, 1u);
    if (prev == gridDim.x - 1) {
      atomicExch(&hdr->next_tile, 0ull);
      atomicExch(&hdr->done, 0u);
      __threadfence();
    }
  }
}

#define CB_BATCH_INSTQ(R, M, T, UNI, ILU, MODE, Q)                                                \
  {R, M, sizeof(T) == 8 ? 0 : 1, UNI, ILU, MODE, Q, line_max_threads<R, M, T, MODE, UNI>(),        \
   (const void *)&k_batched<R, M, T, UNI, ILU, MODE, Q>}
#define CB_BATCH_INST(R, M, T, UNI, ILU, MODE) \
  CB_BATCH_INSTQ(R, M, T, UNI, ILU, MODE, 2), CB_BATCH_INSTQ(R, M, T, UNI, ILU, MODE, 3)
#define CB_BATCH_MODE(R, M, T, UNI, ILU) CB_BATCH_INST(R, M, T, UNI, ILU, MODE_X), CB_BATCH_INST(R, M, T, UNI, ILU, MODE_S)
#define CB_BATCH_T(R, M, UNI, ILU) CB_BATCH_MODE(R, M, double, UNI, ILU), CB_BATCH_MODE(R, M, float, UNI, ILU)
#define CB_BATCH_R(M, UNI, ILU) CB_BATCH_T(1, M, UNI, ILU), CB_BATCH_T(2, M, UNI, ILU)

#define CB_LINE_INST(R, M, T, MODE, Q, UNI, ILU) \
  {R, M, sizeof(T) == 8 ? 0 : 1, MODE, Q, UNI, ILU, line_max_threads<R, M, T, MODE, UNI>(), \
   (const void *)&k_line<R, M, T, MODE, Q, UNI, ILU>}
#define CB_LINE_Q(R, M, T, MODE, UNI, ILU)                                             \
  CB_LINE_INST(R, M, T, MODE, 0, UNI, ILU), CB_LINE_INST(R, M, T, MODE, 2, UNI, ILU), \
      CB_LINE_INST(R, M, T, MODE, 3, UNI, ILU)
#define CB_LINE_MODE(R, M, T, UNI, ILU) CB_LINE_Q(R, M, T, MODE_X, UNI, ILU), CB_LINE_Q(R, M, T, MODE_S, UNI, ILU)
#define CB_LINE_T(R, M, UNI, ILU) CB_LINE_MODE(R, M, double, UNI, ILU), CB_LINE_MODE(R, M, float, UNI, ILU)
#define CB_LINE_R(M, UNI, ILU) CB_LINE_T(1, M, UNI, ILU), CB_LINE_T(2, M, UNI, ILU)

// Per-M instance tables of the line and batched kernels (lines_m<M>.hip).
const LineKernel *line_table_m4(int *count);
const LineKernel *line_table_m6(int *count);
const LineKernel *line_table_m8(int *count);
const LineKernel *line_table_m12(int *count);
const LineKernel *line_table_m16(int *count);
const LineKernel *line_table_m32(int *count);
const BatchKernel *batch_table_m4(int *count);
const BatchKernel *batch_table_m6(int *count);
const BatchKernel *batch_table_m8(int *count);
const BatchKernel *batch_table_m12(int *count);
const BatchKernel *batch_table_m16(int *count);
const BatchKernel *batch_table_m32(int *count);
// heptadiagonal (r = 3) instances (lines_r3_m<M>.hip)
const LineKernel *line_table_r3_m8(int *count);
const LineKernel *line_table_r3_m16(int *count);
const BatchKernel *batch_table_r3_m8(int *count);
const BatchKernel *batch_table_r3_m16(int *count);

}  // namespace cb
