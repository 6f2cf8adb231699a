// Kernels of lines split over P > 1 workgroup partitions (Sec. 3-4 with
// workgroups as partitions), shared by the FP64 instances in kernels.hip and
// the FP32 + refinement ones in wg_fp32.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "launch.h"

namespace cb {

// ------------------------------------------------------------------------
// Lines split over P > 1 workgroup partitions (Sec. 3-4 with workgroups as
// partitions).  Phase A: the interface RHS b~_i and the first/last R rows of
// y_i = D_i^{-1} b_i (the only data a partition shares, Sec. 4 on the
// sparsity of L~ and U~) go to a small scratch array; the rows of y_i are
// dot products with the plan's boundary rows of D_i^{-1}.  Phase B: per
// line, b^ (Eq. (21)) and the P-block reduced system (Algorithm 1's level
// loop with detach/reattach, precomputed as a program of phases).  Phase C:
// each partition solves its interior with the interface values as
// right-hand-side couplings (Eq. (9)) and stores.
// FP32 + refinement runs the three phases once on b with the interior solve
// in FP32 (x = the result), then per iteration on the residual r = b - A x,
// formed in FP64 on the fly from b and the stored x, adding the FP32
// correction to x in place.  Phase A then also copies x at each partition's
// interface rows to the scratch array, so that phase C never reads a row
// that another workgroup rewrites.
// ------------------------------------------------------------------------
// The FP64 band entry A[g][g+o] of the residual: constant bands, or the
// plan's per-row table (per-row bands, and the truncated end rows of acyclic
// matrices).
template <int R>
__device__ __forceinline__ double wg_band(const WgArgs &a, int64_t g, int o) {
  return a.band_rows ? a.bands[g * (2 * R + 1) + o + R] : a.band_c[o + R];
}

template <int R, int M, int MODE>
__device__ __forceinline__ void wg_setup(const WgArgs &a, int64_t tile, LanePos &p, int64_t &line, bool &active,
                                         int64_t &base) {
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
  line = tile * p.W + p.li;
  active = line < a.nlines;
  const FastDiv fd{a.nudiv.d, a.nudiv.mul, a.nudiv.s1, a.nudiv.s2};
  const uint32_t line32 = active ? (uint32_t)line : 0u;
  const uint32_t lv = fd.div(line32), lu = line32 - lv * a.nudiv.d;
  base = (int64_t)lu * a.su + (int64_t)lv * a.sv;
}

// Workgroup -> (line tile, partition).  a.part_fast: a 1D grid with the
// partition varying fastest, so workgroups dispatched together read one
// line's partitions one after the other (contiguous memory for unit-stride
// lines: x 249 -> 270 GDOF/s at n = 8192, P = 16; y 3-4 % faster); else a 2D
// grid (tile, part) with the tile varying fastest, for strided lines that
// form one contiguous run across planes (z of a C-order array), whose
// consecutive tiles then read contiguous row segments (3-14 % faster).
__device__ __forceinline__ void wg_block(const WgArgs &a, int64_t &tile, int &part) {
  if (a.part_fast) {
    part = (int)(blockIdx.x % (unsigned)a.P);
    tile = blockIdx.x / (unsigned)a.P;
  } else {
    part = blockIdx.y;
    tile = blockIdx.x;
  }
}

// First row of workgroup partition i (i = P: n).  The full-block form has
// equal partitions of fb.S rows, so no table is read.
template <bool FB>
__device__ __forceinline__ int64_t part_start(const WgArgs &a, int i) {
  return FB ? (int64_t)i * a.fb.S : (int64_t)a.wg_start[i];
}

// Block-PCR levels whose multipliers the full-block form loads with the
// data: tridiagonal partitions of up to 512 rows, log2(512 / M) levels (a
// level more costs registers for nothing: 16-row lanes take 71 VGPRs with 5
// levels, 85 with 6).
template <int R, int M, bool FB>
constexpr int wg_red_prefetch() {
  return FB && R == 1 ? ceil_log2_c(512 / M) : 0;
}

// Solve the interior block D_i of workgroup partition `part` for the lane's
// rows.  With xi/xi1 given (phase C), the right-hand side first loses the
// couplings to the interface unknowns x~_i (first r rows of D_i) and
// x~_{i+1} (last r rows), so the solve returns x_i = D_i^{-1}[b_i - L_i x~_i
// - U_i x~_{i+1}] directly (Eq. (9)).
// Staged unit-stride rows: the L lanes of a line read (or write) its S
// interior rows with consecutive 8-byte words through an LDS tile in which one
// pad word follows every M words.
template <int M>
__device__ __forceinline__ int tile_at(int e) {
  return e + e / M;
}

// T: arithmetic of the interior solve.  RES: the right-hand side is the
// residual b - A x of the current x, whose rows this lane holds in xo on
// return (xif0 / xif1: x at this partition's and the next one's interface
// rows, from the scratch array).
// FB: the whole partition as one block (the full-block plan a.fb): its
// first R rows take the interface values x~_i as identity equations, every
// lane holds M rows and reads the middle lanes' coefficient block through
// the scalar cache (solve_segment's UACYC form).
template <int R, int M, int MODE, int Q, bool ADJ, bool ILU, typename T = double, bool RES = false, bool FB = false>
__device__ __forceinline__ void wg_solve_interior(const WgArgs &a, const LanePos &p, bool active,
                                                  int64_t base, int part, Xchg &xc, double (&v)[M],
                                                  int &start, int &m, double *coef_lds, double *tb,
                                                  const double (&xi)[R], const double (&xi1)[R], double (&xo)[M],
                                                  const double (&xif0)[R], const double (&xif1)[R]) {
  // Every global read that does not depend on the data (lane type, the
  // couplings of the block's end rows to the interface values, the
  // coefficient blocks) is issued together with the data, so the workgroup
  // waits for one round trip to memory instead of several in a row.
  const SegDev &sg = FB ? a.fb : a.segs[part];
  int type;
  if (FB) {
    start = p.l * M;
    m = M;
    type = a.fb_type;
  } else {
    lane_rows(sg.S, p.lgL, p.l, start, m);
    type = sg.lane_type[p.l];
  }
  const int S = sg.S;
  // first row of the block: D_i, or with FB the partition's first row
  const int64_t seg0 = part_start<FB>(a, part) + (FB ? 0 : R);
  const int64_t row0 = seg0 + start;
  const bool staged = MODE == MODE_X && tb != nullptr;
  constexpr int QQ = Q > 0 ? Q : 1;
  double gp[QQ], gn[QQ];  // stencil halo rows beyond D_i's ends
  double t[M];
  if (staged) {
    if (Q > 0) {
#pragma unroll
      for (int i = 0; i < QQ; ++i) {
        const int e0 = start - QQ + i, e1 = start + m + i;
        int64_t r0 = seg0 + e0, r1 = seg0 + e1;
        r0 = r0 < 0 ? r0 + a.n : r0;
        r1 = r1 >= a.n ? r1 - a.n : r1;
        gp[i] = (active && e0 < 0) ? a.in[base + r0 * a.rs] : 0.0;
        gn[i] = (active && e1 >= S) ? a.in[base + r1 * a.rs] : 0.0;
      }
    }
    const double *lin = a.in + base + seg0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int e = p.l + k * p.L;
      t[k] = (active && e < S) ? __builtin_nontemporal_load(lin + e) : 0.0;
    }
  } else {
    const double *in = a.in + base + row0 * a.rs;
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = (active && k < m) ? in[k * a.rs] : 0.0;
    if (Q > 0) {
#pragma unroll
      for (int i = 0; i < QQ; ++i) {
        int64_t r0 = seg0 - QQ + i, r1 = part_start<FB>(a, part + 1) + i;
        r0 = r0 < 0 ? r0 + a.n : r0;
        r1 = r1 >= a.n ? r1 - a.n : r1;
        gp[i] = (active && p.l == 0) ? a.in[base + r0 * a.rs] : 0.0;
        gn[i] = (active && p.l == p.L - 1) ? a.in[base + r1 * a.rs] : 0.0;
      }
    }
  }
  constexpr int TP = wg_red_prefetch<R, M, FB>();
  RedPre<T, R, TP> pre;
  if (TP > 0) red_prefetch<T, R, TP>(sg, p.l, pre);
  if (RES) {  // the current x of the lane's rows (written by the previous phase C)
    const double *xin = a.out + base + row0 * a.rs;
#pragma unroll
    for (int k = 0; k < M; ++k) xo[k] = (active && k < m) ? xin[k * a.rs] : 0.0;
  }
  // Eq. (9): the block's first R rows couple to x~_i (first lane), its last R
  // rows to x~_{i+1} (last lane); those terms move to the right-hand side
  double head[R], tail[R];
#pragma unroll
  for (int c = 0; c < R; ++c) head[c] = tail[c] = 0.0;
  if (ADJ) {
    constexpr int W2 = 2 * R + 1;
    if (p.l == 0 && !FB) {
#pragma unroll
      for (int c = 0; c < R; ++c) {  // row c of D_i
        const double *bd = a.bands + (seg0 + c) * W2;
#pragma unroll
        for (int o = -R; o < 0; ++o)
          if (c + o < 0) head[c] += bd[o + R] * xi[R + c + o];
      }
    }
    if (p.l == p.L - 1) {
#pragma unroll
      for (int c = 0; c < R; ++c) {  // row S-R+c of D_i
        const double *bd = a.bands + (seg0 + S - R + c) * W2;
#pragma unroll
        for (int o = 1; o <= R; ++o)
          if (c + o >= R) tail[c] += bd[o + R] * xi1[c + o - R];
      }
    }
  }
  if (a.coef_lds && !FB) stage_coef<T>(sg, reinterpret_cast<T *>(coef_lds), p.tid, blockDim.x);
  if (staged) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int e = p.l + k * p.L;
      if (e < S) tb[tile_at<M>(e)] = t[k];
    }
    xc.sync();  // the line's tile is read and written by its own lanes only
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = k < m ? tb[tile_at<M>(start + k)] : 0.0;
  }
  if (Q > 0) {  // fused stencil; the halo at the block's ends comes from global memory
    double fp[QQ], fn[QQ];
    if (staged) {  // neighbours inside D_i from the tile, beyond its ends prefetched
#pragma unroll
      for (int i = 0; i < QQ; ++i) {
        const int e0 = start - QQ + i, e1 = start + m + i;
        fp[i] = e0 >= 0 ? tb[tile_at<M>(e0)] : gp[i];
        fn[i] = e1 < S ? tb[tile_at<M>(e1)] : gn[i];
      }
    } else {
      halo<QQ, M>(v, m, false, p, xc, fp, fn);
      if (p.l == 0) {
#pragma unroll
        for (int i = 0; i < QQ; ++i) fp[i] = gp[i];
      }
      if (p.l == p.L - 1) {
#pragma unroll
        for (int i = 0; i < QQ; ++i) fn[i] = gn[i];
      }
    }
    double bb[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int q = -QQ; q <= QQ; ++q) acc += a.stc[q + 3] * row_at<QQ, M>(v, fp, fn, k + q, m, false);
      bb[k] = k < m ? acc : 0.0;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = bb[k];
  }
  if (RES) {  // r = b - A x in FP64; x beyond the lane from its neighbours
    double xp[R], xn[R];
    halo<R, M>(xo, m, false, p, xc, xp, xn);
    if (p.l == 0) {
#pragma unroll
      for (int c = 0; c < R; ++c) xp[c] = xif0[c];  // the rows before D_i: its interface rows
    }
    if (p.l == p.L - 1) {
#pragma unroll
      for (int c = 0; c < R; ++c) xn[c] = xif1[c];  // the rows after D_i: the next interface rows
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (k < m) {
        const int64_t g = seg0 + start + k;
        double ax = 0.0;
#pragma unroll
        for (int o = -R; o <= R; ++o) ax += wg_band<R>(a, g, o) * row_at<R, M>(xo, xp, xn, k + o, m, false);
        v[k] -= ax;
      }
    }
  }
  if (ADJ) {
    if (p.l == 0) {
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = FB ? xi[c] : v[c] - head[c];  // FB: the interface rows' values
    }
    if (p.l == p.L - 1) {
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (k >= m - R && k < m) v[k] -= select_idx(tail, k - (m - R));
    }
  }
  if constexpr (FB && sizeof(T) == sizeof(double)) {
    solve_segment<R, M, T, true, CSRC_GLOBAL, ILU, true, TP>(v, sg, p, type, M, xc, nullptr, &pre);
  } else if constexpr (FB) {  // the FP32 interior solve of the refinement pattern
    T vt[M];
#pragma unroll
    for (int k = 0; k < M; ++k) vt[k] = (T)v[k];
    solve_segment<R, M, T, true, CSRC_GLOBAL, ILU, true, TP>(vt, sg, p, type, M, xc, nullptr, &pre);
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = (double)vt[k];
  } else if constexpr (sizeof(T) == sizeof(double)) {
    if (a.coef_lds)
      solve_segment<R, M, double, false, CSRC_LDS, ILU>(v, sg, p, type, m, xc, coef_lds);
    else
      solve_segment<R, M, double, false, CSRC_GLOBAL, ILU>(v, sg, p, type, m, xc);
  } else {
    T vt[M];
#pragma unroll
    for (int k = 0; k < M; ++k) vt[k] = (T)v[k];
    if (a.coef_lds)
      solve_segment<R, M, T, false, CSRC_LDS, ILU>(vt, sg, p, type, m, xc, reinterpret_cast<const T *>(coef_lds));
    else
      solve_segment<R, M, T, false, CSRC_GLOBAL, ILU>(vt, sg, p, type, m, xc);
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = (double)vt[k];
  }
}

// Workgroup bound of the partitioned kernels: unit-stride 16-row instances
// (LDS tile plus general-layout coefficients) get 256 VGPRs at 512 threads.
template <int M, int MODE>
constexpr int wg_max_threads() {
  return (MODE == MODE_X && M > 8) ? 512 : 1024;
}

// Phase A: what a partition shares with the others.  Only b~_i (the RHS of
// its R interface rows) and the first and last R rows of y_i = D_i^{-1} b_i
// enter the reduced system (Eq. (21); the sparsity of L~ and U~), and those
// rows of y_i are dot products of b_i with the boundary rows of D_i^{-1}
// that the plan holds over a window of kw rows at each end of D_i.  So the
// phase reads only those windows (and the interface rows), computing b on
// the fly when the stencil is fused.  T threads share one (line, partition)
// and take every T-th row of both windows, all loads issued before the
// first product.  Unit-stride lines: 16 lanes each, 4 per wavefront
// (consecutive rows in consecutive lanes, 128-byte segments; windows of up
// to 80 rows in one round of loads), consecutive pairs the partitions of one
// line, summed by a shuffle tree.  Strided
// lines: 4 threads each, 64 adjacent lines per workgroup (one contiguous row
// segment per access), summed through LDS.  Both sums run in a fixed order.
template <int R, int MODE, int Q, bool RES = false>
__global__ __launch_bounds__(256) void k_wg_a(const WgArgs a) {
  extern __shared__ double smem[];
  constexpr int NTA = 256;
  constexpr int T = MODE == MODE_X ? 16 : NTA / 64;
  constexpr int WA = NTA / T;  // lines per workgroup
  const int tid = threadIdx.x;
  const int li = MODE == MODE_X ? tid / T : tid % WA;
  const int t = MODE == MODE_X ? tid % T : tid / WA;
  int part;
  int64_t line;
  if (MODE == MODE_X) {
    // WA (line, partition) pairs per workgroup, the partition varying
    // fastest: neighbouring pairs read adjacent windows (the last one of
    // partition i, the interface rows and the first window of i + 1)
    const int64_t pair = (int64_t)blockIdx.x * WA + li;
    line = pair / a.P;
    part = (int)(pair - line * a.P);
  } else {
    int64_t tile;
    wg_block(a, tile, part);
    line = tile * WA + li;
  }
  const bool active = line < a.nlines;
  const FastDiv fd{a.nudiv.d, a.nudiv.mul, a.nudiv.s1, a.nudiv.s2};
  const uint32_t line32 = active ? (uint32_t)line : 0u;
  const uint32_t lv = fd.div(line32), lu = line32 - lv * a.nudiv.d;
  const double *in = a.in + (int64_t)lu * a.su + (int64_t)lv * a.sv;
  const int64_t g0 = a.wg_start[part];
  const int64_t d0 = g0 + R;  // first row of D_i
  const int N = (int)(a.wg_start[part + 1] - d0);
  const int K = a.kw;
  const double *gf = a.bfun + (size_t)part * 2 * R * K, *gl = gf + (size_t)R * K;
  const double *xin = a.out + (int64_t)lu * a.su + (int64_t)lv * a.sv;  // RES: the current x
  // b of row j of D_i (j < 0: the interface rows), from the fused stencil or
  // the input itself; RES: the residual b - A x of that row, in FP64
  auto rhs = [&](int64_t j) -> double {
    double acc;
    if constexpr (Q > 0) {
      acc = 0.0;
#pragma unroll
      for (int q = -Q; q <= Q; ++q) {
        int64_t r = d0 + j + q;
        r = r < 0 ? r + a.n : (r >= a.n ? r - a.n : r);
        acc += a.stc[q + 3] * in[r * a.rs];
      }
    } else {
      acc = in[(d0 + j) * a.rs];
    }
    if constexpr (RES) {
      const int64_t g = d0 + j;
      double ax = 0.0;
#pragma unroll
      for (int o = -R; o <= R; ++o) {
        int64_t c = g + o;
        c = c < 0 ? c + a.n : (c >= a.n ? c - a.n : c);
        ax += wg_band<R>(a, g, o) * xin[c * a.rs];
      }
      acc -= ax;
    }
    return acc;
  };
  // interface rows first (their loads overlap the windows')
  double bt[R];
#pragma unroll
  for (int c = 0; c < R; ++c) bt[c] = (active && t == 0) ? rhs(c - R) : 0.0;
  double yf[R], yl[R];
#pragma unroll
  for (int c = 0; c < R; ++c) yf[c] = yl[c] = 0.0;
  if (active) {
    // rows t, t+T, ... of the first window [0, K) and of the last [N-K, N)
    constexpr int CH = MODE == MODE_X ? 5 : 12;  // rows per thread and window issued together
    for (int j0 = 0; j0 < K; j0 += CH * T) {
      double bf[CH], bl[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        // a block one row shorter than the window has a zero weight there
        const int j = j0 + u * T + t, jl = N - K + j;
        bf[u] = (j < K && j < N) ? rhs(j) : 0.0;
        bl[u] = (j < K && jl >= 0) ? rhs(jl) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int j = j0 + u * T + t;
        if (j < K) {
#pragma unroll
          for (int c = 0; c < R; ++c) {
            yf[c] += gf[c * K + j] * bf[u];
            yl[c] += gl[c * K + j] * bl[u];
          }
        }
      }
    }
  }
  if (MODE == MODE_X) {
    // the T partial sums of the (line, partition), by a shuffle tree
#pragma unroll
    for (int off = T / 2; off >= 1; off >>= 1) {
#pragma unroll
      for (int c = 0; c < R; ++c) {
        yf[c] += __shfl_xor(yf[c], off, 64);
        yl[c] += __shfl_xor(yl[c], off, 64);
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      smem[(size_t)c * NTA + tid] = yf[c];
      smem[(size_t)(R + c) * NTA + tid] = yl[c];
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double sf = 0.0, sl = 0.0;
#pragma unroll
        for (int u = 0; u < T; ++u) {
          sf += smem[(size_t)c * NTA + u * WA + li];
          sl += smem[(size_t)(R + c) * NTA + u * WA + li];
        }
        yf[c] = sf;
        yl[c] = sl;
      }
    }
  }
  if (t != 0 || !active) return;
  double *sc = a.scratch + (line * a.P + part) * a.sc_stride;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    sc[c] = bt[c];           // b~_i: interface row g0 + c
    sc[R + c] = yf[c];       // first R rows of y_i
    sc[2 * R + c] = yl[c];   // last R rows of y_i
    if (RES) sc[3 * R + c] = xin[(g0 + c) * a.rs];  // x at the interface rows
  }
}

// Phase B: the P-block reduced system of each line, solved once.  Every
// thread owns one (line, partition) pair: it assembles b^_i (Eq. (21)) from
// the scratch values of its partition and the previous one, then the
// precomputed program of Algorithm 1 (block-PCR levels with detach/reattach
// for any P, the final folded solve) runs in LDS; x~_i replaces b~_i in the
// scratch array.  With a.prog_lds the program itself (its term ranges,
// sources and matrices) is copied to LDS first, together with the scratch
// reads, so the phases wait on no memory round trip.
template <int R>
__global__ __launch_bounds__(256) void k_wg_b(const WgArgs a) {
  extern __shared__ double smem[];
  const int P = a.P, NT = blockDim.x;
  const int WB = NT / P > 0 ? NT / P : 1;  // lines per block
  double *cur = smem, *nxt = smem + (size_t)WB * P * R;
  const int64_t line0 = (int64_t)blockIdx.x * WB;
  const int *prog_ro = a.row_off, *prog_src = a.src;
  const double *prog_m = a.mats;
  if (a.prog_lds) {
    double *lm = smem + (size_t)2 * WB * P * R;
    int *lro = reinterpret_cast<int *>(lm + (size_t)a.nterms * R * R);
    int *lsrc = lro + (size_t)a.nphase * (P + 1);
    for (int i = threadIdx.x; i < a.nterms * R * R; i += NT) lm[i] = a.mats[i];
    for (int i = threadIdx.x; i < a.nphase * (P + 1); i += NT) lro[i] = a.row_off[i];
    for (int i = threadIdx.x; i < a.nterms; i += NT) lsrc[i] = a.src[i];
    prog_ro = lro;
    prog_src = lsrc;
    prog_m = lm;
  }
  for (int idx = threadIdx.x; idx < WB * P; idx += NT) {
    const int li = idx / P, j = idx % P;
    const int64_t ln = line0 + li;
    double bh[R];
    if (ln < a.nlines) {
      const double *sj = a.scratch + (ln * P + j) * a.sc_stride;
      const double *sp = a.scratch + (ln * P + (j + P - 1) % P) * a.sc_stride;
      const double *lt = a.LtUt + (size_t)j * 2 * R * R, *ut = lt + R * R;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double acc = sj[r];
#pragma unroll
        for (int c = 0; c < R; ++c) acc -= lt[r * R + c] * sp[2 * R + c] + ut[r * R + c] * sj[R + c];
        bh[r] = acc;
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) bh[r] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) cur[(li * P + j) * R + r] = bh[r];
  }
  __syncthreads();
  for (int ph = 0; ph < a.nphase; ++ph) {
    const int *ro = prog_ro + ph * (P + 1);
    for (int idx = threadIdx.x; idx < WB * P; idx += NT) {
      const int li = idx / P, j = idx % P;
      const int t0 = ro[j], t1 = ro[j + 1];
      double acc[R];
      if (t0 == t1) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = cur[(li * P + j) * R + r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int t = t0; t < t1; ++t) {
          const double *mt = prog_m + (size_t)t * R * R;
          const double *xs = cur + (li * P + prog_src[t]) * R;
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < R; ++c) acc[r] += mt[r * R + c] * xs[c];
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) nxt[(li * P + j) * R + r] = acc[r];
    }
    __syncthreads();
    double *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  for (int idx = threadIdx.x; idx < WB * P; idx += NT) {
    const int li = idx / P, j = idx % P;
    const int64_t ln = line0 + li;
    if (ln >= a.nlines) continue;
    double *sj = a.scratch + (ln * P + j) * a.sc_stride;
#pragma unroll
    for (int r = 0; r < R; ++r) sj[r] = cur[(li * P + j) * R + r];
  }
}

// Phase C: x_i = D_i^{-1}[b_i - L_i x~_i - U_i x~_{i+1}] (Eq. (9), equal to
// the back-substitution of Eq. (22)) from the interface values of phase B.
// T: arithmetic of the interior solve (FP32 for the refinement pattern).
// RES: refinement iteration, the interior solve gives a correction that is
// added to the stored x (the partition's own rows only; the rows it needs
// from the next partition come from the scratch array).
template <int R, int M, int MODE, int Q, bool ILU, typename T = double, bool RES = false, bool FB = false>
__global__ __launch_bounds__((wg_max_threads<M, MODE>())) void k_wg_c(const WgArgs a) {
  extern __shared__ double smem[];
  constexpr int RS = Q > R ? 2 * Q : 2 * R;
  LanePos p;
  int64_t line, base;
  bool active;
  int part;
  int64_t tile;
  wg_block(a, tile, part);
  wg_setup<R, M, MODE>(a, tile, p, line, active, base);
  const int P = a.P, NT = blockDim.x;
  double xi[R], xi1[R], xif0[R], xif1[R];
  {
    const int64_t ln = active ? line : 0;
    const double *s0 = a.scratch + (ln * P + part) * a.sc_stride;
    const double *s1 = a.scratch + (ln * P + (part + 1) % P) * a.sc_stride;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xi[r] = s0[r];
      xi1[r] = s1[r];
      xif0[r] = RES ? s0[3 * R + r] : 0.0;
      xif1[r] = RES ? s1[3 * R + r] : 0.0;
    }
  }
  Xchg xc{smem, RS, NT, 0, a.wave_local == 0};
  double v[M], xo[M];
  int start, m;
  double *tb = a.stage_x ? smem + a.stage_off_c + (size_t)p.li * a.stage_pitch : nullptr;
  wg_solve_interior<R, M, MODE, Q, true, ILU, T, RES, FB>(a, p, active, base, part, xc, v, start, m,
                                                         smem + a.coef_off_c, tb, xi, xi1, xo, xif0, xif1);
  if (RES) {
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] += xo[k];
  }
  const int64_t seg0 = part_start<FB>(a, part) + (FB ? 0 : R);
  if (MODE == MODE_X && tb != nullptr) {
    // mirror of the staged load: every lane has finished reading the tile
    // (its stencil halo) before any lane overwrites it
    xc.sync();
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (k < m) tb[tile_at<M>(start + k)] = v[k];
    xc.sync();
    const int S = FB ? a.fb.S : a.segs[part].S;
    double *lout = a.out + base + seg0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int e = p.l + k * p.L;
      if (active && e < S) __builtin_nontemporal_store(tb[tile_at<M>(e)], lout + e);
    }
  } else if (active) {
    double *out = a.out + base + (seg0 + start) * a.rs;
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (k < m) out[k * a.rs] = v[k];
  }
  if (!active || FB) return;  // FB: the interface rows were stored with the block
  if (p.l == 0) {
    const int64_t g0 = a.wg_start[part];
#pragma unroll
    for (int c = 0; c < R; ++c) a.out[base + (g0 + c) * a.rs] = RES ? xif0[c] + xi[c] : xi[c];
  }
}

}  // namespace cb
