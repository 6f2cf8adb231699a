// Kernel argument blocks and dispatch tables shared by kernels.hip and api.cpp.
#pragma once
#include <cstddef>
#include <cstdint>

#include "plan.h"

namespace cb {

// Row layout of a launch: unit-stride lines (MODE_X) or strided lines (MODE_S).
enum { MODE_X = 0, MODE_S = 1 };

// Magic numbers for dividing a 32-bit line index by nu (see FastDiv in device.h).
struct DivMagic {
  uint32_t d, mul, s1, s2;
};
inline DivMagic make_divmagic(uint32_t d) {
  if (d == 0) d = 1;  // an empty grid has no line to index
  uint32_t l = 0;
  while (l < 32 && (uint64_t(1) << l) < d) ++l;
  DivMagic m;
  m.d = d;
  m.mul = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
  m.s1 = l > 0 ? 1 : 0;
  m.s2 = l > 0 ? l - 1 : 0;
  return m;
}

struct LineArgs {
  const double *in;
  double *out;
  int64_t nlines, nu, su, sv, rs;
  DivMagic nudiv;            // line -> (u, v) = (line % nu, line / nu)
  int lgL, lgW, block_sync, refine_iters;
  int coef_lds;              // general layout: coefficient blocks staged in LDS
  int stage_x;               // unit-stride lines go through an LDS tile
  int stage_vec;             // ... read and written as 16-byte pairs (even n, aligned lines)
  int n;                     // line length
  int xcds;                  // > 1: tiles in XCD-grouped order over this many XCDs
  int64_t stage_off;         // LDS offset (doubles) of the tile
  int64_t stage_pitch;       // doubles per line in the tile (n + n/M + 1)
  SegDev seg;
  double stc[7];             // stencil coefficients for q = -3..3 (zero padded)
  double bands[2 * kMaxR + 1];  // constant bands a_{-R..R} (refinement residual)
  const double *bands_row;   // per-row bands [n][2R+1] or nullptr
};

struct WgArgs {
  const double *in;
  double *out;
  double *scratch;           // [nlines][P][3R]
  int64_t nlines, nu, su, sv, rs, n;
  DivMagic nudiv;
  double stc[7];             // fused stencil q = -3..3 (Q > 0 kernels)
  int lgL, lgW, P, nphase;
  int coef_lds;              // stage each partition's coefficient blocks in LDS
  int64_t coef_off_a, coef_off_c;  // their LDS offsets (doubles) in phases A and C
  int stage_x;               // unit-stride lines: load/store through an LDS tile
  int64_t stage_off_a, stage_off_c, stage_pitch;  // its offsets and per-line pitch (doubles)
  const SegDev *segs;        // [P]
  const int *wg_start;       // [P+1]
  const double *bands;       // [n][2R+1] band rows of the line (Eq. (9) couplings)
  const double *SR;          // S^G, R^G per partition
  const int64_t *SR_off;     // [P]
  const double *LtUt;        // [P][2][R][R]
  const int *row_off, *src;  // reduced program
  const double *mats;
  int nterms;                // its terms (src entries, R x R matrices)
  int prog_lds;              // phase B copies the program to LDS first
  const double *bfun;        // [P][2][R][kw] boundary rows of D_i^{-1} (phase A)
  int kw;                    // their window length
  int wave_local;            // phase C: every line lies in one wavefront (its
                             // exchanges need only wavefront-local ordering)
  int sc_stride;             // scratch doubles per (line, partition): 3R, or 4R
                             // when refining (+ the current x at the interface rows)
  SegDev fb;                 // phase C on whole partitions: the full-block plan,
                             // by value so that its fields arrive with the
                             // arguments (partition i starts at row i * fb.S)
  int fb_type;               // ... and its middle lanes' coefficient block
  int part_fast;             // phases A and C: 1D grid, partition fastest
  int band_rows;             // FP64 residual: 1 reads bands per row, 0 band_c
  double band_c[2 * kMaxR + 1];  // constant bands a_{-R..R}
};

struct StencilArgs {
  const double *f;
  double *b;
  int64_t total, n, nu, su, sv, rs;
  int lo, hi;
  double c[7];
};

struct LineKernel {
  int R, M, fp32, mode, Q;
  bool uni, ilu;
  int max_threads;  // workgroup size bound of the instance
  const void *fn;
};
struct WgKernel {
  int R, M, mode, Q;
  bool ilu;                        // lane interiors by banded elimination
  int max_threads;                 // workgroup size bound of phases A and C
  const void *fn_a, *fn_b, *fn_c;  // phases A (interface data), B (reduced system), C (interiors)
  // FP32 + FP64 refinement: phase A forming the residual b - A x, phase C
  // with an FP32 interior solve storing x, and adding its correction to x
  const void *fn_a_res, *fn_c32, *fn_c32_res;
  const void *fn_c_fb;             // FP64 phase C on whole partitions (full-block plans)
  const void *fn_c32_fb, *fn_c32_res_fb;  // ... and its FP32 + refinement forms
};

// Persistent batched launch: queue header and one work-table entry per item.
struct BatchHdr {
  unsigned long long next_tile;  // next tile to hand out
  unsigned int done;             // workgroups that have left
  int n_items;
  int64_t total_tiles;
};
struct BatchItemDev {
  LineArgs a;
  int64_t tile_begin;  // first global tile index of this item
  int mode;
  int pad;
};
struct BatchKernel {
  int R, M, fp32;
  bool uni, ilu;
  int mode, Q, threads;  // row mode, stencil half-width and workgroup size of the instance
  const void *fn;
};
static_assert(sizeof(BatchHdr) <= 64, "batch queue header must fit its 64-byte slot");

// A caller-owned device buffer that P > 1 launches use for their partition
// scratch instead of allocating one.
struct FixedScratch {
  void *ptr;
  size_t bytes;
};

// cb_solve with the partition scratch in `fs` (NULL: the plan's kept
// buffer, or under graph capture a stream-ordered allocation), and the
// error reporting of the C ABI
// (cb_last_error's message).
cb_status solve_entry(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *b, double *x, void *stream,
                      const FixedScratch *fs);
cb_status set_error(cb_status s, const char *msg);

const LineKernel *find_line_kernel(int R, int M, int fp32, int mode, int Q, bool uni, bool ilu);
// copy-only instances (copy_lines.hip): the load and store path of each rows
// per lane, row layout and lane layout
const LineKernel *find_copy_kernel(int M, int mode, bool uni);
const BatchKernel *find_batch_kernel(int R, int M, int fp32, bool uni, bool ilu, int mode, int Q);
const WgKernel *find_wg_kernel(int R, int M, int mode, int Q, bool ilu);
// FP32 + refinement instances of the partitioned kernels (wg_fp32.hip)
const WgKernel *find_wg32_kernel(int R, int M, int mode, int Q, bool ilu);
const void *stencil_kernel();

}  // namespace cb
