// C ABI of libcb: argument checking, plan upload, launch configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cb.h"
#include "launch.h"
#include "plan.h"

struct cb_plan_s {
  cb::Plan p;
};

namespace cb {
namespace {

thread_local std::string g_err;

// The launches of each built batch workspace: one persistent kernel per
// kernel class, with its queue header, work-table slice and LDS size.
struct BatchLaunch {
  const void *fn;
  size_t hdr_off, items_off, lds;
  int threads;
  int64_t tiles;
};
// An item whose plan splits lines over P > 1 workgroup partitions: it runs
// as its own phase launches, with its partition scratch in the workspace.
struct WgItem {
  cb_plan_t plan;
  const Plan *wp;  // what runs: the plan (P > 1) or its partitioned strided copy
  cb_grid grid;
  int axis;
  const double *in;
  double *out;
  bool has_stencil;
  cb_stencil stencil;
  size_t sc_off, sc_bytes;
};
// Per workspace: its launches, the pinned host copy its table is uploaded
// from, and the event recorded on the build stream after that upload.
struct BatchState {
  std::vector<BatchLaunch> launches;
  std::vector<WgItem> wg_items;
  hipStream_t stream = nullptr;
  hipEvent_t copied = nullptr;
  char *pinned = nullptr;
  size_t cap = 0;
};
std::mutex g_batch_mu;
std::map<void *, BatchState> g_batch;
// workspaces remembered before finished ones are forgotten
constexpr size_t kBatchKeep = 256;

// streams a plan keeps partition scratch for before it drops them all
constexpr size_t kKeptScratchStreams = 16;

// batch workspace layout: kBatchHdrBytes per class header (at most one class
// per item), then the work table from a 256-byte boundary
constexpr size_t kBatchHdrBytes = 64;
size_t batch_items_offset(size_t n_items) { return (std::max<size_t>(n_items, 1) * kBatchHdrBytes + 255) / 256 * 256; }

// LDS a workgroup may allocate on the current device (160 KB on gfx950),
// queried once per device; 64 KB if the query fails.
size_t lds_cap() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  size_t cap = 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    cap = (size_t)v;
  cache[dev] = cap;
  return cap;
}

// Number of XCDs (chiplets with their own L2) of the current device; 1 when
// the runtime does not report it.
int xcd_count() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || v < 1) v = 1;
  cache[dev] = v;
  return v;
}

cb_status fail(cb_status s, const std::string &m) {
  g_err = m;
  return s;
}

cb_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return CB_ERR_HIP;
}

int ilog2(int v) {
  int t = 0;
  while ((1 << t) < v) ++t;
  return t;
}

// --------------------------------------------------------- plan upload ----
struct Arena {
  std::vector<char> host;
  size_t add(const void *src, size_t bytes) {
    const size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + bytes);
    if (bytes) std::memcpy(host.data() + off, src, bytes);
    return off;
  }
  template <typename V> size_t add(const std::vector<V> &v) { return add(v.data(), v.size() * sizeof(V)); }
};

std::vector<float> to_f32(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }

cb_status upload(Plan &p) {
  Arena ar;
  struct SegOff { size_t lt, ls, c64, r64, w64, c32, r32, w32; };
  std::vector<SegOff> so(p.segs.size());
  for (size_t i = 0; i < p.segs.size(); ++i) {
    const SegPlan &s = p.segs[i];
    so[i].lt = ar.add(s.lane_type);
    so[i].ls = ar.add(s.lane_start);
    so[i].c64 = ar.add(s.coef);
    so[i].r64 = ar.add(s.red);
    so[i].w64 = ar.add(s.wf);
    so[i].c32 = ar.add(to_f32(s.coef));
    so[i].r32 = ar.add(to_f32(s.red));
    so[i].w32 = ar.add(to_f32(s.wf));
  }
  const size_t o_bands = ar.add(p.bands);
  size_t o_wg = 0, o_sr = 0, o_sroff = 0, o_ltut = 0, o_ro = 0, o_src = 0, o_mats = 0, o_bfun = 0;
  if (p.P > 1) {
    o_bfun = ar.add(p.bfun);
    o_wg = ar.add(p.wg_start);
    o_sr = ar.add(p.SRg);
    o_sroff = ar.add(p.SRg_off);
    o_ltut = ar.add(p.LtUtg);
    o_ro = ar.add(p.prog.row_off);
    o_src = ar.add(p.prog.src);
    o_mats = ar.add(p.prog.mats);
  }
  const size_t o_segdev = ar.add(nullptr, sizeof(SegDev) * p.segs.size());
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, ar.host.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? fail(CB_ERR_OOM, "cb_plan: device allocation failed")
                                    : hip_fail(e, "cb_plan: hipMalloc");
  }
  char *base = static_cast<char *>(d);
  p.segdev_host.resize(p.segs.size());
  for (size_t i = 0; i < p.segs.size(); ++i) {
    const SegPlan &s = p.segs[i];
    SegDev &g = p.segdev_host[i];
    g.S = s.S;
    g.L = s.L;
    g.M = s.M;
    g.Tint = s.Tint;
    g.Tred = s.Tred;
    g.uniform = s.uniform;
    g.m = s.m_uniform;
    g.block = s.block;
    g.ntypes = s.ntypes;
    g.ilu = s.ilu;
    g.lane_type = reinterpret_cast<const int *>(base + so[i].lt);
    g.lane_start = reinterpret_cast<const int *>(base + so[i].ls);
    g.coef64 = reinterpret_cast<const double *>(base + so[i].c64);
    g.red64 = reinterpret_cast<const double *>(base + so[i].r64);
    g.wf64 = reinterpret_cast<const double *>(base + so[i].w64);
    g.coef32 = reinterpret_cast<const float *>(base + so[i].c32);
    g.red32 = reinterpret_cast<const float *>(base + so[i].r32);
    g.wf32 = reinterpret_cast<const float *>(base + so[i].w32);
  }
  std::memcpy(ar.host.data() + o_segdev, p.segdev_host.data(), sizeof(SegDev) * p.segs.size());
  e = hipMemcpy(d, ar.host.data(), ar.host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "cb_plan: hipMemcpy");
  }
  p.dev_base = d;
  p.dev_bytes = (int64_t)ar.host.size();
  p.segdev = reinterpret_cast<SegDev *>(base + o_segdev);
  p.d_bands = reinterpret_cast<const double *>(base + o_bands);
  if (p.P > 1) {
    p.d_wg_start = reinterpret_cast<const int *>(base + o_wg);
    p.d_SRg = reinterpret_cast<const double *>(base + o_sr);
    p.d_SRg_off = reinterpret_cast<const int64_t *>(base + o_sroff);
    p.d_LtUtg = reinterpret_cast<const double *>(base + o_ltut);
    p.d_row_off = reinterpret_cast<const int *>(base + o_ro);
    p.d_src = reinterpret_cast<const int *>(base + o_src);
    p.d_mats = reinterpret_cast<const double *>(base + o_mats);
    p.d_bfun = reinterpret_cast<const double *>(base + o_bfun);
  }
  if (p.strided_wg) {
    cb_status sw = upload(*p.strided_wg);
    if (sw != CB_OK) {
      (void)hipFree(p.dev_base);
      p.dev_base = nullptr;
      return sw;
    }
  }
  return CB_OK;
}

// ------------------------------------------------------- geometry checks --
struct Geo {
  int64_t n, nu, su, sv, rs, nlines;
};

cb_status geometry(const cb_grid *g, int axis, Geo &o) {
  if (!g) return fail(CB_ERR_INVALID_ARG, "grid is NULL");
  if (axis < 0 || axis > 2) return fail(CB_ERR_INVALID_ARG, "axis must be 0, 1 or 2");
  for (int i = 0; i < 3; ++i)
    if (g->n[i] < 0 || g->stride[i] <= 0)
      return fail(CB_ERR_INVALID_ARG, "grid extents must be non-negative and strides positive");
  if (g->n[axis] == 0) return fail(CB_ERR_INVALID_ARG, "grid extent along the solve axis must be positive");
  const int u = axis == 0 ? 1 : 0, v = axis == 2 ? 1 : 2;
  o.n = g->n[axis];
  o.rs = g->stride[axis];
  o.nu = g->n[u];
  o.su = g->stride[u];
  o.sv = g->stride[v];
  o.nlines = g->n[u] * g->n[v];
  return CB_OK;
}

int64_t span_elems(const cb_grid *g) {
  for (int i = 0; i < 3; ++i)
    if (g->n[i] == 0) return 0;  // empty grid: no element
  int64_t s = 1;
  for (int i = 0; i < 3; ++i) s += (g->n[i] - 1) * g->stride[i];
  return s;
}

// Do [a, a + ea) and [b, b + eb) (FP64 elements) intersect?
bool overlap2(const void *a, int64_t ea, const void *b, int64_t eb) {
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + eb * 8 && pb < pa + ea * 8;
}
bool overlap(const void *a, const void *b, int64_t elems) { return overlap2(a, elems, b, elems); }

void stencil_q(const cb_stencil *st, double out[7]) {
  for (int i = 0; i < 7; ++i) out[i] = 0.0;
  for (int q = st->lo; q <= st->hi; ++q) out[q + 3] = st->coef[q - st->lo];
}

cb_status check_stencil(const cb_stencil *st) {
  if (!st) return fail(CB_ERR_INVALID_ARG, "stencil is NULL");
  if (st->lo < -3 || st->hi > 3 || st->lo > st->hi)
    return fail(CB_ERR_INVALID_ARG, "stencil offsets must satisfy -3 <= lo <= hi <= 3");
  return CB_OK;
}

cb_status launch_wg(const Plan &p, const Geo &g, const double *in, double *out, const cb_stencil *st,
                    hipStream_t stream, const FixedScratch *fs);

// Partition scratch of a P > 1 launch: b~, the two ends of y and, when
// refining, the current x at the interface rows, per (line, partition).
size_t wg_scratch_bytes(const Plan &p, int64_t nlines) {
  const int stride = (p.precision != CB_FP64 && p.refine_iters > 0 ? 4 : 3) * p.R;
  return (size_t)nlines * p.P * stride * sizeof(double);
}
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Workspace bytes of a batch: queue headers and work table, then from a
// 256-byte boundary the partition scratch of each P > 1 item.
// The plan a batch item runs as workgroup-partition phase launches, as a
// single call of it would: the plan itself when it has P > 1, its
// partitioned copy for strided lines when it has one; else nullptr (the
// item's lines run whole in the batched line kernels).
const Plan *batch_wg_plan(const Plan &p, const Geo &g) {
  if (p.P != 1) return &p;
  if (g.rs != 1 && p.strided_wg) return p.strided_wg.get();
  return nullptr;
}

size_t batch_bytes(const cb_batch_item *items, int32_t n_items) {
  const size_t nn = (size_t)(n_items > 0 ? n_items : 0);
  const size_t table = batch_items_offset(nn) + nn * sizeof(BatchItemDev);
  size_t scratch = 0;
  for (int32_t i = 0; i < n_items; ++i) {
    const cb_batch_item &it = items[i];
    if (!it.plan) continue;
    Geo g;
    if (geometry(&it.grid, it.axis, g) != CB_OK) continue;
    const Plan *wp = batch_wg_plan(it.plan->p, g);
    if (wp) scratch += align256(wg_scratch_bytes(*wp, g.nlines));
  }
  return scratch ? align256(table) + scratch : table;
}

// Strided tiles in XCD-grouped order (workgroups are dealt to the XCDs in
// turn, so in launch order neighbouring tiles run on different XCDs):
// automatic when neighbouring tiles share L2 lines -- row segments narrower
// than a 128-byte line, or segments that are not whole aligned lines (the
// tile width does not divide a plane's lines, or the plane pitch is not a
// multiple of 128 bytes: measured +15-37 % for 200-960-row lines of ragged
// planes) -- or when rows lie at most 64 KB apart (measured: 3-4 KB row
// strides gain 4-10 %, 1.5-2 MB ones with whole aligned segments lose 4-10 %).
// Returns the XCD count to group over, or 1 for launch order.
int tile_xcds(const Plan &p, int mode, int W, const Geo &g) {
  const int64_t seg = (int64_t)W * (int64_t)sizeof(double);
  const bool whole = g.su == 1 && seg % 128 == 0 && (g.nlines <= g.nu || (g.nu % W == 0 &&
                                                      (g.sv * (int64_t)sizeof(double)) % 128 == 0));
  const bool on = mode == MODE_S && (p.desc.tile_order == 2 ||
                                     (p.desc.tile_order == 0 &&
                                      (!whole || g.rs * (int64_t)sizeof(double) <= 65536)));
  return on ? xcd_count() : 1;
}

// Bands of the FP64 refinement residual b - A x.  Constant cyclic bands are
// the same on every row and go by value; per-row bands, and acyclic plans
// (whose first and last r rows lose the entries that fall outside the
// matrix), are read per row from the plan's expanded [n][2r+1] table.
void residual_bands(const Plan &p, LineArgs &a) {
  const int W = 2 * p.R + 1;
  const size_t mid = (size_t)(p.n / 2) * W;  // an interior row: every entry present
  for (int o = 0; o < W; ++o) a.bands[o] = p.bands[mid + o];
  a.bands_row = (p.desc.per_row || !p.desc.cyclic) ? p.d_bands : nullptr;
}

// --------------------------------------------------------- P = 1 launch --
// copy: the same launch with the copy-only kernel (no stencil, no solve).
cb_status launch_line(const Plan &p, const Geo &g, const double *in, double *out, const cb_stencil *st,
                      hipStream_t stream, const FixedScratch *fs, bool copy = false) {
  // long strided lines: workgroup partitions of the same matrix (whole lines
  // for in-place FP32 + refinement, whose partitioned form re-reads b)
  if (g.rs != 1 && p.strided_wg && !(in == out && p.strided_wg->refine_iters > 0)) {
    if (copy) return fail(CB_ERR_UNSUPPORTED, "cb_copy_lines: this launch runs in workgroup partitions");
    return launch_wg(*p.strided_wg, g, in, out, st, stream, fs);
  }
  const int si = g.rs == 1 ? 0 : p.seg_s;  // lane layout for this launch's row stride
  const SegPlan &sp = p.segs[si];
  const bool uni = sp.uniform != 0;
  const int Q = st ? (st->lo >= -2 && st->hi <= 2 ? 2 : 3) : 0;
  if (g.nlines >= (int64_t(1) << 31)) return fail(CB_ERR_UNSUPPORTED, "more than 2^31 lines in one call");
  const bool fp32 = p.precision != CB_FP64;
  // MODE_X needs unit row stride.  Its lines go through an LDS tile unless
  // asked otherwise or, automatically, when one line's tile would exceed
  // 64 KB (long lines: the tile would cost occupancy).  The vectorised direct
  // loads of uniform layouts also need 16-byte aligned line starts.
  int mode = (g.rs == 1) ? MODE_X : MODE_S;
  const int64_t tile1 = (g.n + g.n / sp.M + 1 + (int64_t)sp.L * 4 * p.R) * (int64_t)sizeof(double);
  const bool stage_x =
      mode == MODE_X && (p.desc.x_staging == 2 || (p.desc.x_staging == 0 && tile1 <= 65536));
  if (mode == MODE_X && uni && !stage_x) {
    const bool al = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0) &&
                    (g.nu == 1 || g.su % 2 == 0) && (g.nlines <= g.nu || g.sv % 2 == 0) && sp.M % 2 == 0;
    if (!al) mode = MODE_S;
  }
  const LineKernel *lk = copy ? find_copy_kernel(sp.M, mode, uni)
                              : find_line_kernel(p.R, sp.M, fp32 ? 1 : 0, mode, Q, uni, sp.ilu != 0);
  if (!lk) return fail(CB_ERR_UNSUPPORTED, "no kernel instance for this plan layout");
  const void *fn = lk->fn;
  const int L = sp.L;
  if (L > 1024 && p.strided_wg && !copy) return launch_wg(*p.strided_wg, g, in, out, st, stream, fs);
  if (L > 1024) return fail(CB_ERR_UNSUPPORTED, "line needs more than 1024 lanes");
  int W;
  if (p.desc.lines_per_wg > 0) {
    W = p.desc.lines_per_wg;
  } else if (mode == MODE_X) {
    // staged unit-stride lines: one line per workgroup measured best for
    // uniform lanes (512^3), but at least one wavefront per workgroup for
    // short lines; general FP64 layouts (ragged n) 256 threads (n = 200-1000:
    // 3-17 % faster than one 64-thread wavefront or line); direct loads:
    // 512-thread workgroups
    W = stage_x ? std::max(1, (uni || fp32 ? 64 : 256) / L) : std::max(1, 512 / L);
  } else {
    // adjacent lines: 16 (128-byte row segments), 32 with 32 rows per lane.
    // FP32 lines with refinement: at most 512 threads unless that leaves
    // fewer than 8 lines (their three solves pass more workgroup barriers,
    // which cost more in larger workgroups: measured 189 vs 154 GDOF/s for
    // 8 vs 16 lines of 64 lanes)
    W = std::max(1, std::min(sp.M == 32 ? 32 : 16, 1024 / L));
    // 128-row lines on 4 lanes of 32 rows: 64 lines (256 threads; 1-7 %
    // faster than 32 along y and z)
    if (sp.M == 32 && L == 4) W = 64;
    if (fp32 && p.refine_iters > 0) W = std::min(W, std::max(8, 512 / L));
    // FP64 general layouts of r >= 2 over 64 lanes (ragged n of 513..1024
    // rows), on lines that do not form one contiguous run across planes
    // (e.g. along y of a C-order array): 8 lines, 512 threads (pentadiagonal
    // n = 613-1000 along y: 5-18 % faster than 16 lines; along z the two
    // measured either way by plane size)
    const bool contiguous = g.su == 1 && (g.nlines <= g.nu || g.sv == g.nu);
    if (!fp32 && !uni && p.R >= 2 && L == 64 && !contiguous) W = 8;
  }
  // LDS: two exchange regions of max(2Q, 2r) doubles per thread (2r when the
  // unit-stride tile is staged: its halo comes from the tile), within the
  // device's LDS per workgroup
  const int RS = stage_x ? 2 * p.R : std::max(2 * Q, 2 * p.R);
  // general layouts stage their coefficient blocks in LDS when they are small
  const size_t coef_bytes = uni ? 0 : (size_t)sp.ntypes * sp.block * (fp32 ? 4 : 8);
  const bool coef_lds = !uni && coef_bytes <= 16384;
  const size_t coef_dbl = coef_lds ? (coef_bytes + 7) / 8 : 0;
  // unit-stride lines of general layouts (and, on request, uniform ones) are
  // loaded and stored through an LDS tile of W lines
  const int64_t pitch = stage_x ? g.n + g.n / sp.M + 1 : 0;
  auto lds_of = [&](int w) {
    return ((size_t)w * L * 2 * RS + coef_dbl + (size_t)w * pitch) * sizeof(double);
  };
  const size_t cap = lds_cap();
  while (W > 1 && (lds_of(W) > cap || W * L > lk->max_threads)) W /= 2;
  const int NT = W * L;
  if (lds_of(W) > cap || NT > lk->max_threads) {
    // a line longer than one workgroup of this kernel holds: the workgroup
    // partitions of the same matrix when the plan has them (FP64, n > 4096)
    if (p.strided_wg && !copy) return launch_wg(*p.strided_wg, g, in, out, st, stream, fs);
    return fail(CB_ERR_UNSUPPORTED, "line too long for one workgroup of this kernel");
  }
  // lanes of a line are adjacent threads in MODE_X: with L <= 64 a line lies in
  // one wavefront and its exchanges need no workgroup barrier
  const bool wave_local = mode == MODE_X && L <= 64 && (64 % L == 0) && p.desc.block_barriers == 0;
  LineArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.nlines = g.nlines;
  a.nu = g.nu;
  a.su = g.su;
  a.sv = g.sv;
  a.rs = g.rs;
  a.nudiv = make_divmagic((uint32_t)g.nu);
  a.lgL = ilog2(L);
  a.lgW = ilog2(W);
  a.block_sync = wave_local ? 0 : 1;
  a.refine_iters = p.refine_iters;
  a.coef_lds = coef_lds ? 1 : 0;
  a.stage_x = stage_x ? 1 : 0;
  a.stage_vec = (stage_x && g.n % 2 == 0 && sp.M % 2 == 0 && (uintptr_t)in % 16 == 0 && (uintptr_t)out % 16 == 0 &&
                 (g.nu == 1 || g.su % 2 == 0) && (g.nlines <= g.nu || g.sv % 2 == 0))
                    ? 1
                    : 0;
  a.n = (int)g.n;
  a.stage_off = (int64_t)NT * 2 * RS + (int64_t)coef_dbl;
  a.stage_pitch = pitch;
  a.seg = p.segdev_host[si];
  if (st) stencil_q(st, a.stc);
  residual_bands(p, a);
  const size_t lds = lds_of(W);
  const int64_t blocks = (g.nlines + W - 1) / W;
  if (blocks > 0x7fffffff) return fail(CB_ERR_UNSUPPORTED, "too many lines for one launch");
  a.xcds = tile_xcds(p, mode, W, g);
  void *args[] = {&a};
  hipError_t e = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(NT), args, lds, stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return CB_OK;
}

// --------------------------------------------------------- P > 1 launch --
// The 3r values per (line, partition) that phases A-C share live in a
// stream-ordered allocation of the launch, or in the caller's fixed buffer
// `fs` (checked against its size before anything is enqueued).
cb_status launch_wg(const Plan &p, const Geo &g, const double *in, double *out, const cb_stencil *st,
                    hipStream_t stream, const FixedScratch *fs) {
  int mode = (g.rs == 1) ? MODE_X : MODE_S;
  const int Q = st ? (st->lo >= -2 && st->hi <= 2 ? 2 : 3) : 0;  // stencil half-width of the kernel
  if (g.nlines >= (int64_t(1) << 31)) return fail(CB_ERR_UNSUPPORTED, "more than 2^31 lines in one call");
  // the partitions' lane layout for this launch's row stride
  const int so = mode == MODE_S ? p.seg_s : 0;
  const int M = p.segs[so].M;
  const bool fp32 = p.precision != CB_FP64;
  const WgKernel *k = fp32 ? find_wg32_kernel(p.R, M, mode, Q, p.segs[so].ilu != 0)
                           : find_wg_kernel(p.R, M, mode, Q, p.segs[so].ilu != 0);
  if (!k) return fail(CB_ERR_UNSUPPORTED, "no partitioned kernel for this layout");
  const int iters = fp32 ? p.refine_iters : 0;  // refinement iterations after the first solve
  // FP64 phase C on whole partitions when the plan has a full-block plan for
  // this layout (equal partitions of L*M rows, constant bands)
  const int fbi = mode == MODE_S ? p.fb_seg_s : p.fb_seg_u;
  const bool use_fb = fbi >= 0 && p.desc.x_staging != 1 &&
                      (fp32 ? (k->fn_c32_fb != nullptr && k->fn_c32_res_fb != nullptr) : k->fn_c_fb != nullptr);
  const int L = use_fb ? p.segs[fbi].L : p.segs[so].L;
  // unit-stride tiles: 2 lines of a full-block plan (measured fastest; more
  // workgroups of fewer waves each), else 256 threads, which amortise the
  // staging of per-partition coefficients; strided tiles: 16 lines
  int NT = mode == MODE_X ? std::max(L, use_fb ? 128 : 256) : std::min(1024, 16 * L);
  if (p.desc.lines_per_wg > 0) NT = p.desc.lines_per_wg * L;
  NT = std::min(std::max(NT, L), k->max_threads);
  if (L > k->max_threads) return fail(CB_ERR_UNSUPPORTED, "partition needs too many lanes");
  // keep the LDS of phases A and C (lane exchange, coefficients, tile) within
  // the device's LDS per workgroup
  const int RSw = 2 * std::max(p.R, Q);
  size_t coef_doubles = 0;
  for (int i = so; i < so + p.P; ++i) coef_doubles = std::max(coef_doubles, (size_t)p.segs[i].ntypes * p.segs[i].block);
  // (the full-block form reads one coefficient block through the scalar cache)
  const bool coef_lds = coef_doubles * 8 <= 16384 && !use_fb;
  const size_t extra = coef_lds ? coef_doubles : 0;
  // unit-stride lines are loaded and stored through an LDS tile of W lines
  const bool stage_x = mode == MODE_X && p.desc.x_staging != 1;
  int smax = 0;
  for (int i = so; i < so + p.P; ++i) smax = std::max(smax, p.segs[i].S);
  if (use_fb) smax = p.segs[fbi].S;
  const int64_t pitch = stage_x ? smax + smax / M + 1 : 0;
  auto lds_c_of = [&](int nt) { return ((size_t)nt * 2 * RSw + extra + (size_t)(nt / L) * pitch) * 8; };
  // phase B: one thread per (line, partition), 256-thread blocks
  const int NTB = 256, WB = std::max(1, NTB / p.P);
  const size_t lds_b0 = (size_t)2 * WB * p.P * p.R * sizeof(double);
  const size_t nterms = p.prog.src.size();
  const size_t lds_bp = lds_b0 + nterms * p.R * p.R * sizeof(double) +
                        (p.prog.row_off.size() + nterms) * sizeof(int);
  const size_t cap = lds_cap();
  if (lds_b0 > cap) return fail(CB_ERR_UNSUPPORTED, "too many partitions for the reduced solve");
  // the program goes to LDS with the block's values when both fit (always on
  // gfx950 for P <= 64 and r <= 3: at most 104 KB of its 160 KB; the reads
  // from memory remain for a device that reports less)
  const bool prog_lds = lds_bp <= cap;
  const size_t lds_b = prog_lds ? lds_bp : lds_b0;
  while (NT > L && lds_c_of(NT) > cap) NT /= 2;
  if (lds_c_of(NT) > cap) return fail(CB_ERR_UNSUPPORTED, "partition too long for one workgroup");
  const int W = NT / L;
  WgArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.nlines = g.nlines;
  a.nu = g.nu;
  a.su = g.su;
  a.sv = g.sv;
  a.rs = g.rs;
  a.n = g.n;
  a.nudiv = make_divmagic((uint32_t)g.nu);
  if (st) stencil_q(st, a.stc);
  a.lgL = ilog2(L);
  a.lgW = ilog2(W);
  a.P = p.P;
  a.nphase = p.prog.nphase;
  a.coef_lds = coef_lds ? 1 : 0;
  a.coef_off_a = (int64_t)NT * 2 * RSw;
  a.coef_off_c = a.coef_off_a;
  a.stage_x = stage_x ? 1 : 0;
  a.stage_off_a = a.coef_off_a + (int64_t)extra;
  a.stage_off_c = a.coef_off_c + (int64_t)extra;
  a.stage_pitch = pitch;
  a.segs = p.segdev + so;
  a.wg_start = p.d_wg_start;
  a.bands = p.d_bands;
  a.SR = p.d_SRg;
  a.SR_off = p.d_SRg_off;
  a.LtUt = p.d_LtUtg;
  a.row_off = p.d_row_off;
  a.src = p.d_src;
  a.mats = p.d_mats;
  a.nterms = (int)nterms;
  a.prog_lds = prog_lds ? 1 : 0;
  a.bfun = p.d_bfun;
  a.kw = p.Kw;
  // scratch per (line, partition): b~, the two ends of y, and when refining
  // the current x at the interface rows
  a.sc_stride = (iters > 0 ? 4 : 3) * p.R;
  {
    const int W2 = 2 * p.R + 1;
    const size_t mid = (size_t)(p.n / 2) * W2;  // an interior row: every entry present
    for (int o = 0; o < W2; ++o) a.band_c[o] = p.bands[mid + o];
    a.band_rows = (p.desc.per_row || !p.desc.cyclic) ? 1 : 0;
  }
  a.wave_local = (mode == MODE_X && L <= 64 && 64 % L == 0 && p.desc.block_barriers == 0) ? 1 : 0;
  if (use_fb) a.fb = p.segdev_host[fbi];
  a.fb_type = use_fb ? (mode == MODE_S ? p.fb_type_s : p.fb_type_u) : 0;
  // phase A: 256 threads; unit-stride lines 16 lanes each (consecutive rows
  // in consecutive lanes), strided lines 64 adjacent ones per row access
  constexpr int kNTA = 256;
  const int WA = mode == MODE_X ? kNTA / 16 : 64;
  const size_t sbytes = wg_scratch_bytes(p, g.nlines);
  const int64_t tiles = (g.nlines + W - 1) / W;
  const int64_t tiles_a = (g.nlines + WA - 1) / WA;
  // 1D grids with the partition varying fastest (tile * P + part), except for
  // strided lines that form one contiguous run of memory across planes (a
  // C-order array along z): there consecutive tiles of the same partition
  // read contiguous row segments, and the grid is (tile, part), the tile
  // fastest.  Measured at n = 8192, P = 16: y (row strides 0.5-8 KB) 3-4 %
  // faster partition-fastest, z 3-14 % faster tile-fastest
  const bool contiguous_lines = g.su == 1 && (g.nlines <= g.nu || g.sv == g.nu);
  const bool part_fast = g.rs == 1 || !contiguous_lines;
  if (part_fast && std::max(tiles, tiles_a) * p.P >= (int64_t(1) << 31))
    return fail(CB_ERR_UNSUPPORTED, "too many line tiles times partitions for one launch");
  // Partition scratch: the caller's fixed buffer; else the plan's buffer
  // for this stream (grown on demand); while the stream is being captured
  // into a graph, a stream-ordered allocation (a graph memory node)
  hipStreamCaptureStatus capst = hipStreamCaptureStatusNone;
  if (!fs && hipStreamIsCapturing(stream, &capst) != hipSuccess) {
    (void)hipGetLastError();
    capst = hipStreamCaptureStatusNone;
  }
  const bool kept = !fs && capst == hipStreamCaptureStatusNone;
  void *scratch = nullptr;
  hipError_t e = hipSuccess;
  if (fs) {
    if (sbytes > fs->bytes)
      return fail(CB_ERR_UNSUPPORTED, "this solve needs " + std::to_string(sbytes) +
                                          " bytes of partition scratch, more than the " + std::to_string(fs->bytes) +
                                          " bytes of the fixed buffer");
    scratch = fs->ptr;
  } else if (kept) {
    ScratchCache &c = *p.sc;
    std::lock_guard<std::mutex> lk(c.mu);
    void *key = static_cast<void *>(stream);
    if (!c.bufs.count(key) && c.bufs.size() >= kKeptScratchStreams) {
      // many streams: wait for the device, then drop every kept buffer
      e = hipDeviceSynchronize();
      for (auto &kv : c.bufs)
        if (e == hipSuccess && kv.second.first) e = hipFree(kv.second.first);
      c.bufs.clear();
      if (e != hipSuccess) return hip_fail(e, "cb_solve: releasing partition scratch");
    }
    std::pair<void *, size_t> &buf = c.bufs[key];
    if (buf.second < sbytes) {  // grow: after this stream's earlier use of the buffer
      if (buf.first) {
        e = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = hipFree(buf.first);
        buf = {nullptr, 0};
        if (e != hipSuccess) return hip_fail(e, "cb_solve: releasing partition scratch");
      }
      const size_t want = std::max<size_t>(sbytes, 256);
      e = hipMalloc(&buf.first, want);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        c.bufs.erase(key);
        return fail(CB_ERR_OOM, "cb_solve: scratch allocation failed");
      }
      buf.second = want;
    }
    scratch = buf.first;
  } else {
    e = hipMallocAsync(&scratch, std::max<size_t>(sbytes, 256), stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(CB_ERR_OOM, "cb_solve: scratch allocation failed");
    }
  }
  a.scratch = static_cast<double *>(scratch);
  a.part_fast = part_fast ? 1 : 0;
  const dim3 grid = part_fast ? dim3((unsigned)(tiles * p.P)) : dim3((unsigned)tiles, (unsigned)p.P);
  // (unit-stride phase A: WA consecutive (line, partition) pairs per workgroup)
  const dim3 grid_a = mode == MODE_X ? dim3((unsigned)((g.nlines * p.P + WA - 1) / WA))
                      : part_fast    ? dim3((unsigned)(tiles_a * p.P))
                                     : dim3((unsigned)tiles_a, (unsigned)p.P);
  void *args[] = {&a};
  const size_t lds_a = mode == MODE_X ? 0 : (size_t)kNTA * 2 * p.R * sizeof(double);
  const size_t lds_c = lds_c_of(NT);
  // FP64: phases A, B, C once.  FP32: the same with the interior solve in
  // FP32, then per refinement iteration the three phases on the residual,
  // phase C adding its correction to x
  for (int it = 0; it <= iters && e == hipSuccess; ++it) {
    const void *fa = it == 0 ? k->fn_a : k->fn_a_res;
    const void *fc = !fp32     ? (use_fb ? k->fn_c_fb : k->fn_c)
                     : it == 0 ? (use_fb ? k->fn_c32_fb : k->fn_c32)
                               : (use_fb ? k->fn_c32_res_fb : k->fn_c32_res);
    e = hipLaunchKernel(fa, grid_a, dim3(kNTA), args, lds_a, stream);
    if (e == hipSuccess)
      e = hipLaunchKernel(k->fn_b, dim3((unsigned)((g.nlines + WB - 1) / WB)), dim3(NTB), args, lds_b, stream);
    if (e == hipSuccess) e = hipLaunchKernel(fc, grid, dim3(NT), args, lds_c, stream);
  }
  const hipError_t e2 = (fs || kept) ? hipSuccess : hipFreeAsync(scratch, stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return CB_OK;
}

cb_status check_plan_for_solve(cb_plan_t plan) {
  if (!plan) return fail(CB_ERR_INVALID_ARG, "plan is NULL");
  if (plan->p.host_only || !plan->p.dev_base)
    return fail(CB_ERR_INVALID_ARG, "plan was built host-only");
  return CB_OK;
}

}  // namespace

// x = A^{-1} b along one axis: cb_solve (fs == NULL: partitioned lines take
// a stream-ordered scratch allocation) and the allocation-free variant (fs:
// the caller's fixed buffer).
cb_status solve_entry(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *b, double *x, void *stream,
                      const FixedScratch *fs) {
  cb_status s = check_plan_for_solve(plan);
  if (s) return s;
  Geo g;
  if ((s = geometry(grid, axis, g))) return s;
  if (g.n != plan->p.n) return fail(CB_ERR_INVALID_ARG, "grid extent along axis differs from plan n");
  if (g.nlines == 0) return CB_OK;  // empty grid: nothing is read or written
  if (!b || !x) return fail(CB_ERR_INVALID_ARG, "b and x must be non-NULL");
  if (b != x && overlap(b, x, span_elems(grid))) return fail(CB_ERR_INVALID_ARG, "b and x overlap");
  // partitioned refinement re-reads b after x has been written
  if (b == x && plan->p.P > 1 && plan->p.refine_iters > 0)
    return fail(CB_ERR_UNSUPPORTED, "partitioned FP32 + refinement solves need b and x apart (not in place)");
  if (plan->p.P == 1) return launch_line(plan->p, g, b, x, nullptr, static_cast<hipStream_t>(stream), fs);
  return launch_wg(plan->p, g, b, x, nullptr, static_cast<hipStream_t>(stream), fs);
}

cb_status set_error(cb_status s, const char *msg) { return fail(s, msg); }

}  // namespace cb

using namespace cb;

extern "C" {

cb_status cb_plan(const cb_plan_desc *desc, cb_plan_t *out) {
  try {
    if (!desc || !out) return fail(CB_ERR_INVALID_ARG, "desc and out must be non-NULL");
    *out = nullptr;
    cb_plan_s *h = new (std::nothrow) cb_plan_s();
    if (!h) return fail(CB_ERR_OOM, "host allocation failed");
    std::string msg;
    cb_status s = build_plan(*desc, h->p, msg);
    if (s != CB_OK) {
      delete h;
      return fail(s, "cb_plan: " + msg);
    }
    h->p.host_only = desc->host_only;
    if (!desc->host_only) {
      s = upload(h->p);
      if (s != CB_OK) {
        delete h;
        return s;
      }
    }
    *out = h;
    g_err.clear();
    return CB_OK;
  } catch (const std::bad_alloc &) {
    return fail(CB_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(CB_ERR_INVALID_ARG, "cb_plan: unexpected error");
  }
}

cb_status cb_plan_destroy(cb_plan_t plan) {
  if (!plan) return CB_OK;
  cb_status s = CB_OK;
  // the partition scratch the plan (and its strided partitioned form) kept
  // per stream (hipFree waits for work still using it)
  for (cb::Plan *q : {&plan->p, plan->p.strided_wg.get()}) {
    if (!q || !q->sc) continue;
    std::lock_guard<std::mutex> lk(q->sc->mu);
    for (auto &kv : q->sc->bufs) {
      const hipError_t e = kv.second.first ? hipFree(kv.second.first) : hipSuccess;
      if (e != hipSuccess) s = hip_fail(e, "cb_plan_destroy: partition scratch");
    }
    q->sc->bufs.clear();
  }
  if (plan->p.strided_wg && plan->p.strided_wg->dev_base) {
    hipError_t e = hipFree(plan->p.strided_wg->dev_base);
    if (e != hipSuccess) s = hip_fail(e, "cb_plan_destroy: hipFree");
  }
  if (plan->p.dev_base) {
    hipError_t e = hipFree(plan->p.dev_base);
    if (e != hipSuccess) s = hip_fail(e, "cb_plan_destroy: hipFree");
  }
  delete plan;
  return s;
}

cb_status cb_rhs_stencil(const cb_stencil *stencil, const cb_grid *grid, int32_t axis, const double *f,
                         double *b, void *stream) {
  cb_status s = check_stencil(stencil);
  if (s) return s;
  Geo g;
  if ((s = geometry(grid, axis, g))) return s;
  if (g.nlines == 0) return CB_OK;  // empty grid: nothing is read or written
  if (!f || !b) return fail(CB_ERR_INVALID_ARG, "f and b must be non-NULL");
  if (overlap(f, b, span_elems(grid))) return fail(CB_ERR_INVALID_ARG, "f and b overlap");
  StencilArgs a;
  a.f = f;
  a.b = b;
  a.n = g.n;
  a.nu = g.nu;
  a.su = g.su;
  a.sv = g.sv;
  a.rs = g.rs;
  a.total = g.nlines * g.n;
  a.lo = stencil->lo;
  a.hi = stencil->hi;
  for (int i = 0; i < 7; ++i) a.c[i] = i <= stencil->hi - stencil->lo ? stencil->coef[i] : 0.0;
  const int64_t blocks = (a.total + 255) / 256;
  if (blocks > 0x7fffffff) return fail(CB_ERR_UNSUPPORTED, "grid too large for one launch");
  void *args[] = {&a};
  hipError_t e = hipLaunchKernel(stencil_kernel(), dim3((unsigned)blocks), dim3(256), args, 0,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return CB_OK;
}

cb_status cb_solve(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *b, double *x,
                   void *stream) {
  return solve_entry(plan, grid, axis, b, x, stream, nullptr);
}

cb_status cb_apply_derivative(cb_plan_t plan, const cb_stencil *stencil, const cb_grid *grid, int32_t axis,
                              const double *f, double *out, void *stream) {
  cb_status s = check_plan_for_solve(plan);
  if (s) return s;
  if ((s = check_stencil(stencil))) return s;
  Geo g;
  if ((s = geometry(grid, axis, g))) return s;
  if (g.n != plan->p.n) return fail(CB_ERR_INVALID_ARG, "grid extent along axis differs from plan n");
  if (!plan->p.desc.cyclic) return fail(CB_ERR_INVALID_ARG, "the fused stencil needs a cyclic plan");
  if (g.nlines == 0) return CB_OK;  // empty grid: nothing is read or written
  if (!f || !out) return fail(CB_ERR_INVALID_ARG, "f and out must be non-NULL");
  if (overlap(f, out, span_elems(grid))) return fail(CB_ERR_INVALID_ARG, "f and out overlap");
  if (plan->p.P != 1) {
    return launch_wg(plan->p, g, f, out, stencil, static_cast<hipStream_t>(stream), nullptr);
  }
  return launch_line(plan->p, g, f, out, stencil, static_cast<hipStream_t>(stream), nullptr);
}

cb_status cb_copy_lines(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *in, double *out,
                        void *stream) {
  cb_status s = check_plan_for_solve(plan);
  if (s) return s;
  Geo g;
  if ((s = geometry(grid, axis, g))) return s;
  if (g.n != plan->p.n) return fail(CB_ERR_INVALID_ARG, "grid extent along axis differs from plan n");
  if (plan->p.P != 1) return fail(CB_ERR_UNSUPPORTED, "cb_copy_lines: one-partition plans only");
  if (g.nlines == 0) return CB_OK;
  if (!in || !out) return fail(CB_ERR_INVALID_ARG, "in and out must be non-NULL");
  if (overlap(in, out, span_elems(grid))) return fail(CB_ERR_INVALID_ARG, "in and out overlap");
  return launch_line(plan->p, g, in, out, nullptr, static_cast<hipStream_t>(stream), nullptr, true);
}

size_t cb_batch_workspace_size(int32_t n_items) {
  const size_t n = (size_t)(n_items > 0 ? n_items : 0);
  return batch_items_offset(n) + n * sizeof(BatchItemDev);
}

cb_status cb_batch_build(const cb_batch_item *items, int32_t n_items, void *workspace, size_t workspace_bytes,
                         void *stream) {
  if (!items || n_items <= 0) return fail(CB_ERR_INVALID_ARG, "cb_batch_build: no items");
  const size_t need = batch_bytes(items, n_items);
  if (!workspace || workspace_bytes < need)
    return fail(CB_ERR_INVALID_ARG, "cb_batch_build: workspace missing or too small (needs " + std::to_string(need) +
                                        " bytes: cb_batch_workspace_bytes)");
  std::vector<WgItem> wg_items;
  size_t sc_next = align256(batch_items_offset((size_t)n_items) + (size_t)n_items * sizeof(BatchItemDev));
  struct Cls {
    int R, M, fp;
    bool uni, ilu;
    const void *fn;
    int threads;
    size_t lds;
    std::vector<int> members;
  };
  std::vector<Cls> cls;
  std::vector<int> cls_of(n_items);
  std::vector<BatchItemDev> tab(n_items);
  std::vector<int64_t> ntiles(n_items);
  for (int i = 0; i < n_items; ++i) {
    const cb_batch_item &it = items[i];
    cb_status s = check_plan_for_solve(it.plan);
    if (s) return s;
    const Plan &p = it.plan->p;
    Geo g;
    if ((s = geometry(&it.grid, it.axis, g))) return s;
    if (g.n != p.n) return fail(CB_ERR_INVALID_ARG, "cb_batch_build: grid extent differs from plan n");
    if (g.nlines > 0 && (!it.in || !it.out)) return fail(CB_ERR_INVALID_ARG, "cb_batch_build: NULL data pointer");
    if (overlap(it.in, it.out, span_elems(&it.grid)))
      return fail(CB_ERR_INVALID_ARG, "cb_batch_build: in and out overlap");
    if (it.stencil) {
      if ((s = check_stencil(it.stencil))) return s;
      if (!p.desc.cyclic) return fail(CB_ERR_INVALID_ARG, "cb_batch_build: a stencil needs a cyclic plan");
    }
    if (g.nlines >= (int64_t(1) << 31)) return fail(CB_ERR_UNSUPPORTED, "cb_batch_build: more than 2^31 lines");
    if (const Plan *wp = batch_wg_plan(p, g)) {  // its own phase launches, scratch in the workspace
      WgItem w;
      w.plan = it.plan;
      w.wp = wp;
      w.grid = it.grid;
      w.axis = it.axis;
      w.in = it.in;
      w.out = it.out;
      w.has_stencil = it.stencil != nullptr;
      if (it.stencil) w.stencil = *it.stencil;
      w.sc_bytes = wg_scratch_bytes(*wp, g.nlines);
      w.sc_off = sc_next;
      sc_next += align256(w.sc_bytes);
      wg_items.push_back(w);
      cls_of[i] = -1;
      continue;
    }
    // the plan's lane layout for this item's row stride, as a single launch uses
    const int si = g.rs == 1 ? 0 : p.seg_s;
    const SegPlan &sp = p.segs[si];
    const int fp = p.precision != CB_FP64;
    const bool uni = sp.uniform != 0, ilu = sp.ilu != 0;
    const int L = sp.L;
    // tile shape and LDS: unit-stride lines through an LDS tile when it fits
    // in 64 KB (halo from the tile, exchange regions of 2r values), else with
    // direct loads; strided lines as W adjacent lines per row segment.  Items
    // of one kernel class and workgroup size share a launch; W = threads / L.
    const size_t coef_bytes = uni ? 0 : (size_t)sp.ntypes * sp.block * (fp ? 4 : 8);
    const size_t coef_dbl_if = (coef_bytes + 7) / 8;
    // kernels for stencils of half-width 2 (plain solves use the identity)
    // and 3; exchange regions carry the +-Q halo
    const int Qi = (!it.stencil || (it.stencil->lo >= -2 && it.stencil->hi <= 2)) ? 2 : 3;
    const int RSs = std::max(2 * Qi, 2 * p.R);
    int W = 0;
    auto lds_bytes = [&](int RS, bool coef, int64_t pitch) {
      return ((size_t)W * L * 2 * RS + (coef ? coef_dbl_if : 0) + (size_t)W * pitch) * 8;
    };
    int mode = g.rs == 1 ? MODE_X : MODE_S;
    bool stage = false, coef_lds = false;
    int64_t pitch = 0;
    int RS = RSs;
    const BatchKernel *bk = nullptr;
    // workgroup size: 512 threads, or up to the instance's bound when a line
    // needs more lanes (unit stride) or 16 strided lines would not fit
    int nt = 0;
    if (mode == MODE_X) {
      bk = find_batch_kernel(p.R, sp.M, fp, uni, ilu, MODE_X, Qi);
      if (bk) nt = std::min(bk->threads, std::max(512, L));
      if (bk && L <= nt) {
        W = nt / L;
        const int64_t pt = g.n + g.n / sp.M + 1;
        if (lds_bytes(2 * p.R, false, pt) <= 65536) {
          stage = true;
          pitch = pt;
          RS = 2 * p.R;
        } else if (uni) {  // direct loads of a uniform layout use 16-byte vectors
          const bool al = ((uintptr_t)it.in % 16 == 0) && ((uintptr_t)it.out % 16 == 0) &&
                          (g.nu == 1 || g.su % 2 == 0) && (g.nlines <= g.nu || g.sv % 2 == 0) && sp.M % 2 == 0;
          if (!al) mode = MODE_S;
        }
      } else {
        mode = MODE_S;
      }
    }
    if (mode == MODE_S) {
      bk = find_batch_kernel(p.R, sp.M, fp, uni, ilu, MODE_S, Qi);
      // 512 threads, or 16 lines (8 with FP32 refinement, as in launch_line)
      // where lanes need more
      if (bk) nt = std::min(bk->threads, std::max(512, (fp && p.refine_iters > 0 ? 8 : 16) * L));
      // 8 lines of 64 lanes for FP64 general layouts of r >= 2 on lines
      // that are not one contiguous run across planes (as in launch_line)
      const bool contiguous = g.su == 1 && (g.nlines <= g.nu || g.sv == g.nu);
      if (bk && !fp && !uni && p.R >= 2 && L == 64 && !contiguous) nt = std::min(nt, 512);
      if (bk && L <= nt) W = nt / L;
    }
    if (!bk || W == 0)
      return fail(CB_ERR_UNSUPPORTED, "cb_batch_build: no batched kernel for an item's lane layout");
    const void *fn = bk->fn;
    const size_t cap = lds_cap();
    coef_lds = !uni && coef_bytes <= 16384 && lds_bytes(RS, true, pitch) <= cap;
    const size_t lds = lds_bytes(RS, coef_lds, pitch);
    if (lds > cap) return fail(CB_ERR_UNSUPPORTED, "cb_batch_build: an item's tile exceeds the LDS of a workgroup");
    BatchItemDev &d = tab[i];
    std::memset(&d, 0, sizeof(d));
    LineArgs &a = d.a;
    a.in = it.in;
    a.out = it.out;
    a.nlines = g.nlines;
    a.nu = g.nu;
    a.su = g.su;
    a.sv = g.sv;
    a.rs = g.rs;
    a.n = (int)g.n;
    a.nudiv = make_divmagic((uint32_t)g.nu);
    a.lgL = ilog2(L);
    a.lgW = ilog2(W);
    a.xcds = tile_xcds(p, mode, W, g);  // used by one-workgroup-per-tile launches
    // lanes of a unit-stride line are adjacent threads: with L <= 64 a line
    // lies in one wavefront and its exchanges need no workgroup barrier
    a.block_sync = (mode == MODE_X && L <= 64 && 64 % L == 0 && p.desc.block_barriers == 0) ? 0 : 1;
    a.refine_iters = p.refine_iters;
    a.coef_lds = coef_lds ? 1 : 0;
    a.stage_x = stage ? 1 : 0;
    a.stage_vec = (stage && g.n % 2 == 0 && sp.M % 2 == 0 && (uintptr_t)it.in % 16 == 0 &&
                   (uintptr_t)it.out % 16 == 0 && (g.nu == 1 || g.su % 2 == 0) &&
                   (g.nlines <= g.nu || g.sv % 2 == 0))
                      ? 1
                      : 0;
    a.stage_off = (int64_t)W * L * 2 * RS + (coef_lds ? (int64_t)coef_dbl_if : 0);
    a.stage_pitch = pitch;
    a.seg = p.segdev_host[si];
    if (it.stencil) stencil_q(it.stencil, a.stc);
    else a.stc[3] = 1.0;  // identity stencil: b = input
    residual_bands(p, a);
    d.mode = mode;
    ntiles[i] = (g.nlines + W - 1) / W;
    int c = 0;
    while (c < (int)cls.size() && !(cls[c].fn == fn && cls[c].threads == nt)) ++c;
    if (c == (int)cls.size()) cls.push_back(Cls{p.R, sp.M, fp, uni, ilu, fn, nt, 0, {}});
    cls[c].lds = std::max(cls[c].lds, lds);
    cls[c].members.push_back(i);
    cls_of[i] = c;
  }
  for (int i = 0; i < n_items; ++i)
    for (int j = i + 1; j < n_items; ++j)
      if (overlap2(items[i].out, span_elems(&items[i].grid), items[j].out, span_elems(&items[j].grid)))
        return fail(CB_ERR_INVALID_ARG, "cb_batch_build: outputs of two items overlap");
  // workspace: one queue header per class, then the work table grouped by class
  std::vector<char> host(batch_items_offset((size_t)n_items) + (size_t)n_items * sizeof(BatchItemDev), 0);
  std::vector<BatchLaunch> launches;
  size_t slot = 0;
  for (size_t c = 0; c < cls.size(); ++c) {
    int64_t tiles = 0;
    for (int i : cls[c].members) {
      tab[i].tile_begin = tiles;
      tiles += ntiles[i];
      std::memcpy(host.data() + batch_items_offset(n_items) + (slot++) * sizeof(BatchItemDev), &tab[i],
                  sizeof(BatchItemDev));
    }
    BatchHdr h;
    std::memset(&h, 0, sizeof(h));
    h.n_items = (int)cls[c].members.size();
    h.total_tiles = tiles;
    std::memcpy(host.data() + c * kBatchHdrBytes, &h, sizeof(h));
    launches.push_back({cls[c].fn, c * kBatchHdrBytes,
                        batch_items_offset(n_items) + (slot - cls[c].members.size()) * sizeof(BatchItemDev),
                        cls[c].lds, cls[c].threads, tiles});
  }
  // The table goes up from a pinned buffer kept per workspace, in stream
  // order, without waiting on the host: a serving loop keeps admitting work
  // while earlier batches run.  The buffer is rewritten only after its
  // previous upload has finished.
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (g_batch.size() >= kBatchKeep && !g_batch.count(workspace)) {
    for (auto it = g_batch.begin(); it != g_batch.end();) {
      if (it->second.copied && hipEventQuery(it->second.copied) == hipSuccess) {
        (void)hipEventDestroy(it->second.copied);
        if (it->second.pinned) (void)hipHostFree(it->second.pinned);
        it = g_batch.erase(it);
      } else {
        ++it;
      }
    }
  }
  BatchState &bs = g_batch[workspace];
  hipError_t e = hipSuccess;
  if (bs.copied) e = hipEventSynchronize(bs.copied);
  else e = hipEventCreateWithFlags(&bs.copied, hipEventDisableTiming);
  if (e == hipSuccess && bs.cap < host.size()) {
    if (bs.pinned) e = hipHostFree(bs.pinned);
    bs.pinned = nullptr;
    bs.cap = 0;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&bs.pinned), host.size(), hipHostMallocDefault);
    if (e == hipSuccess) bs.cap = host.size();
  }
  if (e != hipSuccess) {  // forget the workspace: its launches must not run on a stale table
    if (bs.copied) (void)hipEventDestroy(bs.copied);
    if (bs.pinned) (void)hipHostFree(bs.pinned);
    g_batch.erase(workspace);
    return hip_fail(e, "cb_batch_build: staging buffer");
  }
  std::memcpy(bs.pinned, host.data(), host.size());
  e = hipMemcpyAsync(workspace, bs.pinned, host.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(bs.copied, st);
  if (e != hipSuccess) {
    bs.launches.clear();
    bs.wg_items.clear();
    return hip_fail(e, "cb_batch_build: copy");
  }
  bs.stream = st;
  bs.launches = std::move(launches);
  bs.wg_items = std::move(wg_items);
  return CB_OK;
}

cb_status cb_batch_launch(void *workspace, int32_t max_ctas, void *stream) {
  if (!workspace) return fail(CB_ERR_INVALID_ARG, "cb_batch_launch: workspace is NULL");
  std::vector<BatchLaunch> ls;
  std::vector<WgItem> wgs;
  hipStream_t built_on = nullptr;
  hipEvent_t copied = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto itr = g_batch.find(workspace);
    if (itr == g_batch.end() || (itr->second.launches.empty() && itr->second.wg_items.empty()))
      return fail(CB_ERR_INVALID_ARG, "cb_batch_launch: workspace was not built");
    ls = itr->second.launches;
    wgs = itr->second.wg_items;
    built_on = itr->second.stream;
    copied = itr->second.copied;
  }
  const hipStream_t ls_stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (ls_stream != built_on) {
    // the table upload was enqueued on another stream: wait for it on the
    // device; a stream being captured cannot wait for work outside the
    // capture, so there the host waits, with this thread's capture mode
    // relaxed for that call
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(ls_stream, &cs);
    if (e != hipSuccess) return hip_fail(e, "cb_batch_launch: capture status");
    if (cs == hipStreamCaptureStatusNone) {
      e = hipStreamWaitEvent(ls_stream, copied, 0);
    } else {
      hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
      e = hipThreadExchangeStreamCaptureMode(&mode);
      if (e == hipSuccess) {
        e = hipEventSynchronize(copied);
        const hipError_t e2 = hipThreadExchangeStreamCaptureMode(&mode);  // restore
        if (e == hipSuccess) e = e2;
      }
    }
    if (e != hipSuccess) return hip_fail(e, "cb_batch_launch: waiting for the table upload");
  }
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "cb_batch_launch: device query");
  for (const BatchLaunch &l : ls) {
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, l.fn, l.threads, l.lds);
    if (e != hipSuccess) return hip_fail(e, "cb_batch_launch: occupancy query");
    int ctas = std::max(1, ncu * std::max(per_cu, 1));
    if (max_ctas > 0) ctas = std::min(ctas, (int)max_ctas);
    int per_tile = 0;
    if (max_ctas < 0) {  // one workgroup per tile instead of the persistent queue
      if (l.tiles > 0x7fffffff) return fail(CB_ERR_UNSUPPORTED, "cb_batch_launch: too many tiles for one grid");
      per_tile = 1;
      ctas = (int)std::max<int64_t>(l.tiles, 1);
    }
    BatchHdr *hdr = reinterpret_cast<BatchHdr *>(static_cast<char *>(workspace) + l.hdr_off);
    const BatchItemDev *its = reinterpret_cast<const BatchItemDev *>(static_cast<char *>(workspace) + l.items_off);
    void *args[] = {&hdr, &its, &per_tile};
    e = hipLaunchKernel(l.fn, dim3(ctas), dim3(l.threads), args, l.lds, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "cb_batch_launch: kernel launch");
  }
  // items split over workgroup partitions: their phase launches, with the
  // partition scratch in the workspace (no allocation, so capturable)
  for (const WgItem &w : wgs) {
    Geo g;
    cb_status s = geometry(&w.grid, w.axis, g);
    if (s) return s;
    if (g.nlines == 0) continue;
    const FixedScratch fs{static_cast<char *>(workspace) + w.sc_off, w.sc_bytes};
    s = launch_wg(*w.wp, g, w.in, w.out, w.has_stencil ? &w.stencil : nullptr, static_cast<hipStream_t>(stream), &fs);
    if (s) return s;
  }
  return CB_OK;
}

size_t cb_batch_workspace_bytes(const cb_batch_item *items, int32_t n_items) {
  if (!items || n_items <= 0) return cb_batch_workspace_size(n_items);
  return batch_bytes(items, n_items);
}

cb_status cb_solve_batched(const cb_batch_item *items, int32_t n_items, void *workspace, size_t workspace_bytes,
                           int32_t max_ctas, void *stream) {
  cb_status s = cb_batch_build(items, n_items, workspace, workspace_bytes, stream);
  if (s) return s;
  return cb_batch_launch(workspace, max_ctas, stream);
}

cb_status cb_plan_get_info(cb_plan_t plan, cb_plan_info *info) {
  if (!plan || !info) return fail(CB_ERR_INVALID_ARG, "plan and info must be non-NULL");
  const Plan &p = plan->p;
  std::memset(info, 0, sizeof(*info));
  info->r = p.R;
  info->n = p.n;
  info->cyclic = p.desc.cyclic;
  info->precision = p.precision;
  info->refine_iters = p.refine_iters;
  info->partitions = p.P;
  info->lanes = p.L;
  info->rows_per_lane = p.M;
  info->uniform = p.segs.empty() ? 0 : p.segs[0].uniform;
  info->interior_levels = p.segs.empty() ? 0 : p.segs[0].Tint;
  info->lane_levels = p.segs.empty() ? 0 : p.segs[0].Tred;
  info->red_phases = p.prog.nphase;
  info->red_pcr_steps = p.prog.pcr_steps;
  info->red_detach_steps = p.prog.detach_steps;
  info->device_bytes = p.dev_bytes + (p.strided_wg ? p.strided_wg->dev_bytes : 0);
  info->rows_per_lane_strided = p.segs.empty() ? 0 : p.segs[p.seg_s].M;
  info->lanes_strided = p.segs.empty() ? 0 : p.segs[p.seg_s].L;
  info->interior_elimination = p.segs.empty() ? 0 : p.segs[0].ilu;
  info->interior_elimination_strided = p.segs.empty() ? 0 : p.segs[p.seg_s].ilu;
  info->partitions_strided = p.strided_wg ? p.strided_wg->P : p.P;
  info->boundary_window = p.Kw;
  info->fullblock_seg = p.fb_seg_u;
  info->fullblock_seg_strided = p.fb_seg_s;
  return CB_OK;
}

cb_status cb_plan_get_schedule(cb_plan_t plan, int32_t *out, int32_t cap, int32_t *len) {
  if (!plan || !len) return fail(CB_ERR_INVALID_ARG, "plan and len must be non-NULL");
  std::vector<int32_t> v;
  for (const auto &lvl : plan->p.prog.detached) {
    for (int d : lvl) v.push_back(d);
    v.push_back(-1);
  }
  *len = (int32_t)v.size();
  if (out)
    for (int32_t i = 0; i < std::min<int32_t>(cap, (int32_t)v.size()); ++i) out[i] = v[i];
  return CB_OK;
}

cb_status cb_plan_get_array(cb_plan_t plan, int32_t seg, int32_t which, double *out, int64_t cap, int64_t *len) {
  if (!plan || !len) return fail(CB_ERR_INVALID_ARG, "plan and len must be non-NULL");
  const Plan &p = plan->p;
  if (seg < 0 || seg >= (int32_t)p.segs.size()) return fail(CB_ERR_INVALID_ARG, "segment index out of range");
  const SegPlan &s = p.segs[seg];
  std::vector<double> v;
  switch (which) {
    case 0: v = s.coef; break;
    case 1: v = s.red; break;
    case 2: v = s.wf; break;
    case 3: v.assign(s.lane_type.begin(), s.lane_type.end()); break;
    case 4: v.assign(s.lane_start.begin(), s.lane_start.end()); break;
    case 5: v = p.SRg; break;
    case 6: v = p.LtUtg; break;
    case 7: v.assign(p.wg_start.begin(), p.wg_start.end()); break;
    case 8: v.assign(p.prog.row_off.begin(), p.prog.row_off.end()); break;
    case 9: v.assign(p.prog.src.begin(), p.prog.src.end()); break;
    case 10: v = p.prog.mats; break;
    case 11: v = {(double)s.S, (double)s.L, (double)s.M, (double)s.R, (double)s.Tint, (double)s.Tred,
                  (double)s.ilu, (double)s.uniform, (double)s.cyclic};
      break;
    case 12: v = p.bfun; break;
    default: return fail(CB_ERR_INVALID_ARG, "unknown array id");
  }
  *len = (int64_t)v.size();
  if (out) std::memcpy(out, v.data(), sizeof(double) * (size_t)std::min<int64_t>(cap, (int64_t)v.size()));
  return CB_OK;
}

const char *cb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
