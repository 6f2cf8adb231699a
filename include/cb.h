/*
 * cb.h -- C ABI of libcb.so: batched solution of cyclic (or acyclic) compact
 * banded systems A x = b by parallel cyclic reduction on AMD Instinct MI355X
 * (gfx950), for compact finite-difference derivatives and interpolation along
 * x, y or z of a 3D grid.
 *
 * Method (Song et al., "Scalable parallel linear solver for compact banded
 * systems on heterogeneous architectures"):
 *   - A has bandwidth w = 2r+1 (Sec. 2; r = 1 tridiagonal, r = 2
 *     pentadiagonal) and is cyclic when the grid is periodic (Sec. 3).
 *   - Each line is split into partitions; the first r rows of a partition are
 *     its interface rows, the rest an acyclic banded block D_i (Sec. 3, the
 *     partitioned system of Eqs. (7)-(8)).
 *   - D_i y_i = b_i, D_i S_i = L_i, D_i R_i = U_i are solved by generalized
 *     PCR (Sec. 2 Eqs. (3)-(6); Sec. 4 Eqs. (15)-(17)); the interface unknowns
 *     form the reduced block system of Eqs. (18)-(21), solved by block PCR
 *     with detach/reattach for sizes that are not powers of two (Sec. 3, the
 *     11x11 example; Sec. 4, Algorithms 1-4); Eq. (22) back-substitutes.
 *   - A is constant while b varies, so everything that does not depend on b
 *     is computed once by cb_plan and kept on the device (Sec. 4, the
 *     paragraph on pre-factorisation).
 *
 * Conventions for every entry point:
 *   - Data pointers (f, b, x, out) are DEVICE pointers to FP64 arrays owned
 *     by the caller.  Host pointers (desc, bands, grid, stencil) are read
 *     during the call only.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous with respect to the host: they enqueue kernels and return.
 *   - Arguments are validated before anything is enqueued; on an error no
 *     output is written, the call returns a non-zero cb_status and
 *     cb_last_error() holds a message.  No C++ exception crosses the ABI.
 *   - A plan may be used from several host threads and streams at once; it
 *     is read-only after cb_plan returns.  Calls that write the same output
 *     on different streams race, as any two kernels would.
 */
#ifndef CB_H
#define CB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CB_OK = 0,
  CB_ERR_INVALID_ARG = 1, /* bad pointer, size, axis, stride or descriptor */
  CB_ERR_UNSUPPORTED = 2, /* valid request the library does not implement */
  CB_ERR_SINGULAR = 3,    /* cb_plan: a pivot or reduction system is singular */
  CB_ERR_OOM = 4,         /* device allocation failed */
  CB_ERR_HIP = 5          /* a HIP runtime call failed; see cb_last_error() */
} cb_status;

typedef enum {
  CB_FP64 = 0,        /* every step in FP64 */
  CB_FP32 = 1,        /* reduction arithmetic in FP32, FP64 input/output */
  CB_FP32_REFINE = 2  /* FP32 reduction + FP64 residual iterative refinement */
} cb_precision;

typedef struct cb_plan_s *cb_plan_t;

/* The problem statement A x = b (Sec. 2-3). */
typedef struct {
  int32_t r;             /* half bandwidth: 1 tridiagonal, 2 pentadiagonal, 3
                            heptadiagonal (1..3; r = 3 takes rows_per_lane
                            0, 8 or 16) */
  int32_t n;             /* system (line) length */
  const double *bands;   /* HOST.  per_row = 0: 2r+1 values a_{-r..r}, row j reads
                            A[j][j+o] = a_o.  per_row = 1: n*(2r+1) values,
                            row-major [row][o+r].  Column indices wrap modulo n
                            when cyclic; when acyclic, entries whose column
                            falls outside [0,n) are ignored. */
  int32_t per_row;       /* 0 constant coefficients, 1 per-row bands */
  int32_t cyclic;        /* 1 periodic (corner blocks present), 0 acyclic */
  int32_t partitions;    /* P >= 1 workgroup partitions per line (Sec. 3 p);
                            P > 1 solves the reduced P-block system across
                            workgroups (any P, detach/reattach when P is not a
                            power of two).  0 = let the library choose: 1
                            while a line fits one workgroup (n <= 16384 in
                            FP64, n <= 8192 in FP32), else ceil(n / 1024) up
                            to 64.  FP32 + refinement with P > 1 refines
                            across the partitions (each iteration runs the
                            partitioned solve on the FP64 residual) and
                            needs b and x apart. */
  int32_t precision;     /* cb_precision */
  int32_t refine_iters;  /* CB_FP32_REFINE: refinement iterations, 1..8, or 0:
                            automatic, the fewest k >= 1 with
                            (kappa 2^-24)^(k+1) <= 1e-13, kappa from the
                            symbol of constant symmetric bands (1 for the
                            sixth-order schemes, 2 for the tenth-order
                            pentadiagonal one); 2 for other bands */
  int32_t rows_per_lane; /* 0 = automatic; else 4, 6, 8, 12, 16 or 32 (32:
                            uniform lanes with interior elimination only) */
  int32_t host_only;     /* 1: factorise on the host only (no device memory is
                            touched); such a plan can be inspected with
                            cb_plan_get_* but solve calls reject it */
  /* Launch tuning (0 = automatic).  rows_per_lane above sets where the
   * reduction switches from registers (ceil(log2(rows_per_lane - r)) levels
   * of generalized PCR per lane) to LDS (log2(lanes) block-PCR levels). */
  int32_t lines_per_wg;   /* lines per workgroup: 1..1024, power of two, with
                             lines_per_wg * lanes <= 1024 */
  int32_t block_barriers; /* 0: lane exchanges of a line that lies inside one
                             wavefront use wavefront-local ordering only;
                             1: always workgroup barriers */
  int32_t x_staging;      /* unit-stride lines: 0 automatic (2 when one line's
                             tile fits in 64 KB of LDS, else 1), 1 lanes load
                             their rows directly, 2 through a coalesced LDS tile */
  int32_t interior;       /* solve of each lane's interior block D_l: 0 automatic
                             (unit-stride launches: 1 on uniform FP64 lanes,
                             else 2 where available; strided launches: 2 where
                             available), 1 generalized PCR (Sec. 2), 2 banded
                             elimination in registers (rows_per_lane 8/12/16/32) */
  int32_t tile_order;     /* strided launches: order in which workgroups take
                             the tiles of adjacent lines.  0 automatic (2 when
                             a tile's row segments are narrower than 128 bytes
                             or its rows lie at most 64 KB apart, else 1),
                             1 launch order, 2 grouped by XCD: the
                             workgroups one XCD runs take consecutive tiles, so
                             neighbouring segments share that XCD's L2 */
} cb_plan_desc;

/* A strided 3D array of FP64: element (i0,i1,i2) at ptr[i0*stride[0] +
 * i1*stride[1] + i2*stride[2]].  Index 0 is x.  A C-order (nz,ny,nx) array
 * has n = {nx,ny,nz}, stride = {1,nx,nx*ny}.  Strides are in elements and
 * must be positive; lines along `axis` have n[axis] == plan n.  The other two
 * extents may be 0 (an empty grid: the call succeeds, launches nothing and
 * does not read the data pointers, which may then be NULL). */
typedef struct {
  int64_t n[3];
  int64_t stride[3];
} cb_grid;

/* A periodic right-hand-side stencil (Eq. (1)-(2), App. A.2):
 *   b_j = sum_{q = lo}^{hi} coef[q - lo] * f_{(j + q) mod n}
 * with -3 <= lo <= hi <= 3.  Derivative stencils fold 1/h into coef. */
typedef struct {
  int32_t lo;
  int32_t hi;
  double coef[7];
} cb_stencil;

/* Build a plan: the pre-factorisation of Sec. 4 in FP64 on the host,
 * uploaded to the current HIP device.  Returns CB_ERR_SINGULAR when a pivot
 * of a generalized-PCR reduction system or a reduced-system block is
 * (numerically) singular.  *out receives the plan on success. */
cb_status cb_plan(const cb_plan_desc *desc, cb_plan_t *out);

/* Free a plan and its device buffers.  The caller must make sure no work
 * using it is still pending.  NULL is accepted. */
cb_status cb_plan_destroy(cb_plan_t plan);

/* b = stencil(f) along `axis` (0 x, 1 y, 2 z), periodic wrap: the
 * right-hand side of the compact derivative and interpolation (Sec. 1
 * Eqs. (1)-(2); App. A.2 for the staggered forms).  f and b are device
 * arrays laid out by `grid`; they must not overlap.  Errors: bad stencil,
 * grid or axis, NULL or overlapping pointers (CB_ERR_INVALID_ARG). */
cb_status cb_rhs_stencil(const cb_stencil *stencil, const cb_grid *grid, int32_t axis,
                         const double *f, double *b, void *stream);

/* x = A^{-1} b along `axis` for every line of the grid (Sec. 4, Algorithm 1
 * applied to all lines at once).  b == x is allowed (in place); other
 * overlaps are not.  Lines split over P > 1 workgroups (also strided
 * launches of FP64 one-partition plans with n > 4096) need a partition
 * scratch of 3r doubles (4r when refining) per line and partition: the plan
 * keeps one buffer per stream it is used on (calls on one stream are
 * ordered by it, calls on different streams use different buffers),
 * allocated by the first such call on a stream and grown (hipMalloc, after
 * synchronizing that stream) when a call needs more; after 16 streams the
 * device is synchronized and the buffers are released; cb_plan_destroy frees
 * them.  While the stream is being captured into a graph the scratch is a
 * stream-ordered allocation instead (hipMallocAsync / hipFreeAsync). */
cb_status cb_solve(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *b,
                   double *x, void *stream);

/* out = A^{-1} (stencil(f)) along `axis`: the compact derivative or
 * interpolation A f' = B f of Sec. 1 Eqs. (1)-(2) (App. A.2) with the
 * stencil B fused into the solve of Sec. 4 (b never goes to memory).
 * Requires a cyclic plan (the stencil is periodic).  f and out must not
 * overlap.  Same errors as cb_solve, plus CB_ERR_INVALID_ARG for a bad
 * stencil or an acyclic plan. */
cb_status cb_apply_derivative(cb_plan_t plan, const cb_stencil *stencil, const cb_grid *grid,
                              int32_t axis, const double *f, double *out, void *stream);

/* cb_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, checks and results (bitwise) as cb_solve, which may
 * allocate the partition scratch of lines split over P > 1 workgroups (also
 * strided launches of FP64 one-partition plans with n > 4096): 3r doubles
 * per line and partition.  This variant uses instead a
 * fixed array of CB_NOALLOC_SCRATCH_BYTES inside the library, one per GPU,
 * held until the process ends, and never calls hipMalloc, hipFree or any
 * other allocating routine.  A solve that would need more scratch (lines x
 * partitions x 3r x 8 bytes above the limit, e.g. more than 1,398,101
 * tridiagonal line-partitions) returns CB_ERR_UNSUPPORTED before anything is
 * enqueued.  The first call on a device resolves the array's address there
 * (make that call outside graph capture).  Every call on one GPU shares its
 * array, so calls that overlap in time on one GPU (other streams, other
 * threads) race; calls in one stream's order do not. */
#define CB_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
cb_status cb_solve_noalloc(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *b,
                           double *x, void *stream);

/* Diagnostic for the roofline: out = in along `axis`, moved exactly as
 * cb_solve with this plan moves the data (the same workgroup tiles, lane
 * layout, loads, LDS staging, stores and tile order) with the arithmetic
 * left out, so its time is the ceiling of the solve's memory access pattern.
 * One-partition launches only (CB_ERR_UNSUPPORTED for partitioned plans and
 * for strided launches of long lines, which run in partitions).  in and out
 * must not overlap. */
cb_status cb_copy_lines(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *in, double *out,
                        void *stream);

/* One work item of a batched launch: a solve (stencil == NULL) or a fused
 * derivative along one axis of one grid. */
typedef struct {
  cb_plan_t plan;
  const cb_stencil *stencil; /* HOST pointer or NULL */
  cb_grid grid;
  int32_t axis;
  const double *in;          /* device: b (solve) or f (derivative) */
  double *out;               /* device; must not overlap `in` or another item's out */
} cb_batch_item;

/* Batched execution: the lines of many items -- uneven grids, any axes,
 * different plans -- run in ONE kernel launch per kernel class present in the
 * batch, either persistent (a resident grid takes line tiles from a device
 * work queue) or with one workgroup per line tile
 * (a class is r, rows per lane, arithmetic, uniform or general lane layout,
 * interior solve, unit-stride or strided rows and stencil half-width (2 or
 * 3), as an item's plan, row stride and stencil select them; a batch of plans built alike for one scheme and
 * precision is usually a few classes).  Items whose plan splits lines over
 * P > 1 workgroup partitions (Sec. 3-4) run after those as their own phase
 * launches (three per solve and refinement iteration), with their partition
 * scratch in the workspace.  A plan must be cyclic when a stencil is given;
 * n, P, axis, grid, stencil, precision and refinement count may differ
 * between items.  Each line goes through the same arithmetic as in a single
 * cb_solve / cb_apply_derivative call with the same plan.
 *
 * `workspace` is a caller-owned DEVICE buffer of at least
 * cb_batch_workspace_bytes(items, n_items) bytes holding the queue, the work
 * table and the partition scratch of P > 1 items; without such items that
 * is cb_batch_workspace_size(n_items).
 * cb_batch_build validates the items and enqueues the upload of the table on
 * `stream` from a pinned host buffer the library keeps per workspace; it does
 * not wait for the upload (only for the workspace's previous one), so the
 * workspace must not be in use by a launch on another stream.
 * cb_batch_launch enqueues the kernels only: it allocates nothing, copies
 * nothing and leaves the queue reset when it finishes, so it may be captured
 * in a HIP graph and replayed.  Launched on a stream other
 * than the build's, it first makes that stream wait for the upload (while
 * such a stream is being captured, the calling thread waits for it instead).
 * Launches that share a
 * workspace must not overlap in time.  `max_ctas` >= 0 selects the
 * persistent form and caps its resident workgroups (0 = as many as fit on
 * the device at once); a negative value launches one workgroup per tile
 * instead (each item's tiles in the order its single launch would take;
 * measured the faster form). */
size_t cb_batch_workspace_size(int32_t n_items);
size_t cb_batch_workspace_bytes(const cb_batch_item *items, int32_t n_items);
cb_status cb_batch_build(const cb_batch_item *items, int32_t n_items, void *workspace,
                         size_t workspace_bytes, void *stream);
cb_status cb_batch_launch(void *workspace, int32_t max_ctas, void *stream);
/* cb_batch_build followed by cb_batch_launch. */
cb_status cb_solve_batched(const cb_batch_item *items, int32_t n_items, void *workspace,
                           size_t workspace_bytes, int32_t max_ctas, void *stream);

/* Read-only description of a plan's decomposition, for tests and tuning. */
typedef struct {
  int32_t r, n, cyclic, precision, refine_iters;
  int32_t partitions;      /* P workgroup partitions */
  int32_t lanes;           /* L lanes (sub-partitions) per segment */
  int32_t rows_per_lane;   /* M register slots per lane */
  int32_t uniform;         /* 1: every lane partition identical */
  int32_t interior_levels; /* generalized-PCR levels inside a lane partition */
  int32_t lane_levels;     /* block-PCR levels across the lanes */
  int32_t red_phases;      /* phases of the workgroup-level reduced solve */
  int32_t red_pcr_steps;   /* block-PCR steps in it (Sec. 4 step counts) */
  int32_t red_detach_steps;/* detach (= reattach) steps in it */
  int64_t device_bytes;    /* device memory held by the plan */
  int32_t rows_per_lane_strided; /* layout used by strided launches (P = 1); */
  int32_t lanes_strided;         /* equal to the above when one layout serves both */
  int32_t interior_elimination;  /* 1 when lane interiors use banded elimination */
  int32_t interior_elimination_strided; /* the same for strided launches */
  int32_t partitions_strided;    /* workgroup partitions of strided launches
                                    (one-partition plans with n > 4096,
                                    or on a general lane layout with
                                    n > 1024 in FP64, n > 2048 in FP32,
                                    split strided lines into ~512-row
                                    parts; in-place FP32 + refinement
                                    solves keep whole lines) */
  int32_t boundary_window;       /* P > 1: rows at each end of an interior
                                    block that phase A reads (the kept part
                                    of the boundary rows of D_i^{-1}) */
  int32_t fullblock_seg;         /* P > 1: segment index (cb_plan_get_array)
                                    of the full-block lane plan phase C uses
                                    on unit-stride launches, -1 when phase C
                                    solves each interior block D_i itself */
  int32_t fullblock_seg_strided; /* the same for strided launches */
} cb_plan_info;
cb_status cb_plan_get_info(cb_plan_t plan, cb_plan_info *info);

/* Copy the detach schedule of the workgroup-level reduced solve: for each
 * level, the (zero-based) rows detached at that level, -1 terminated per
 * level.  Writes at most `cap` ints to `out`; returns the count in *len. */
cb_status cb_plan_get_schedule(cb_plan_t plan, int32_t *out, int32_t cap, int32_t *len);

/* Copy one host-side array of a plan (FP64 values; integer arrays are
 * converted) for inspection by tests.  `seg` selects the segment: for a
 * one-partition plan 0 is the lane layout of unit-stride launches and 1 (when
 * the layout or interior solve of strided launches differs) that of strided
 * launches; for P > 1 the workgroup partition.  which:
 *   0 lane coefficient blocks [ntypes][block] (layout: k[Tint][N][2r] or,
 *     with elimination, lu[N][2r]; then dinv[N], Lt[r][r], Ut[r][r],
 *     S[N][r], Rm[N][r], N = M - r)
 *   1 lane block-PCR multipliers [Tred][L][2][r][r] (MU then ML)
 *   2 lane final blocks [L][r][r]
 *   3 lane types [L]          4 lane starts [L+1]
 *   5 workgroup S,R blocks (per partition [N_i][r] twice)
 *   6 workgroup L~,U~ [P][2][r][r]   7 partition starts [P+1]
 *   8 reduced-solve program: term ranges [phases][P+1]
 *   9 its source rows per term          10 its matrices per term [r][r]
 *  11 segment shape: S, L, M, r, Tint, Tred, elimination, uniform, cyclic
 *  12 boundary rows of D_i^{-1} [P][2][r][boundary_window]: rows 0..r-1 over
 *     the block's first boundary_window rows, then rows N_i-r..N_i-1 over
 *     its last boundary_window rows
 * Writes min(cap, size) values; *len receives the full size. */
cb_status cb_plan_get_array(cb_plan_t plan, int32_t seg, int32_t which, double *out, int64_t cap,
                            int64_t *len);

/* Message of the last error on the calling thread ("" if none). */
const char *cb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CB_H */
