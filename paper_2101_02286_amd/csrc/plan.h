// Internal plan structures of libcb (host side plus the POD views the kernels
// read).  The factorisation itself is in plan.cpp.
#pragma once
#include <cstdint>
#include <string>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/cb.h"

namespace cb {

// Widest band the library handles: half bandwidth r <= kMaxR (w = 2r+1 <= 7).
constexpr int kMaxR = 3;

// ---------------------------------------------------------------------------
// Lane-level plan of one "segment": a run of S consecutive rows of a line that
// one workgroup solves (the whole line when the line has one partition, else
// the interior block D_i of a workgroup partition).  The segment is split into
// L lane partitions (L a power of two); lane l owns rows [start_l, start_l+m_l)
// held in M register slots.  Its first R rows are the lane's interface rows,
// the remaining N_l = m_l - R rows its interior block (Sec. 3, Eqs. (7)-(8),
// applied with lanes as partitions).
//
// Per lane-type coefficient block (T = double or float), N = M - R slots:
//   k     [Tint][N][2R]  generalized-PCR multipliers (Sec. 2 Eq. (3)); index
//                        R-q for the row q*s above, R+q-1 for q*s below
//   dinv  [N]            1 / diagonal after the last level
//   Lt    [R][R]         interface row a  <- last R interior rows of lane l-1
//   Ut    [R][R]         interface row a  <- first R interior rows of lane l
//   S     [N][R]         D^{-1} L  (Sec. 4 Eq. (15))
//   Rm    [N][R]         D^{-1} U  (Sec. 4 Eq. (16))
// Reduced system across lanes (block PCR, Sec. 4 Algorithm 3):
//   red   [Tred][L][2][R][R]   MU = U^ W_{l+s}^{-1}, ML = L^ W_{l-s}^{-1}
//   wf    [L][R][R]            (W + L^ + U^)^{-1} after the last level
// ---------------------------------------------------------------------------
struct SegPlan {
  int S = 0, cyclic = 0, L = 0, M = 0, R = 0, N = 0, Tint = 0, Tred = 0, ilu = 0;
  int uniform = 0, m_uniform = 0;
  int ntypes = 0, block = 0;
  std::vector<int> lane_type, lane_start;  // L, L+1
  std::vector<double> coef;                // ntypes * block
  std::vector<double> red;                 // Tred * L * 2R^2
  std::vector<double> wf;                  // L * R^2
};

// Interior solve of a lane's block D_l: generalized PCR (k multipliers for
// Tint levels) or, with `ilu`, banded elimination (D_l = L U, unit L):
//   lu  [N][2R]  l_{j,q} = L[j][j-q] (index q-1), u'_{j,q} = U[j][j+q]/U[j][j]
//                (index R+q-1); dinv = 1/U[j][j].
constexpr int interior_size(int R, int M, int Tint, bool ilu) {
  return ilu ? (M - R) * 2 * R : Tint * (M - R) * 2 * R;
}
constexpr int coef_block_size(int R, int M, int Tint, bool ilu = false) {
  return interior_size(R, M, Tint, ilu) + (M - R) + 2 * R * R + 2 * (M - R) * R;
}
struct CoefOff {
  int k, dinv, Lt, Ut, S, Rm;
};
constexpr CoefOff coef_offsets(int R, int M, int Tint, bool ilu = false) {
  return CoefOff{0,
                 interior_size(R, M, Tint, ilu),
                 interior_size(R, M, Tint, ilu) + (M - R),
                 interior_size(R, M, Tint, ilu) + (M - R) + R * R,
                 interior_size(R, M, Tint, ilu) + (M - R) + 2 * R * R,
                 interior_size(R, M, Tint, ilu) + (M - R) + 2 * R * R + (M - R) * R};
}

// ---------------------------------------------------------------------------
// Workgroup-level reduced system (P > 1 partitions per line), solved as a
// program of phases.  In a phase every listed row gets
//     x_new[dst] = sum_terms mat[t] * x_old[src[t]]
// and unlisted rows keep their value.  The program is Algorithm 1's level
// loop (detach, block-PCR step, final solve, reattach; Algorithms 2-4)
// written out for the RHS-dependent updates only.
// ---------------------------------------------------------------------------
struct RedProgram {
  int P = 0, R = 0;
  int nphase = 0;
  std::vector<int> row_off;   // [nphase][P+1] term ranges per (phase, dst)
  std::vector<int> src;       // per term
  std::vector<double> mats;   // per term R*R
  int pcr_steps = 0, detach_steps = 0;
  std::vector<std::vector<int>> detached;  // rows detached at each level
};

// Device view of a segment plan (POD, passed inside kernel arguments).
struct SegDev {
  int S, L, M, Tint, Tred, uniform, m, block, ntypes, ilu;
  const int *lane_type, *lane_start;
  const double *coef64, *red64, *wf64;
  const float *coef32, *red32, *wf32;
};

// Partition scratch a plan keeps for cb_solve (P > 1): one device buffer
// per stream the plan is used on (calls on one stream are ordered by the
// stream, calls on different streams use different buffers), grown on
// demand.  Keys and values are a hipStream_t and device pointers.
struct ScratchCache {
  std::mutex mu;
  std::map<void *, std::pair<void *, size_t>> bufs;
};

struct Plan {
  cb_plan_desc desc{};
  std::vector<double> bands;  // n*(2r+1) (expanded when per_row = 0)
  int R = 1, n = 0, P = 1, M = 8, L = 1;
  int precision = CB_FP64, refine_iters = 0;
  int host_only = 0;
  // segments: P == 1 -> segs[0] is the whole line laid out for unit-stride
  // launches and segs[seg_s] for strided launches (the same when seg_s = 0);
  // P > 1 -> segs[i] = D_i of workgroup partition i
  std::vector<SegPlan> segs;
  int seg_s = 0;
  // workgroup level (P > 1)
  std::vector<int> wg_start;           // P+1
  std::vector<double> SRg;             // per partition: S^G [N_i][R] then R^G [N_i][R]
  std::vector<int64_t> SRg_off;        // P
  std::vector<double> LtUtg;           // [P][2][R][R]
  // Full-block segments (P > 1, equal partitions of L*M rows, constant
  // bands): the whole partition as one acyclic segment whose first R rows
  // are identity equations (x = x~_i, known after phase B) and whose
  // couplings to the next partition move to the right-hand side.  Every lane
  // then holds M rows, and the lanes' coefficient blocks are one block
  // (fb_type) apart from lane 0's interface couplings and the last lane's
  // forward coupling, which are zero: phase C runs the uniform lane code
  // with those two terms masked.  Indices into segs, -1 when absent.
  int fb_seg_u = -1, fb_seg_s = -1, fb_type_u = 0, fb_type_s = 0;
  // rows 0..R-1 and N_i-R..N_i-1 of D_i^{-1} over windows of Kw rows at the
  // ends of D_i (entries beyond the window are below 2^-56 of the row's
  // absolute sum): [P][2][R][Kw], first-end window rows 0..Kw-1, last-end
  // window rows N_i-Kw..N_i-1
  int Kw = 0;
  std::vector<double> bfun;
  RedProgram prog;
  // device buffers
  void *dev_base = nullptr;
  int64_t dev_bytes = 0;
  std::vector<SegDev> segdev_host;     // P (or 1) views with device pointers
  SegDev *segdev = nullptr;            // device copy of segdev_host
  const int *d_wg_start = nullptr;
  const double *d_SRg = nullptr;
  const int64_t *d_SRg_off = nullptr;
  const double *d_LtUtg = nullptr;
  const int *d_row_off = nullptr, *d_src = nullptr;
  const double *d_mats = nullptr;
  const double *d_bfun = nullptr;
  const double *d_bands = nullptr;     // n*(2r+1) per-row bands
  // long lines (n > 4096) of a one-partition plan, and ragged ones on
  // general lane layouts (FP64 n > 1024, FP32 n > 2048): strided launches run the same
  // matrix split into workgroup partitions of about 512 rows, since a whole
  // line per workgroup would leave room for only a few adjacent lines
  std::shared_ptr<Plan> strided_wg;
  std::shared_ptr<ScratchCache> sc = std::make_shared<ScratchCache>();
};

// Builds the host-side factorisation.  Returns CB_OK or an error with msg.
cb_status build_plan(const cb_plan_desc &d, Plan &p, std::string &msg);

}  // namespace cb
