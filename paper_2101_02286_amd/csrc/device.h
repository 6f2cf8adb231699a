// Device-side building blocks of the line solver (gfx950).
//
// Mapping of the paper's two-level factorisation onto a workgroup:
//   * a line (or a workgroup partition's interior block) is a "segment" of S
//     rows split over L lanes; lane l owns m_l <= M consecutive rows in
//     registers.  Lanes play the role of the paper's partitions: the first R
//     rows of a lane are its interface rows, the rest its interior block D_l
//     (Sec. 3, Eqs. (7)-(8)).
//   * D_l y_l = b_l is solved in registers by generalized PCR with the
//     plan's stored multipliers (Sec. 2 Eq. (3); Sec. 4 Eq. (17)).
//   * The interface right-hand side b^_l (Eq. (21)) needs only the last R
//     rows of y_{l-1} (the sparsity of L~), exchanged through LDS.
//   * The reduced cyclic block system across the L lanes is solved by block
//     PCR (Algorithm 3), each level exchanging R values with lanes l+-s.
//   * Back-substitution x_l = y_l - S_l x~_l - R_l x~_{l+1} (Eq. (22)).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.h"
#include "plan.h"

namespace cb {

typedef double dbl2 __attribute__((ext_vector_type(2)));

// Plan coefficients are read-only for the whole launch.  Reading them through
// the constant address space lets uniform reads become scalar (s_load) reads
// that land in SGPRs instead of occupying vector registers.
template <typename T>
__device__ __forceinline__ T cld(const T *p) {
  return *reinterpret_cast<const __attribute__((address_space(4))) T *>(reinterpret_cast<uintptr_t>(p));
}

constexpr int ceil_log2_c(int v) { return v <= 1 ? 0 : 1 + ceil_log2_c((v + 1) / 2); }

template <typename T> __device__ __forceinline__ const T *coef_of(const SegDev &s);
template <> __device__ __forceinline__ const double *coef_of<double>(const SegDev &s) { return s.coef64; }
template <> __device__ __forceinline__ const float *coef_of<float>(const SegDev &s) { return s.coef32; }
template <typename T> __device__ __forceinline__ const T *red_of(const SegDev &s);
template <> __device__ __forceinline__ const double *red_of<double>(const SegDev &s) { return s.red64; }
template <> __device__ __forceinline__ const float *red_of<float>(const SegDev &s) { return s.red32; }
template <typename T> __device__ __forceinline__ const T *wf_of(const SegDev &s);
template <> __device__ __forceinline__ const double *wf_of<double>(const SegDev &s) { return s.wf64; }
template <> __device__ __forceinline__ const float *wf_of<float>(const SegDev &s) { return s.wf32; }

// LDS exchange between the lanes of one line.  Each thread owns two regions
// of RS doubles; exchange number k writes region k&1, waits at a barrier, and
// reads partners' region k&1.  Exchange k+2 reuses the region only after the
// barrier of exchange k+1, which every thread reaches after its reads of
// exchange k, so one barrier per exchange suffices.  Value i of thread t in
// region r lives at base[(r * RS + i) * NT + t]: consecutive threads touch
// consecutive words, so writes and (shifted) partner reads are free of bank
// conflicts.
struct Xchg {
  double *base;  // LDS, NT * 2 * RS doubles
  int RS;        // doubles per region
  int NT;
  int k;         // exchange counter
  bool block_sync;
  __device__ __forceinline__ void sync() {
    if (block_sync) {
      __syncthreads();
    } else {
      // all lanes of every line are in this wave: LDS traffic of a wave is
      // processed in order, only the compiler must not reorder it
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // value i of thread tid in the current region is slot(tid)[i * NT]
  __device__ __forceinline__ double *slot(int tid) { return base + (size_t)(k & 1) * RS * NT + tid; }
  template <int CNT, typename V>
  __device__ __forceinline__ void publish(int tid, const V (&vals)[CNT]) {
    double *p = slot(tid);
#pragma unroll
    for (int i = 0; i < CNT; ++i) p[(size_t)i * NT] = (double)vals[i];
    sync();
  }
  template <int CNT, typename V>
  __device__ __forceinline__ void fetch(int tid_src, V (&out)[CNT]) {
    const double *p = slot(tid_src);
#pragma unroll
    for (int i = 0; i < CNT; ++i) out[i] = (V)p[(size_t)i * NT];
  }
  __device__ __forceinline__ void done() { ++k; }
};

// Position of this thread: lane l of line li inside a tile of W lines.
struct LanePos {
  int tid, l, li, L, W, lgL, lgW, mode;
  __device__ __forceinline__ int tid_of(int lane) const {
    return mode == MODE_X ? (li << lgL) + lane : (lane << lgW) + li;
  }
};

template <typename T, int N>
__device__ __forceinline__ T select_idx(const T (&y)[N], int idx) {
  T r = (T)0;
#pragma unroll
  for (int j = 0; j < N; ++j) r = (j == idx) ? y[j] : r;
  return r;
}

// Rows of lane l in a segment of S rows over L = 2^lgL lanes: the first
// S mod L lanes hold one row more (the layout the plan builds), so a lane's
// first row and row count follow without a table lookup.
__device__ __forceinline__ void lane_rows(int S, int lgL, int l, int &start, int &m) {
  const int base = S >> lgL, extra = S & ((1 << lgL) - 1);
  start = l * base + (l < extra ? l : extra);
  m = base + (l < extra ? 1 : 0);
}

// Where a lane's coefficient block is read from: the plan in global memory
// through the constant address space (uniform plans: scalar loads), or a
// copy staged in LDS (general plans, whose lanes read different blocks).
enum { CSRC_GLOBAL = 0, CSRC_LDS = 1 };
template <int CSRC, typename T>
__device__ __forceinline__ T cget(const T *p) {
  if (CSRC == CSRC_LDS) return *p;
  return cld(p);
}

// Copy the plan's lane-type coefficient blocks into LDS (all threads take
// part; ends with a workgroup barrier).
template <typename T>
__device__ __forceinline__ void stage_coef(const SegDev &sg, T *dst, int tid, int nt) {
  const T *src = coef_of<T>(sg);
  const int cnt = sg.ntypes * sg.block;
  for (int i = tid; i < cnt; i += nt) dst[i] = src[i];
  __syncthreads();
}

// One lane's block-PCR multipliers for the first TP levels of the reduced
// system and its final solve, loaded ahead of the data they act on.  Lanes
// whose multipliers differ (the full-block form) read them with vector loads;
// inside the level loop each would wait for a memory round trip after the
// exchange.  Levels >= TP (and plans with fewer levels) are not affected.
template <typename T, int R, int TP>
struct RedPre {
  T mu[TP > 0 ? TP : 1][R * R], ml[TP > 0 ? TP : 1][R * R], w[R * R];
};
template <typename T, int R, int TP>
__device__ __forceinline__ void red_prefetch(const SegDev &sg, int lr, RedPre<T, R, TP> &pre) {
  constexpr int RR = R * R;
  const T *rd = red_of<T>(sg);
#pragma unroll
  for (int t = 0; t < TP; ++t) {
    const int tt = t < sg.Tred ? t : 0;  // levels the plan lacks are never used: stay in bounds
    const T *mu = rd + ((size_t)(tt * sg.L + lr) * 2) * RR;
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      pre.mu[t][i] = cld(mu + i);
      pre.ml[t][i] = cld(mu + RR + i);
    }
  }
  const T *w = wf_of<T>(sg) + (size_t)lr * RR;
#pragma unroll
  for (int i = 0; i < RR; ++i) pre.w[i] = cld(w + i);
}

// Solve the segment in place: on entry v[0..m) holds b of the lane's rows, on
// exit x.  Padding slots (k >= m) hold zero and stay zero.  `cl` is the LDS
// copy of the coefficient blocks when CSRC == CSRC_LDS.
// UACYC (with UNI: every lane holds M rows): an acyclic segment whose lanes
// all read the coefficient block `type`, except that lane 0's interface rows
// are identity equations (x~ = b, its couplings to other lanes zero) and the
// last lane has no forward coupling; the reduced-system multipliers are read
// per lane.  Used for whole workgroup partitions (the full-block plans).
// `pre`: the lane's multipliers for the first TP levels, from red_prefetch.
template <int R, int M, typename T, bool UNI, int CSRC = CSRC_GLOBAL, bool ILU = false, bool UACYC = false,
          int TP = 0>
__device__ __forceinline__ void solve_segment(T (&v)[M], const SegDev &sg, const LanePos &p, int type,
                                              int m, Xchg &xc, const T *cl = nullptr,
                                              const RedPre<T, R, TP> *pre = nullptr) {
  constexpr int N = M - R;
  constexpr int TI = ceil_log2_c(N);
  constexpr int RR = R * R;
  constexpr CoefOff off = coef_offsets(R, M, TI, ILU);
  const T *cf = (CSRC == CSRC_LDS ? cl : coef_of<T>(sg)) + (size_t)((UNI && !UACYC) ? 0 : type) * sg.block;

  T y[N];
#pragma unroll
  for (int j = 0; j < N; ++j) y[j] = v[R + j];
  if (ILU) {
    // ---- interior by banded elimination in place, D_l = L U ----
#pragma unroll
    for (int j = 1; j < N; ++j)
#pragma unroll
      for (int q = 1; q <= R; ++q)
        if (j - q >= 0) y[j] -= cget<CSRC>(cf + off.k + j * 2 * R + q - 1) * y[j - q];
#pragma unroll
    for (int j = N - 1; j >= 0; --j) {
      T acc = y[j] * cget<CSRC>(cf + off.dinv + j);
#pragma unroll
      for (int q = 1; q <= R; ++q)
        if (j + q < N) acc -= cget<CSRC>(cf + off.k + j * 2 * R + R + q - 1) * y[j + q];
      y[j] = acc;
    }
  }
  // ---- interior generalized PCR, D_l y = b (Eq. (3) with stored k) ----
#pragma unroll
  for (int t = 0; t < (ILU ? 0 : TI); ++t) {
    const int s = 1 << t;
    T yn[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T acc = y[j];
      const T *kj = cf + off.k + (t * N + j) * 2 * R;
#pragma unroll
      for (int q = 1; q <= R; ++q) {
        if (j - q * s >= 0) acc -= cget<CSRC>(kj + R - q) * y[j - q * s];
        if (j + q * s < N) acc -= cget<CSRC>(kj + R + q - 1) * y[j + q * s];
      }
      yn[j] = acc;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) y[j] = yn[j];
  }
  if (!ILU) {
#pragma unroll
    for (int j = 0; j < N; ++j) y[j] *= cget<CSRC>(cf + off.dinv + j);
  }

  // ---- interface RHS b^_l = b~_l - L~_l y_{l-1} - U~_l y_l (Eq. (21)) ----
  const int nl = m - R;  // real interior rows of this lane
  T ylast[R];
#pragma unroll
  for (int a = 0; a < R; ++a) ylast[a] = UNI ? y[N - R + a] : select_idx(y, nl - R + a);
  xc.publish(p.tid, ylast);
  T yprev[R];
  xc.fetch(p.tid_of((p.l - 1) & (p.L - 1)), yprev);
  xc.done();
  T xt[R];
#pragma unroll
  for (int a = 0; a < R; ++a) {
    T acc = v[a];
#pragma unroll
    for (int c = 0; c < R; ++c) acc -= cget<CSRC>(cf + off.Lt + a * R + c) * yprev[c] + cget<CSRC>(cf + off.Ut + a * R + c) * y[c];
    xt[a] = (UACYC && p.l == 0) ? v[a] : acc;  // identity rows: x~ = b
  }

  // ---- reduced cyclic block system across lanes: block PCR (Alg. 3) ----
  const T *rd = red_of<T>(sg);
  const int lr = (UNI && !UACYC) ? 0 : p.l;
  // one level: x~_l -= MU x~_{l+s} + ML x~_{l-s}, multipliers from mu(i), ml(i)
  auto level = [&](int t, auto mu, auto ml) {
    const int s = 1 << t;
    xc.publish(p.tid, xt);
    T xp[R], xm[R];
    xc.fetch(p.tid_of((p.l + s) & (p.L - 1)), xp);
    xc.fetch(p.tid_of((p.l - s) & (p.L - 1)), xm);
    xc.done();
    T xn[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      T acc = xt[a];
#pragma unroll
      for (int c = 0; c < R; ++c) acc -= mu(a * R + c) * xp[c] + ml(a * R + c) * xm[c];
      xn[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < R; ++a) xt[a] = xn[a];
  };
#pragma unroll
  for (int t = 0; t < TP; ++t)
    if (t < sg.Tred) level(t, [&](int i) { return pre->mu[t][i]; }, [&](int i) { return pre->ml[t][i]; });
  for (int t = TP; t < sg.Tred; ++t) {
    const T *mu = rd + ((size_t)(t * sg.L + lr) * 2) * RR;
    const T *ml = mu + RR;
    level(t, [&](int i) { return cld(mu + i); }, [&](int i) { return cld(ml + i); });
  }
  {
    const T *w = wf_of<T>(sg) + (size_t)lr * RR;
    T xn[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      T acc = (T)0;
#pragma unroll
      for (int c = 0; c < R; ++c) acc += (TP > 0 ? pre->w[a * R + c] : cld(w + a * R + c)) * xt[c];
      xn[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < R; ++a) xt[a] = xn[a];
  }

  // ---- back-substitution x_l = y_l - S_l x~_l - R_l x~_{l+1} (Eq. (22)) ----
  xc.publish(p.tid, xt);
  T xnext[R];
  xc.fetch(p.tid_of((p.l + 1) & (p.L - 1)), xnext);
  xc.done();
  if (UACYC && p.l == p.L - 1) {  // the acyclic segment ends: no forward coupling
#pragma unroll
    for (int c = 0; c < R; ++c) xnext[c] = (T)0;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T acc = y[j];
#pragma unroll
    for (int c = 0; c < R; ++c)
      acc -= cget<CSRC>(cf + off.S + j * R + c) * xt[c] + cget<CSRC>(cf + off.Rm + j * R + c) * xnext[c];
    v[R + j] = acc;
  }
#pragma unroll
  for (int a = 0; a < R; ++a) v[a] = xt[a];
}

// Halo exchange of the Q rows on each side of the lane (periodic through the
// lanes of a cyclic segment): prev[i] = row start-Q+i, next[i] = row start+m+i.
// One exchange: each lane publishes its first Q and last Q rows.
template <int Q, int M, typename V>
__device__ __forceinline__ void halo(const V (&v)[M], int m, bool full, const LanePos &p, Xchg &xc,
                                     V (&prev)[Q], V (&next)[Q]) {
  V out[2 * Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    out[i] = v[i];
    if (full) {
      out[Q + i] = v[M - Q + i];
    } else {
      V r = (V)0;
#pragma unroll
      for (int j = 0; j < M; ++j) r = (j == m - Q + i) ? v[j] : r;
      out[Q + i] = r;
    }
  }
  xc.publish(p.tid, out);
  const double *pp = xc.slot(p.tid_of((p.l - 1) & (p.L - 1)));
  const double *pn = xc.slot(p.tid_of((p.l + 1) & (p.L - 1)));
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    prev[i] = (V)pp[(size_t)(Q + i) * xc.NT];
    next[i] = (V)pn[(size_t)i * xc.NT];
  }
  xc.done();
}

// Unsigned 32-bit division by a runtime-invariant divisor d with a
// host-precomputed multiplier (round-up method): q = (t + ((n - t) >> s1)) >> s2,
// t = mulhi(mul, n).
struct FastDiv {
  uint32_t d, mul, s1, s2;
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    const uint32_t t = __umulhi(mul, n);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

// Value of row (k + q) relative to the lane start, from registers or halos.
template <int Q, int M, typename V>
__device__ __forceinline__ V row_at(const V (&v)[M], const V (&prev)[Q], const V (&next)[Q], int idx,
                                    int m, bool full) {
  if (idx < 0) return prev[Q + idx];
  if (full) return idx < M ? v[idx] : next[idx - M];
  if (idx >= M) return select_idx(next, idx - m);
  return idx < m ? v[idx] : select_idx(next, idx - m);
}

}  // namespace cb
