// Host-side pre-factorisation of a compact banded matrix (FP64).
//
// Everything here is independent of the right-hand side and is computed once
// per matrix (Sec. 4, the paragraph on pre-factorisation): the generalized
// PCR multipliers of every interior block (Sec. 2 Eqs. (3)-(6)), the blocks
// S = D^{-1} L and R = D^{-1} U (Sec. 4 Eqs. (15)-(16)), the reduced blocks
// of Eqs. (18)-(20), and the multipliers of the block-PCR solve of the
// reduced system (Sec. 4 Algorithms 1-4).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

namespace cb {
namespace {

// ------------------------------------------------------------ small dense --
using Mat = std::vector<double>;  // R x R, row-major

Mat zeros(int R) { return Mat(R * R, 0.0); }
Mat eye(int R) {
  Mat m = zeros(R);
  for (int i = 0; i < R; ++i) m[i * R + i] = 1.0;
  return m;
}
Mat mul(const Mat &a, const Mat &b, int R) {
  Mat c = zeros(R);
  for (int i = 0; i < R; ++i)
    for (int k = 0; k < R; ++k)
      for (int j = 0; j < R; ++j) c[i * R + j] += a[i * R + k] * b[k * R + j];
  return c;
}
Mat add(const Mat &a, const Mat &b) {
  Mat c(a);
  for (size_t i = 0; i < c.size(); ++i) c[i] += b[i];
  return c;
}
Mat sub(const Mat &a, const Mat &b) {
  Mat c(a);
  for (size_t i = 0; i < c.size(); ++i) c[i] -= b[i];
  return c;
}
Mat neg(const Mat &a) {
  Mat c(a);
  for (auto &v : c) v = -v;
  return c;
}

// Gauss-Jordan inverse with partial pivoting; false when numerically singular
// (pivot below 1e-12 of the largest entry).
bool inverse(const Mat &a, int R, Mat &out) {
  Mat m(a);
  out = eye(R);
  double amax = 0.0;
  for (double v : m) amax = std::max(amax, std::fabs(v));
  if (!(amax > 0.0) || !std::isfinite(amax)) return false;
  for (int k = 0; k < R; ++k) {
    int p = k;
    for (int i = k + 1; i < R; ++i)
      if (std::fabs(m[i * R + k]) > std::fabs(m[p * R + k])) p = i;
    if (!(std::fabs(m[p * R + k]) > 1e-12 * amax)) return false;
    if (p != k)
      for (int j = 0; j < R; ++j) {
        std::swap(m[k * R + j], m[p * R + j]);
        std::swap(out[k * R + j], out[p * R + j]);
      }
    const double d = 1.0 / m[k * R + k];
    for (int j = 0; j < R; ++j) {
      m[k * R + j] *= d;
      out[k * R + j] *= d;
    }
    for (int i = 0; i < R; ++i) {
      if (i == k) continue;
      const double f = m[i * R + k];
      if (f == 0.0) continue;
      for (int j = 0; j < R; ++j) {
        m[i * R + j] -= f * m[k * R + j];
        out[i * R + j] -= f * out[k * R + j];
      }
    }
  }
  return true;
}

// Small dense solve (size <= 2 * kMaxR), partial pivoting.
bool small_solve(int m, double *a, double *x, double scale) {
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (std::fabs(a[i * m + k]) > std::fabs(a[p * m + k])) p = i;
    if (!(std::fabs(a[p * m + k]) > 1e-13 * scale)) return false;
    if (p != k) {
      for (int j = 0; j < m; ++j) std::swap(a[k * m + j], a[p * m + j]);
      std::swap(x[k], x[p]);
    }
    for (int i = k + 1; i < m; ++i) {
      const double l = a[i * m + k] / a[k * m + k];
      for (int j = k; j < m; ++j) a[i * m + j] -= l * a[k * m + j];
      x[i] -= l * x[k];
    }
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < m; ++j) s -= a[i * m + j] * x[j];
    x[i] = s / a[i * m + i];
  }
  return true;
}

int ceil_log2(int v) {
  int t = 0;
  while ((1 << t) < v) ++t;
  return t;
}
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// ------------------------------------------------- generalized PCR (Sec. 2) --
// An acyclic banded block D of N rows: band[j*(2R+1) + o+R] = D[j][j+o].
struct GPCR {
  int N = 0, R = 0, T = 0;
  std::vector<double> k;     // [T][N][2R]
  std::vector<double> dinv;  // [N]
};

inline int kidx(int q, int R) { return q < 0 ? R + q : R + q - 1; }

// Factor D by generalized PCR (Eq. (3)): at level t (stride s = 2^t) row j
// becomes a_j - sum_q k_q a_{j+qs}, with the k_q chosen so the entries at odd
// multiples of s vanish (Eq. (4); tridiagonal Eq. (5), pentadiagonal Eq. (6)).
// Near the ends of D the neighbour rows j+qs outside D are absent and so are
// the equations of columns outside D; when a side has more rows than
// equations the outermost rows of that side get k = 0 (the equation they
// would serve is vacuous).  `T` levels are stored (>= ceil(log2 N); extra
// levels have k = 0).
cb_status gpcr_factor(int N, int R, const std::vector<double> &band, int T, GPCR &g,
                      std::string &msg) {
  const int W = 2 * R + 1;
  g.N = N;
  g.R = R;
  g.T = T;
  g.k.assign((size_t)T * N * 2 * R, 0.0);
  g.dinv.assign(N, 0.0);
  std::vector<double> c(band), cn(band.size());
  double scale = 0.0;
  for (double v : band) scale = std::max(scale, std::fabs(v));
  // D_cur[j][j + o*s] = c[j*W + o+R]
  auto at = [&](int row, int o) -> double {  // entry of row at offset o*s
    if (o < -R || o > R) return 0.0;
    return c[row * W + o + R];
  };
  for (int t = 0; t < T; ++t) {
    const int s = 1 << t;
    for (int j = 0; j < N; ++j) {
      const int Qm = std::min(2 * R, j / s);            // rows above at stride s
      const int Qp = std::min(2 * R, (N - 1 - j) / s);  // rows below
      const int Em = (std::min(2 * R - 1, Qm) + 1) / 2;  // equations/unknowns above
      const int Ep = (std::min(2 * R - 1, Qp) + 1) / 2;
      int qs[2 * kMaxR], os[2 * kMaxR];
      int m = 0;
      for (int q = Em; q >= 1; --q) qs[m++] = -q;
      for (int q = 1; q <= Ep; ++q) qs[m++] = q;
      int e = 0;
      for (int q = Em; q >= 1; --q) os[e++] = -(2 * q - 1);
      for (int q = 1; q <= Ep; ++q) os[e++] = 2 * q - 1;
      // Deep levels couple rows 2s apart; in a banded inverse those
      // couplings decay geometrically, so an outer equation (column j+-3s)
      // can vanish entirely.  Such an equation is vacuous: the outer row it
      // pairs with (q = +-2) is then not needed and gets k = 0, exactly as at
      // the ends of D.  Remaining equations are scaled to unit row maximum.
      bool vac[2 * kMaxR] = {}, drop[2 * kMaxR] = {};
      for (int r = 0; r < m; ++r) {
        double rmax = 0.0;
        for (int u = 0; u < m; ++u) rmax = std::max(rmax, std::fabs(at(j + qs[u] * s, os[r] - qs[u])));
        vac[r] = !(rmax > 1e-300) && at(j, os[r]) == 0.0 && std::abs(os[r]) > 1;
        if (vac[r]) {
          const int qd = os[r] < 0 ? -(1 - os[r]) / 2 : (os[r] + 1) / 2;
          for (int u = 0; u < m; ++u)
            if (qs[u] == qd) drop[u] = true;
        }
      }
      int qk[2 * kMaxR], ok[2 * kMaxR], mk = 0, ne = 0;
      for (int r = 0; r < m; ++r)
        if (!vac[r]) ok[ne++] = os[r];
      for (int u = 0; u < m; ++u)
        if (!drop[u]) qk[mk++] = qs[u];
      if (ne != mk) {
        msg = "generalized PCR reduction system is singular";
        return CB_ERR_SINGULAR;
      }
      double a[4 * kMaxR * kMaxR], x[2 * kMaxR];
      for (int r = 0; r < mk; ++r) {
        double rmax = 0.0;
        for (int u = 0; u < mk; ++u) {
          a[r * mk + u] = at(j + qk[u] * s, ok[r] - qk[u]);
          rmax = std::max(rmax, std::fabs(a[r * mk + u]));
        }
        x[r] = at(j, ok[r]);
        if (rmax > 0.0) {
          for (int u = 0; u < mk; ++u) a[r * mk + u] /= rmax;
          x[r] /= rmax;
        }
      }
      if (mk > 0 && !small_solve(mk, a, x, 1.0)) {
        msg = "generalized PCR reduction system is singular";
        return CB_ERR_SINGULAR;
      }
      for (int u = 0; u < mk; ++u) g.k[((size_t)t * N + j) * 2 * R + kidx(qk[u], R)] = x[u];
      // the new row keeps the even multiples of s: offsets 2*o2*s, o2 in [-R, R]
      for (int o2 = -R; o2 <= R; ++o2) {
        double v = at(j, 2 * o2);
        for (int u = 0; u < mk; ++u) v -= x[u] * at(j + qk[u] * s, 2 * o2 - qk[u]);
        // offsets that leave D are structurally zero
        const int col = j + 2 * o2 * s;
        cn[j * W + o2 + R] = (col >= 0 && col < N) ? v : 0.0;
      }
    }
    std::swap(c, cn);
  }
  for (int j = 0; j < N; ++j) {
    for (int o = -R; o <= R; ++o)
      if (o != 0 && c[j * W + o + R] != 0.0) {
        msg = "internal: generalized PCR did not reach a diagonal system";
        return CB_ERR_INVALID_ARG;
      }
    const double d = c[j * W + R];
    if (!(std::fabs(d) > 1e-13 * scale)) {
      msg = "generalized PCR produced a zero pivot (singular block)";
      return CB_ERR_SINGULAR;
    }
    g.dinv[j] = 1.0 / d;
  }
  return CB_OK;
}

// y = D^{-1} rhs for one column (length N), by the stored levels.
void gpcr_apply(const GPCR &g, double *y) {
  const int N = g.N, R = g.R;
  std::vector<double> yn(N);
  for (int t = 0; t < g.T; ++t) {
    const int s = 1 << t;
    for (int j = 0; j < N; ++j) {
      double v = y[j];
      for (int q = 1; q <= R; ++q) {
        if (j - q * s >= 0) v -= g.k[((size_t)t * N + j) * 2 * R + kidx(-q, R)] * y[j - q * s];
        if (j + q * s < N) v -= g.k[((size_t)t * N + j) * 2 * R + kidx(q, R)] * y[j + q * s];
      }
      yn[j] = v;
    }
    std::copy(yn.begin(), yn.end(), y);
  }
  for (int j = 0; j < N; ++j) y[j] *= g.dinv[j];
}

// Banded LU without pivoting of one lane's interior block (unit lower L):
// out[j*2R + q-1] = L[j][j-q], out[j*2R + R+q-1] = U[j][j+q] / U[j][j],
// dinv[j] = 1 / U[j][j].
cb_status lane_lu(int N, int R, const std::vector<double> &band, double *out, double *dinv, std::string &msg) {
  const int W = 2 * R + 1;
  std::vector<double> a(band);
  double scale = 0.0;
  for (double v : band) scale = std::max(scale, std::fabs(v));
  for (int k = 0; k < N; ++k) {
    const double piv = a[k * W + R];
    if (!(std::fabs(piv) > 1e-13 * scale)) {
      msg = "interior elimination met a zero pivot";
      return CB_ERR_SINGULAR;
    }
    for (int i = k + 1; i <= std::min(N - 1, k + R); ++i) {
      const double l = a[i * W + (k - i + R)] / piv;
      a[i * W + (k - i + R)] = l;
      for (int j = k + 1; j <= std::min(N - 1, k + R); ++j) a[i * W + (j - i + R)] -= l * a[k * W + (j - k + R)];
    }
  }
  for (int j = 0; j < N; ++j) {
    dinv[j] = 1.0 / a[j * W + R];
    for (int q = 1; q <= R; ++q) {
      out[j * 2 * R + q - 1] = j - q >= 0 ? a[j * W + (R - q)] : 0.0;
      out[j * 2 * R + R + q - 1] = j + q < N ? a[j * W + (R + q)] * dinv[j] : 0.0;
    }
  }
  return CB_OK;
}

// x = D^{-1} x for one column, from the factors lane_lu returns.
void lu_apply(int N, int R, const double *lu, const double *dinv, double *x) {
  for (int j = 1; j < N; ++j)
    for (int q = 1; q <= R; ++q)
      if (j - q >= 0) x[j] -= lu[(size_t)j * 2 * R + q - 1] * x[j - q];
  for (int j = N - 1; j >= 0; --j) {
    double acc = x[j] * dinv[j];
    for (int q = 1; q <= R; ++q)
      if (j + q < N) acc -= lu[(size_t)j * 2 * R + R + q - 1] * x[j + q];
    x[j] = acc;
  }
}

// ------------------------------------------------ partitioned blocks (Sec. 3) --
// A run of S rows split into P parts; part i has rows [st[i], st[i+1]), its
// first R rows are interface rows and the rest the interior block D_i.
// coef(g, o) returns A[row g][row g + o] of the run.  When `cyclic`, part
// indices wrap modulo P; otherwise couplings leaving the run are dropped.
struct Blocks {
  int P, R;
  std::vector<int> st;
  std::vector<GPCR> D;
  std::vector<std::vector<double>> Sm, Rm;  // per part: [N_i][R]
  std::vector<Mat> Dt, Lt, Ut;               // per part R x R
  std::vector<Mat> Lh, Dh, Uh;               // reduced blocks, Eqs. (18)-(20)
};

cb_status build_blocks(int P, int R, const std::vector<int> &st, bool cyclic,
                       const std::function<double(int, int)> &coef, int Tfix, Blocks &B,
                       std::string &msg) {
  const int W = 2 * R + 1;
  B.P = P;
  B.R = R;
  B.st = st;
  B.D.resize(P);
  B.Sm.resize(P);
  B.Rm.resize(P);
  B.Dt.assign(P, zeros(R));
  B.Lt.assign(P, zeros(R));
  B.Ut.assign(P, zeros(R));
  for (int i = 0; i < P; ++i) {
    const int s0 = st[i], m = st[i + 1] - st[i], N = m - R;
    if (N < R) {
      msg = "a partition has fewer than 2r rows";
      return CB_ERR_INVALID_ARG;
    }
    std::vector<double> band((size_t)N * W, 0.0), Lc((size_t)N * R, 0.0), Uc((size_t)N * R, 0.0);
    for (int j = 0; j < N; ++j)
      for (int o = -R; o <= R; ++o) {
        const int t = j + o;
        const double v = coef(s0 + R + j, o);
        if (t < 0) {
          Lc[j * R + (R + t)] = v;  // interface row R+t of this part
        } else if (t < N) {
          band[j * W + o + R] = v;
        } else {  // interface row t-N of the next part
          if (!cyclic && i == P - 1) continue;
          Uc[j * R + (t - N)] = v;
        }
      }
    for (int a = 0; a < R; ++a)
      for (int o = -R; o <= R; ++o) {
        const int t = a + o;
        const double v = coef(s0 + a, o);
        if (t < 0) {
          if (!cyclic && i == 0) continue;
          B.Lt[i][a * R + (R + t)] = v;  // last R interior rows of part i-1
        } else if (t < R) {
          B.Dt[i][a * R + t] = v;
        } else {
          B.Ut[i][a * R + (t - R)] = v;  // first R interior rows of part i
        }
      }
    // Lane partitions (Tfix >= 0) keep the generalized-PCR multipliers of D_i
    // (Eq. (3)), which the kernels use.  Workgroup partitions need only
    // S_i and R_i from D_i, which banded elimination gives as well (deep
    // generalized-PCR levels of a slowly decaying inverse can meet
    // near-singular reduction systems).
    std::vector<double> lu, dv;
    if (Tfix >= 0) {
      cb_status stt = gpcr_factor(N, R, band, Tfix, B.D[i], msg);
      if (stt != CB_OK) return stt;
    } else {
      lu.resize((size_t)N * 2 * R);
      dv.resize(N);
      cb_status stt = lane_lu(N, R, band, lu.data(), dv.data(), msg);
      if (stt != CB_OK) return stt;
    }
    auto apply = [&](double *col) {
      if (Tfix >= 0) gpcr_apply(B.D[i], col);
      else lu_apply(N, R, lu.data(), dv.data(), col);
    };
    // S_i = D_i^{-1} L_i, R_i = D_i^{-1} U_i (Eqs. (15)-(16)), column by column
    B.Sm[i].assign((size_t)N * R, 0.0);
    B.Rm[i].assign((size_t)N * R, 0.0);
    std::vector<double> col(N);
    for (int c = 0; c < R; ++c) {
      for (int j = 0; j < N; ++j) col[j] = Lc[j * R + c];
      apply(col.data());
      for (int j = 0; j < N; ++j) B.Sm[i][j * R + c] = col[j];
      for (int j = 0; j < N; ++j) col[j] = Uc[j * R + c];
      apply(col.data());
      for (int j = 0; j < N; ++j) B.Rm[i][j * R + c] = col[j];
    }
  }
  // Eqs. (18)-(20): only the last R rows of S_{i-1}, R_{i-1} and the first R
  // rows of S_i, R_i enter (the sparsity of L~ and U~).
  B.Lh.assign(P, zeros(R));
  B.Dh.assign(P, zeros(R));
  B.Uh.assign(P, zeros(R));
  for (int i = 0; i < P; ++i) {
    const int ip = (i + P - 1) % P;
    const int Np = st[ip + 1] - st[ip] - R;
    Mat Sl = zeros(R), Rl = zeros(R), Sf = zeros(R), Rf = zeros(R);
    for (int a = 0; a < R; ++a)
      for (int c = 0; c < R; ++c) {
        Sl[a * R + c] = B.Sm[ip][(Np - R + a) * R + c];
        Rl[a * R + c] = B.Rm[ip][(Np - R + a) * R + c];
        Sf[a * R + c] = B.Sm[i][a * R + c];
        Rf[a * R + c] = B.Rm[i][a * R + c];
      }
    B.Lh[i] = neg(mul(B.Lt[i], Sl, R));
    B.Dh[i] = sub(sub(B.Dt[i], mul(B.Lt[i], Rl, R)), mul(B.Ut[i], Sf, R));
    B.Uh[i] = neg(mul(B.Ut[i], Rf, R));
  }
  return CB_OK;
}

// --------------------------------------------- reduced block PCR (Alg. 3) --
// Power-of-two P: log2(P) block-PCR levels, then the final solve with the
// couplings that alias the row itself folded into the diagonal block.
cb_status lane_block_pcr(const Blocks &B, std::vector<double> &red, std::vector<double> &wf,
                         std::string &msg) {
  const int P = B.P, R = B.R, RR = R * R;
  std::vector<Mat> W(B.Dh), Lh(B.Lh), Uh(B.Uh);
  const int T = ceil_log2(P);
  red.assign((size_t)T * P * 2 * RR, 0.0);
  for (int t = 0; t < T; ++t) {
    const int s = 1 << t;
    std::vector<Mat> Winv(P);
    for (int i = 0; i < P; ++i)
      if (!inverse(W[i], R, Winv[i])) {
        msg = "reduced system: singular diagonal block during block PCR";
        return CB_ERR_SINGULAR;
      }
    std::vector<Mat> W2(P), L2(P), U2(P);
    for (int i = 0; i < P; ++i) {
      const int ip = (i + s) % P, im = (i - s % P + P) % P;
      Mat MU = mul(Uh[i], Winv[ip], R), ML = mul(Lh[i], Winv[im], R);
      W2[i] = sub(sub(W[i], mul(MU, Lh[ip], R)), mul(ML, Uh[im], R));
      L2[i] = neg(mul(ML, Lh[im], R));
      U2[i] = neg(mul(MU, Uh[ip], R));
      std::copy(MU.begin(), MU.end(), red.begin() + (((size_t)t * P + i) * 2 + 0) * RR);
      std::copy(ML.begin(), ML.end(), red.begin() + (((size_t)t * P + i) * 2 + 1) * RR);
    }
    W.swap(W2);
    Lh.swap(L2);
    Uh.swap(U2);
  }
  wf.assign((size_t)P * RR, 0.0);
  for (int i = 0; i < P; ++i) {
    Mat inv;
    if (!inverse(add(add(W[i], Lh[i]), Uh[i]), R, inv)) {
      msg = "reduced system is singular (the matrix A is singular)";
      return CB_ERR_SINGULAR;
    }
    std::copy(inv.begin(), inv.end(), wf.begin() + (size_t)i * RR);
  }
  return CB_OK;
}

// Algorithm 1's level loop for any P (Algorithms 2-4), written as phases.
cb_status wg_program(const Blocks &B, RedProgram &pg, std::string &msg) {
  const int P = B.P, R = B.R, RR = R * R;
  pg.P = P;
  pg.R = R;
  std::vector<Mat> W(B.Dh), Lh(B.Lh), Uh(B.Uh);
  struct Term { int dst, src; Mat m; };
  std::vector<std::vector<Term>> phases;
  auto emit = [&](std::vector<Term> &&terms) { phases.push_back(std::move(terms)); };
  auto inv_of = [&](const Mat &a, Mat &out) -> bool {
    if (!inverse(a, R, out)) {
      msg = "reduced system: singular diagonal block";
      return false;
    }
    return true;
  };
  int s = 1, n0 = P, na = P;
  std::vector<int> stack;
  struct Det { int d; Mat Winv, Lh, Uh; };
  std::vector<std::vector<Det>> det_levels;
  while (n0 > 1) {
    const int odd = n0 % 2;
    stack.push_back(odd);
    if (odd) {
      n0 -= 1;
      na -= s;
      // Algorithm 2: the last row d of each sub-system eliminates its
      // couplings into its predecessor d-s and into the sub-system's first
      // row d-na (its cyclic successor), then leaves.
      std::vector<Term> terms;
      std::vector<Det> dets;
      std::vector<Mat> W2(W), L2(Lh), U2(Uh);
      std::vector<int> rows;
      for (int d = na; d < na + s; ++d) {
        Mat Wd;
        if (!inv_of(W[d], Wd)) return CB_ERR_SINGULAR;
        const int i1 = d - s, i2 = d - na;
        Mat M1 = mul(Uh[i1], Wd, R), M2 = mul(Lh[i2], Wd, R);
        W2[i1] = sub(W2[i1], mul(M1, Lh[d], R));
        U2[i1] = neg(mul(M1, Uh[d], R));
        W2[i2] = sub(W2[i2], mul(M2, Uh[d], R));
        L2[i2] = neg(mul(M2, Lh[d], R));
        terms.push_back({i1, i1, eye(R)});
        terms.push_back({i1, d, neg(M1)});
        terms.push_back({i2, i2, eye(R)});
        terms.push_back({i2, d, neg(M2)});
        dets.push_back({d, Wd, Lh[d], Uh[d]});
        rows.push_back(d);
      }
      W.swap(W2);
      Lh.swap(L2);
      Uh.swap(U2);
      emit(std::move(terms));
      det_levels.push_back(std::move(dets));
      pg.detached.push_back(rows);
      pg.detach_steps++;
    } else {
      det_levels.emplace_back();
      pg.detached.emplace_back();
    }
    // Algorithm 3 on the attached rows, neighbours modulo na.
    std::vector<Mat> Winv(na);
    for (int i = 0; i < na; ++i)
      if (!inv_of(W[i], Winv[i])) return CB_ERR_SINGULAR;
    std::vector<Term> terms;
    std::vector<Mat> W2(W), L2(Lh), U2(Uh);
    for (int i = 0; i < na; ++i) {
      const int ip = (i + s) % na, im = (i - s % na + na) % na;
      Mat MU = mul(Uh[i], Winv[ip], R), ML = mul(Lh[i], Winv[im], R);
      W2[i] = sub(sub(W[i], mul(MU, Lh[ip], R)), mul(ML, Uh[im], R));
      L2[i] = neg(mul(ML, Lh[im], R));
      U2[i] = neg(mul(MU, Uh[ip], R));
      terms.push_back({i, i, eye(R)});
      terms.push_back({i, ip, neg(MU)});
      terms.push_back({i, im, neg(ML)});
    }
    W.swap(W2);
    Lh.swap(L2);
    Uh.swap(U2);
    emit(std::move(terms));
    pg.pcr_steps++;
    s *= 2;
    n0 /= 2;
  }
  // Final solve of the attached rows: the couplings at +-s alias the row.
  {
    std::vector<Term> terms;
    for (int i = 0; i < na; ++i) {
      Mat inv;
      if (!inverse(add(add(W[i], Lh[i]), Uh[i]), R, inv)) {
        msg = "reduced system is singular (the matrix A is singular)";
        return CB_ERR_SINGULAR;
      }
      terms.push_back({i, i, inv});
    }
    emit(std::move(terms));
  }
  // Algorithm 4, in reverse level order: x_d = W_d^{-1}(x_d - L^_d x_{d-s} - U^_d x_{d-na}).
  while (!stack.empty()) {
    n0 *= 2;
    s /= 2;
    const int odd = stack.back();
    stack.pop_back();
    std::vector<Det> dets = std::move(det_levels.back());
    det_levels.pop_back();
    if (odd) {
      std::vector<Term> terms;
      for (const Det &dt : dets) {
        const int d = dt.d;
        terms.push_back({d, d, dt.Winv});
        terms.push_back({d, d - s, neg(mul(dt.Winv, dt.Lh, R))});
        terms.push_back({d, d - na, neg(mul(dt.Winv, dt.Uh, R))});
      }
      emit(std::move(terms));
      na += s;
      n0 += 1;
    }
  }
  // Flatten: terms sorted by (phase, dst).
  pg.nphase = (int)phases.size();
  pg.row_off.assign((size_t)pg.nphase * (P + 1), 0);
  pg.src.clear();
  pg.mats.clear();
  for (int ph = 0; ph < pg.nphase; ++ph) {
    auto &terms = phases[ph];
    std::stable_sort(terms.begin(), terms.end(),
                     [](const Term &a, const Term &b) { return a.dst < b.dst; });
    size_t pos = 0;
    for (int dst = 0; dst <= P; ++dst) {
      pg.row_off[(size_t)ph * (P + 1) + dst] = (int)pg.src.size();
      while (dst < P && pos < terms.size() && terms[pos].dst == dst) {
        pg.src.push_back(terms[pos].src);
        pg.mats.insert(pg.mats.end(), terms[pos].m.begin(), terms[pos].m.end());
        ++pos;
      }
    }
  }
  (void)RR;
  return CB_OK;
}

// ---------------------------------------------------- segment (lane level) --
// Lane layout preferences.  Unit-stride launches read a lane's rows as one
// contiguous run, so fewer rows per lane spread each load instruction over
// fewer cache lines; strided launches read whole row segments of adjacent
// lines and prefer more rows per lane (fewer lanes, so more lines share a
// workgroup, and fewer block-PCR levels in LDS).
enum { PREF_X = 0, PREF_S = 1 };

// Rows per lane that have kernel instances for each half bandwidth:
// r = 1, 2: 4, 6, 8, 12, 16, 32; r = 3: 8 and 16.
bool rows_per_lane_built(int R, int M) { return R <= 2 || M == 8 || M == 16; }

bool lane_layout(int S, int R, int M_req, int &L, int &M, bool &uniform, int &m_uni,
                 bool allow_uniform, int L_req = 0, int pref = PREF_S, int m_max = 16, int lcap = 1024) {
  static const int kUniMx[] = {8, 4, 6, 12, 16, 32};
  static const int kUniMs[] = {32, 16, 12, 8, 6, 4};
  const int *kUniM = pref == PREF_X ? kUniMx : kUniMs;
  if (allow_uniform) {
    // first lines of at most 64 lanes in the preferred order, then longer
    // lines with as few lanes as possible (fewer block-PCR levels)
    for (int pass = 0; pass < 2; ++pass)
      for (int mi = 0; mi < 6; ++mi) {
        const int m = pass == 0 ? kUniM[mi] : kUniMs[mi];
        if (M_req && m != M_req) continue;
        if (!M_req && m > m_max) continue;
        if (m < 2 * R || S % m) continue;
        if (!rows_per_lane_built(R, m)) continue;
        const int l = S / m;
        const int lmax = pass == 0 ? 64 : lcap;
        if (!is_pow2(l) || l > lmax) continue;
        L = l;
        M = m;
        uniform = true;
        m_uni = m;
        return true;
      }
  }
  // general layout (lanes of two sizes): unit-stride launches prefer 8 rows
  // per lane while a line needs at most 512 of them (the thread bound of the
  // general unit-stride kernels), strided ones 16 (fewer lanes, so 16 lines
  // share a workgroup)
  uniform = false;
  m_uni = 0;
  if (M_req) M = M_req;
  else if (pref == PREF_S) M = m_max >= 16 ? 16 : 8;
  else M = ((S + 7) / 8 <= 512 || m_max < 16) ? 8 : 16;
  if (M != 8 && M != 16) return false;
  auto fits = [&](int m, int &l) {
    if (L_req > 0) {
      l = L_req;
    } else {
      l = 1;
      while (l * m < S) l *= 2;
      while (l > 1 && S / l < 2 * R) l /= 2;
    }
    return !(l > lcap || (S + l - 1) / l > m || S / l < 2 * R);
  };
  if (fits(M, L)) return true;
  // lanes of 8 rows hold only 2r..8 of them: some lengths need 16-row lanes
  // (r = 3 above all), the other way round when 16-row lanes exceed lcap
  if (M_req || (M == 16 && m_max < 16)) return false;
  const int alt = M == 8 ? 16 : 8;
  if (alt == 16 && m_max < 16) return false;
  if (!fits(alt, L)) return false;
  M = alt;
  return true;
}

// --------------------------------------- boundary rows of D_i^{-1} (Sec. 4) --
// The partitions exchange only b~_i and the first and last R rows of
// y_i = D_i^{-1} b_i (Eq. (21); L~ and U~ touch nothing else).  Those rows
// are fixed linear functionals of b_i: rows 0..R-1 and N-R..N-1 of D_i^{-1}.
// They are rows of the inverse, i.e. solutions of D_i^T g = e_a, computed by
// banded elimination of D_i^T.  For the diagonally dominant compact schemes
// their entries decay geometrically away from the diagonal, so each is kept
// over a window at its own end of D_i: the window is the shortest one whose
// omitted entries sum, in absolute value, to at most 2^-56 of the row's
// absolute sum (below the rounding of the dot product itself).  One window
// length Kw serves every partition and row; Kw <= max N_i.
cb_status boundary_rows(int P, int R, const std::vector<int> &st, const std::function<double(int, int)> &coef,
                        int &Kw, std::vector<double> &out, std::string &msg) {
  const int W = 2 * R + 1;
  const double rel = std::ldexp(1.0, -56);
  std::vector<std::vector<double>> rows((size_t)P * 2 * R);
  int kmax = 1, nmax = 0;
  for (int i = 0; i < P; ++i) {
    const int s0 = st[i] + R, N = st[i + 1] - s0;
    nmax = std::max(nmax, N);
    // band of D_i^T: D^T[j][j+o] = D[j+o][j]
    std::vector<double> bt((size_t)N * W, 0.0);
    for (int j = 0; j < N; ++j)
      for (int o = -R; o <= R; ++o)
        if (j + o >= 0 && j + o < N) bt[(size_t)j * W + o + R] = coef(s0 + j + o, -o);
    std::vector<double> lu((size_t)N * 2 * R), dv(N);
    cb_status s = lane_lu(N, R, bt, lu.data(), dv.data(), msg);
    if (s != CB_OK) {
      msg = "boundary rows of an interior block: " + msg;
      return s;
    }
    for (int end = 0; end < 2; ++end)
      for (int a = 0; a < R; ++a) {
        std::vector<double> g(N, 0.0);
        const int row = end == 0 ? a : N - R + a;
        g[row] = 1.0;
        for (int j = 1; j < N; ++j)
          for (int q = 1; q <= R; ++q)
            if (j - q >= 0) g[j] -= lu[(size_t)j * 2 * R + q - 1] * g[j - q];
        for (int j = N - 1; j >= 0; --j) {
          double acc = g[j] * dv[j];
          for (int q = 1; q <= R; ++q)
            if (j + q < N) acc -= lu[(size_t)j * 2 * R + R + q - 1] * g[j + q];
          g[j] = acc;
        }
        double sum = 0.0;
        for (double v : g) sum += std::fabs(v);
        // shortest window at this end whose omitted entries stay below rel * sum
        double omitted = 0.0;
        int k = N;
        for (int c = N - 1; c >= 1; --c) {  // c = window length if entries beyond it are omitted
          const double v = std::fabs(end == 0 ? g[c] : g[N - 1 - c]);
          if (omitted + v > rel * sum) break;
          omitted += v;
          k = c;
        }
        kmax = std::max(kmax, k);
        rows[((size_t)i * 2 + end) * R + a] = std::move(g);
      }
  }
  // a block shorter than the window (partitions differ by a row) keeps all
  // its entries; the window positions beyond it hold zeros
  Kw = std::min(kmax, nmax);
  out.assign((size_t)P * 2 * R * Kw, 0.0);
  for (int i = 0; i < P; ++i) {
    const int N = st[i + 1] - st[i] - R;
    for (int end = 0; end < 2; ++end)
      for (int a = 0; a < R; ++a) {
        const std::vector<double> &g = rows[((size_t)i * 2 + end) * R + a];
        double *o = out.data() + (((size_t)i * 2 + end) * R + a) * Kw;
        for (int j = 0; j < Kw; ++j) {
          const int row = end == 0 ? j : N - Kw + j;
          o[j] = (row >= 0 && row < N) ? g[row] : 0.0;
        }
      }
  }
  return CB_OK;
}

cb_status build_segment(int S, int R, bool cyclic, bool per_row_any,
                        const std::function<double(int, int)> &coef, int M_req, SegPlan &sp,
                        std::string &msg, int L_req = 0, int pref = PREF_S, int m_max = 16, int interior = 0,
                        int lcap = 1024) {
  int L, M, m_uni;
  bool uni;
  if (!lane_layout(S, R, M_req, L, M, uni, m_uni, cyclic && !per_row_any && L_req == 0, L_req, pref,
                   m_max, lcap)) {
    msg = "no lane layout for this segment length (rows_per_lane unsupported?)";
    return CB_ERR_UNSUPPORTED;
  }
  sp.S = S;
  sp.cyclic = cyclic;
  sp.L = L;
  sp.M = M;
  sp.R = R;
  sp.N = M - R;
  sp.Tint = ceil_log2(sp.N);
  sp.Tred = ceil_log2(L);
  sp.uniform = uni;
  sp.m_uniform = m_uni;
  // interior solve: 0/1 generalized PCR, 2 elimination, 3 elimination where
  // a kernel exists for it (8 or 16 rows per lane, or 12 on uniform lanes),
  // 4 elimination for general layouts only
  // 32 rows per lane (uniform FP64 lanes only) always eliminate
  sp.ilu = (interior == 2 && (M == 8 || M == 12 || M == 16 || M == 32)) ||
                   (interior == 3 && (M == 8 || M == 16 || ((M == 12 || M == 32) && uni))) ||
                   (interior == 4 && !uni && (M == 8 || M == 16)) || (M == 32 && interior != 1)
               ? 1
               : 0;
  if (interior == 2 && !sp.ilu) {
    msg = "interior elimination needs rows_per_lane 8, 12, 16 or 32";
    return CB_ERR_UNSUPPORTED;
  }
  if (M == 32 && (!uni || !sp.ilu)) {
    msg = "32 rows per lane need uniform lanes and interior elimination";
    return CB_ERR_UNSUPPORTED;
  }
  // the first S mod L lanes hold one row more (the kernels recompute these
  // starts from S and L, see lane_rows)
  std::vector<int> st(L + 1);
  const int base = S / L, extra = S % L;
  st[0] = 0;
  for (int l = 0; l < L; ++l) st[l + 1] = st[l] + base + (l < extra ? 1 : 0);
  sp.lane_start = st;
  Blocks B;
  cb_status s = build_blocks(L, R, st, cyclic, coef, sp.Tint, B, msg);
  if (s != CB_OK) return s;
  // coefficient blocks, padded to N = M-R slots, deduplicated by content
  const int blk = coef_block_size(R, M, sp.Tint, sp.ilu);
  const CoefOff off = coef_offsets(R, M, sp.Tint, sp.ilu);
  sp.block = blk;
  sp.lane_type.assign(L, 0);
  sp.coef.clear();
  sp.ntypes = 0;
  const int N = sp.N;
  for (int l = 0; l < L; ++l) {
    std::vector<double> b(blk, 0.0);
    const int Nl = st[l + 1] - st[l] - R;
    if (sp.ilu) {
      // the lane's interior band, rebuilt from the segment rows
      std::vector<double> band((size_t)Nl * (2 * R + 1), 0.0);
      for (int j = 0; j < Nl; ++j)
        for (int o = -R; o <= R; ++o)
          if (j + o >= 0 && j + o < Nl) band[j * (2 * R + 1) + o + R] = coef(st[l] + R + j, o);
      std::vector<double> lu((size_t)Nl * 2 * R), dv(Nl);
      cb_status s2 = lane_lu(Nl, R, band, lu.data(), dv.data(), msg);
      if (s2 != CB_OK) return s2;
      for (int j = 0; j < Nl; ++j) {
        for (int u = 0; u < 2 * R; ++u) b[off.k + j * 2 * R + u] = lu[j * 2 * R + u];
        b[off.dinv + j] = dv[j];
      }
    } else {
      for (int t = 0; t < sp.Tint; ++t)
        for (int j = 0; j < Nl; ++j)
          for (int u = 0; u < 2 * R; ++u)
            b[off.k + ((size_t)t * N + j) * 2 * R + u] = B.D[l].k[((size_t)t * Nl + j) * 2 * R + u];
      for (int j = 0; j < Nl; ++j) b[off.dinv + j] = B.D[l].dinv[j];
    }
    for (int q = 0; q < R * R; ++q) {
      b[off.Lt + q] = B.Lt[l][q];
      b[off.Ut + q] = B.Ut[l][q];
    }
    for (int j = 0; j < Nl; ++j)
      for (int c = 0; c < R; ++c) {
        b[off.S + j * R + c] = B.Sm[l][j * R + c];
        b[off.Rm + j * R + c] = B.Rm[l][j * R + c];
      }
    int found = -1;
    for (int ty = 0; ty < sp.ntypes; ++ty)
      if (std::memcmp(&sp.coef[(size_t)ty * blk], b.data(), sizeof(double) * blk) == 0) {
        found = ty;
        break;
      }
    if (found < 0) {
      found = sp.ntypes++;
      sp.coef.insert(sp.coef.end(), b.begin(), b.end());
    }
    sp.lane_type[l] = found;
  }
  if (uni && sp.ntypes != 1) {
    msg = "internal: uniform layout produced differing lane partitions";
    return CB_ERR_INVALID_ARG;
  }
  return lane_block_pcr(B, sp.red, sp.wf, msg);
}

}  // namespace

// ------------------------------------------------------------------- plan --
// Refinement count when the caller leaves it to the library.  The FP32
// reduction returns x with relative error about kappa(A) u (u = 2^-24), and
// each FP64-residual refinement step multiplies the error by about the same
// factor, since its correction solve has that relative error (the classical
// analysis of mixed-precision iterative refinement); k steps leave about
// (kappa u)^(k+1).  The count is the smallest k >= 1 with
// (kappa u)^(k+1) <= 1e-13, ten times below the 1e-12 target.  kappa comes
// from the symbol f(t) = a_0 + 2 sum_j a_j cos(j t) of constant symmetric
// bands: its values at t = 2 pi k / n are the eigenvalues of the cyclic
// matrix, and its range holds the spectrum of the acyclic one.  Per-row or
// unsymmetric bands, and symbols that change sign, take 2 steps.
int auto_refine_iters(const cb_plan_desc &d) {
  const int R = d.r, n = d.n;
  if (d.per_row) return 2;
  double scale = 0.0;
  for (int o = 0; o <= 2 * R; ++o) scale = std::max(scale, std::fabs(d.bands[o]));
  for (int j = 1; j <= R; ++j)
    if (std::fabs(d.bands[R - j] - d.bands[R + j]) > 1e-15 * scale) return 2;
  const double two_pi = 6.283185307179586476925287;
  const bool exact = d.cyclic && n <= 65536;
  const int np = exact ? n : 65536;
  double fmin = INFINITY, fmax = -INFINITY;
  for (int k = 0; k <= np; ++k) {  // k = np repeats t = 0 (the cyclic case) or reaches t = pi
    const double t = exact ? two_pi * (k % np) / np : two_pi * 0.5 * k / np;
    double f = d.bands[R];
    for (int j = 1; j <= R; ++j) f += 2.0 * d.bands[R + j] * std::cos(j * t);
    fmin = std::min(fmin, f);
    fmax = std::max(fmax, f);
  }
  if (!(fmin > 0.0 || fmax < 0.0)) return 2;
  const double ku = std::max(std::fabs(fmin), std::fabs(fmax)) / std::min(std::fabs(fmin), std::fabs(fmax)) *
                    5.9604644775390625e-8;
  double e = ku * ku;
  int k = 1;
  while (e > 1e-13 && k < 8) {
    e *= ku;
    ++k;
  }
  return k;
}

cb_status build_plan(const cb_plan_desc &d, Plan &p, std::string &msg) {
  if (d.r < 1 || d.r > kMaxR) {
    msg = "r must be 1 (tridiagonal), 2 (pentadiagonal) or 3 (heptadiagonal)";
    return d.r > kMaxR ? CB_ERR_UNSUPPORTED : CB_ERR_INVALID_ARG;
  }
  if (d.r == 3 && d.rows_per_lane && d.rows_per_lane != 8 && d.rows_per_lane != 16) {
    msg = "heptadiagonal plans (r = 3) take 8 or 16 rows per lane";
    return CB_ERR_UNSUPPORTED;
  }
  if (!d.bands) {
    msg = "bands is NULL";
    return CB_ERR_INVALID_ARG;
  }
  if (d.precision < CB_FP64 || d.precision > CB_FP32_REFINE) {
    msg = "unknown precision";
    return CB_ERR_INVALID_ARG;
  }
  if (d.rows_per_lane && d.rows_per_lane != 4 && d.rows_per_lane != 6 && d.rows_per_lane != 8 &&
      d.rows_per_lane != 12 && d.rows_per_lane != 16 && d.rows_per_lane != 32) {
    msg = "rows_per_lane must be 0, 4, 6, 8, 12, 16 or 32";
    return CB_ERR_UNSUPPORTED;
  }
  if (d.lines_per_wg < 0 || d.lines_per_wg > 1024 || (d.lines_per_wg & (d.lines_per_wg - 1)) ||
      d.block_barriers < 0 || d.block_barriers > 1 || d.x_staging < 0 || d.x_staging > 2 || d.interior < 0 ||
      d.interior > 2 || d.tile_order < 0 || d.tile_order > 2) {
    msg = "lines_per_wg must be 0 or a power of two <= 1024; block_barriers 0 or 1; x_staging, interior and "
          "tile_order 0..2";
    return CB_ERR_INVALID_ARG;
  }
  const int R = d.r, n = d.n, W = 2 * R + 1;
  // partitions 0: one workgroup per line while a line fits one (FP64 16384
  // rows: 1024 lanes of 16; FP32 8192: 512 lanes of 16), else ~1024-row
  // workgroup partitions (measured fastest among 512-, 1024- and 2048-row
  // ones at n = 8192), at most 64
  const int one_wg_rows = d.precision == CB_FP64 ? 16384 : 8192;
  const int P = d.partitions > 0 ? d.partitions : (n > one_wg_rows ? std::min(64, (n + 1023) / 1024) : 1);
  if (P > 64) {
    msg = "at most 64 workgroup partitions per line";
    return CB_ERR_UNSUPPORTED;
  }
  if (n < 2 * R * P + (P == 1 ? 0 : R * P) || n < 2 * R + 1 || n > (1 << 24)) {
    msg = "line length n too small for r and the partition count (or too large)";
    return CB_ERR_INVALID_ARG;
  }
  p.desc = d;
  p.desc.bands = nullptr;
  p.R = R;
  p.n = n;
  p.P = P;
  p.precision = d.precision;
  p.refine_iters = d.precision == CB_FP32_REFINE ? (d.refine_iters > 0 ? d.refine_iters : auto_refine_iters(d)) : 0;
  if (p.refine_iters > 8) {
    msg = "at most 8 refinement iterations";
    return CB_ERR_INVALID_ARG;
  }
  p.bands.assign((size_t)n * W, 0.0);
  for (int j = 0; j < n; ++j)
    for (int o = 0; o < W; ++o) {
      const double v = d.per_row ? d.bands[(size_t)j * W + o] : d.bands[o];
      if (!std::isfinite(v)) {
        msg = "bands contain a non-finite value";
        return CB_ERR_INVALID_ARG;
      }
      p.bands[(size_t)j * W + o] = v;
    }
  if (!d.cyclic) {  // acyclic: entries outside the matrix are ignored
    for (int j = 0; j < n; ++j)
      for (int o = -R; o <= R; ++o)
        if (j + o < 0 || j + o >= n) p.bands[(size_t)j * W + o + R] = 0.0;
  }
  const bool per_row = d.per_row != 0;
  const bool cyclic = d.cyclic != 0;
  auto line_coef = [&](int g, int o) -> double { return p.bands[(size_t)g * W + o + R]; };

  if (P == 1) {
    // segs[0]: layout for unit-stride launches; segs[seg_s]: for strided ones
    // the FP32 reduction keeps FP64 refinement state beside it: at most 8 rows
    // per lane unless asked for
    // FP32 line kernels run at most 512 threads, so at most 512 lanes: long
    // FP32 lines may use 16 rows per lane
    // (r = 3: lanes of 8 rows fit only lines of 6..8 rows per lane, so FP32
    // may take 16 there too)
    const int m_max = d.precision == CB_FP64 || n > 8 * 512 || R == 3 ? 16 : 8;
    const int lcap = d.precision == CB_FP64 ? 1024 : 512;
    p.segs.resize(1);
    // unit-stride lines: generalized PCR interiors on uniform FP64 lanes,
    // elimination on general ones and wherever available in FP32 (its three
    // solves make the lane work count: penta +10 %), unless asked
    cb_status s = build_segment(n, R, cyclic, per_row, line_coef, d.rows_per_lane, p.segs[0], msg, 0, PREF_X,
                                m_max, d.interior ? d.interior : (d.precision == CB_FP64 ? 4 : 3), lcap);
    if (s != CB_OK && d.interior == 0)
      s = build_segment(n, R, cyclic, per_row, line_coef, d.rows_per_lane, p.segs[0], msg, 0, PREF_X, m_max, 1,
                        lcap);
    if (s != CB_OK) return s;
    p.seg_s = 0;
    if (!d.rows_per_lane) {
      // strided lines: lane interiors by elimination unless asked otherwise
      // (fewer live registers per lane; PCR if a pivot vanishes)
      SegPlan alt;
      // FP64 strided lines on uniform lanes take 32 rows per lane when the
      // lane count allows (32 adjacent lines per workgroup, 256-byte segments)
      // (FP32: up to 12 rows per lane, measured faster than 6 at n = 384)
      // (32-row lanes always eliminate: not when generalized PCR is asked for)
      const int m_max_s = d.precision == CB_FP64 ? (d.interior == 1 ? 16 : 32) : std::max(m_max, 12);
      // FP32 lines whose rows split into uniform lanes of 16 take those for
      // r >= 2 from n = 256 and for r = 1 at n = 512..1024 (at 512^3 y / z
      // with one refinement: 214 / 157 -> 242 / 223 GDOF/s tridiagonal,
      // 144 / 99 -> 150 / 138 pentadiagonal); tridiagonal lines of 256 or of
      // 2048 and more rows, and general layouts, run faster on 8
      const bool fp32_16 = d.precision != CB_FP64 && n >= 256 && (R >= 2 || (n >= 512 && n <= 1024));
      s = CB_ERR_UNSUPPORTED;
      if (fp32_16) {
        std::string m16;
        s = build_segment(n, R, cyclic, per_row, line_coef, 0, alt, m16, 0, PREF_S, 16, d.interior ? d.interior : 3,
                          lcap);
        if (s == CB_OK && !(alt.uniform && alt.M == 16)) s = CB_ERR_UNSUPPORTED;
      }
      if (s != CB_OK)
        s = build_segment(n, R, cyclic, per_row, line_coef, 0, alt, msg, 0, PREF_S, m_max_s,
                          d.interior ? d.interior : 3, lcap);
      if (s != CB_OK && d.interior == 0)
        s = build_segment(n, R, cyclic, per_row, line_coef, 0, alt, msg, 0, PREF_S, m_max, 1, lcap);
      if (s != CB_OK) return s;
      if (alt.M != p.segs[0].M || alt.L != p.segs[0].L || alt.ilu != p.segs[0].ilu) {
        p.segs.push_back(std::move(alt));
        p.seg_s = 1;
      }
    }
    p.M = p.segs[0].M;
    p.L = p.segs[0].L;
    p.wg_start = {0, n};
    // ragged FP64 lines of 1025..4096 rows (general strided layouts of
    // 128-256 lanes): strided launches run ~512-row workgroup partitions
    // instead (n = 1030-4000 along y / z: 84-174 -> 122-233 GDOF/s; the
    // uniform layouts of 2048 and 4096 rows are faster whole).  FP32 lines
    // the same from 4097 rows and, on general layouts, from 2049 (FP32 +
    // refinement n = 2500-8192 along y / z: 12-65 -> 41-101 GDOF/s; at
    // 1100 rows whole lines are as fast)
    const bool general_s = !p.segs[p.seg_s].uniform;
    const bool split = n > 4096 || (general_s && n > (d.precision == CB_FP64 ? 1024 : 2048));
    if (split && !d.rows_per_lane && !d.lines_per_wg) {
      cb_plan_desc dw = d;
      // (~512-row partitions also beyond 4096 rows, up to the 16384 rows of a
      // one-partition plan: n = 5000-16384 tridiagonal y / z 5-13 % faster
      // than ~1024-row ones, pentadiagonal within 3 % either way)
      dw.partitions = (n + 511) / 512;
      dw.x_staging = 0;
      dw.interior = 0;
      auto w = std::make_shared<Plan>();
      std::string m2;
      if (build_plan(dw, *w, m2) == CB_OK) p.strided_wg = w;  // else strided lines stay whole
    }
    if (d.lines_per_wg && d.lines_per_wg * p.L > 1024) {
      msg = "lines_per_wg * lanes exceeds 1024 threads";
      return CB_ERR_INVALID_ARG;
    }
    return CB_OK;
  }
  // P > 1: workgroup partitions, each with R interface rows and an interior
  // segment D_i solved by the lane-level scheme (banded elimination unless
  // asked otherwise or a pivot vanishes: generalized PCR then).
  p.wg_start.assign(P + 1, 0);
  const int base = n / P, extra = n % P;
  for (int i = 0; i < P; ++i) p.wg_start[i + 1] = p.wg_start[i] + base + (i < extra ? 1 : 0);
  Blocks B;
  cb_status s = build_blocks(P, R, p.wg_start, cyclic, line_coef, -1, B, msg);
  if (s != CB_OK) return s;
  // One lane layout per set of partitions (a kernel has one M): segs[0..P)
  // for unit-stride launches, 8 rows per lane while a partition needs at most
  // 64 lanes of them, else 16; strided launches take 16 rows per lane in
  // segs[P..2P) (measured faster at every P: n = 8192, P = 16: 209 vs 150
  // GDOF/s along y), or the unit-stride set when that already has 16.
  auto build_set = [&](int M, std::vector<SegPlan> &set) -> cb_status {
    const int Smax = base + (extra ? 1 : 0) - R;
    int Lg = 0, m_uni;
    bool uni;
    if (!lane_layout(Smax, R, M, Lg, M, uni, m_uni, false)) {
      msg = "no lane layout for the partition size";
      return CB_ERR_UNSUPPORTED;
    }
    set.assign(P, SegPlan());
    cb_status st = CB_OK;
    for (int pass = 0; pass < 2; ++pass) {
      // one kernel serves all partitions: every segment takes the same
      // interior solve (elimination for all, or generalized PCR for all)
      const int interior = d.interior ? d.interior : (pass == 0 ? 2 : 1);
      st = CB_OK;
      for (int i = 0; i < P && st == CB_OK; ++i) {
        const int g0 = p.wg_start[i] + R;
        const int S = p.wg_start[i + 1] - g0;
        auto seg_coef = [&, g0](int g, int o) -> double { return line_coef(g0 + g, o); };
        st = build_segment(S, R, false, true, seg_coef, M, set[i], msg, Lg, PREF_S, 16, interior);
      }
      if (st == CB_OK || d.interior) break;
    }
    if (st != CB_OK) return st;
    for (int i = 1; i < P; ++i)
      if (set[i].L != set[0].L) {
        msg = "partition sizes need different lane counts; choose n divisible by P";
        return CB_ERR_UNSUPPORTED;
      }
    return CB_OK;
  };
  const int Smax0 = base + (extra ? 1 : 0) - R;
  const int M = d.rows_per_lane ? d.rows_per_lane : ((Smax0 + 7) / 8 <= 64 ? 8 : 16);
  s = build_set(M, p.segs);
  if (s != CB_OK && !d.rows_per_lane && M == 8) s = build_set(16, p.segs);
  if (s != CB_OK) return s;
  p.M = p.segs[0].M;
  p.L = p.segs[0].L;
  p.seg_s = 0;
  if (!d.rows_per_lane && p.M != 16) {
    std::vector<SegPlan> strided;
    std::string m2;
    std::swap(m2, msg);
    if (build_set(16, strided) == CB_OK) {
      p.seg_s = P;
      for (SegPlan &sp : strided) p.segs.push_back(std::move(sp));
    }
    std::swap(m2, msg);  // a strided set that cannot be built leaves the unit-stride one for both
  }
  // full-block segments for phase C (see plan.h), one per lane-layout set
  if (!per_row && n % P == 0) {
    const int sblk = n / P, W2 = 2 * R + 1;
    std::vector<double> bc(W2);
    for (int o = 0; o < W2; ++o) bc[o] = p.bands[(size_t)(n / 2) * W2 + o];
    auto full_block = [&](const SegPlan &like, int &type) -> int {
      const int M = like.M, L = sblk / M;
      if (L * M != sblk || !is_pow2(L) || L < 4 || L > 1024 || !like.ilu) return -1;
      auto coef = [&](int g, int o) -> double {
        if (g < R) return o == 0 ? 1.0 : 0.0;  // interface rows: x = x~_i
        const int c = g + o;
        return (c >= 0 && c < sblk) ? bc[o + R] : 0.0;  // couplings beyond the block move to the RHS
      };
      SegPlan fb;
      std::string m2;
      if (build_segment(sblk, R, false, true, coef, M, fb, m2, L, PREF_S, 16, 2) != CB_OK || !fb.ilu) return -1;
      // lane types: first, middle (all alike), last; the first and last may
      // differ from the middle only in the terms the kernel masks
      const int t0 = fb.lane_type[0], t1 = fb.lane_type[1], t2 = fb.lane_type[L - 1];
      for (int l = 1; l < L - 1; ++l)
        if (fb.lane_type[l] != t1) return -1;
      const CoefOff off = coef_offsets(R, M, fb.Tint, true);
      const double *b0 = &fb.coef[(size_t)t0 * fb.block], *b1 = &fb.coef[(size_t)t1 * fb.block],
                   *b2 = &fb.coef[(size_t)t2 * fb.block];
      for (int q = 0; q < fb.block; ++q) {
        const bool ltut = q >= off.Lt && q < off.S, rm = q >= off.Rm;
        if (b0[q] != (ltut ? 0.0 : b1[q])) return -1;
        if (b2[q] != (rm ? 0.0 : b1[q])) return -1;
      }
      type = t1;
      p.segs.push_back(std::move(fb));
      return (int)p.segs.size() - 1;
    };
    p.fb_seg_u = full_block(p.segs[0], p.fb_type_u);
    if (p.seg_s != 0) {
      p.fb_seg_s = full_block(p.segs[p.seg_s], p.fb_type_s);
    } else {
      p.fb_seg_s = p.fb_seg_u;
      p.fb_type_s = p.fb_type_u;
    }
  }
  p.SRg.clear();
  p.SRg_off.assign(P, 0);
  for (int i = 0; i < P; ++i) {
    p.SRg_off[i] = (int64_t)p.SRg.size();
    p.SRg.insert(p.SRg.end(), B.Sm[i].begin(), B.Sm[i].end());
    p.SRg.insert(p.SRg.end(), B.Rm[i].begin(), B.Rm[i].end());
  }
  p.LtUtg.assign((size_t)P * 2 * R * R, 0.0);
  for (int i = 0; i < P; ++i)
    for (int q = 0; q < R * R; ++q) {
      p.LtUtg[((size_t)i * 2 + 0) * R * R + q] = B.Lt[i][q];
      p.LtUtg[((size_t)i * 2 + 1) * R * R + q] = B.Ut[i][q];
    }
  s = boundary_rows(P, R, p.wg_start, line_coef, p.Kw, p.bfun, msg);
  if (s != CB_OK) return s;
  return wg_program(B, p.prog, msg);
}

}  // namespace cb
