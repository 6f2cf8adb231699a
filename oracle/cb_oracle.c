/*
 * Oracle: plain FP64 CPU reference for compact banded solves.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition the paper's solver reaches (up to
 * rounding): x = A^{-1} b for a compact banded matrix A of bandwidth w = 2r+1,
 * cyclic (periodic corner blocks) or acyclic (Sec. 1 Eq. (1)-(2); Sec. 2 the
 * banded structure with w = 2r+1; Sec. 3, the cyclic case).  It deliberately
 * uses an unrelated algorithm to the paper's PCR: banded Gaussian elimination
 * (no pivoting) of the acyclic band part, plus a Woodbury rank-2r correction
 * for the cyclic corner entries.  No pivoting means the band part must admit
 * an LU factorisation without row exchanges; this holds for every matrix used
 * here (symmetric positive definite or diagonally dominant compact schemes).
 *
 * Band storage: row j of A is given by (2r+1) numbers a[j][o+r], o = -r..r,
 * meaning A[j][(j+o) mod n] (cyclic) or A[j][j+o] (acyclic; entries that
 * fall outside [0,n) must be zero).  A constant-coefficient matrix passes one
 * row (per_row = 0) that applies to every row.
 *
 * The right-hand-side stencil (Eq. (1), Eq. (2), App. A.2) is evaluated as
 * out_j = sum_{q=lo..hi} c[q-lo] * f_{(j+q) mod n}, summed in increasing q.
 *
 * Status codes: 0 ok, 1 bad argument, 3 singular (zero pivot in the band LU
 * or a singular Woodbury capacitance matrix).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_BAD_ARG 1
#define ORC_SINGULAR 3

/* ---- banded LU without pivoting (lower and upper bandwidth r) ---------- */
/* lu: n x (2r+1), lu[i*(2r+1) + (j-i+r)] = A[i][j] for |j-i| <= r.        */
static int band_lu(int n, int r, double *lu) {
  const int w = 2 * r + 1;
  for (int k = 0; k < n; ++k) {
    const double piv = lu[k * w + r];
    if (piv == 0.0 || !isfinite(piv)) return ORC_SINGULAR;
    const int iend = (k + r < n - 1) ? k + r : n - 1;
    for (int i = k + 1; i <= iend; ++i) {
      double *li = &lu[i * w + (k - i + r)];
      const double l = *li / piv;
      *li = l;
      for (int j = k + 1; j <= iend; ++j)
        lu[i * w + (j - i + r)] -= l * lu[k * w + (j - k + r)];
    }
  }
  return ORC_OK;
}

/* Solve (LU) x = b in place. */
static void band_lu_solve(int n, int r, const double *lu, double *x) {
  const int w = 2 * r + 1;
  for (int i = 0; i < n; ++i) {
    const int j0 = (i - r > 0) ? i - r : 0;
    double s = x[i];
    for (int j = j0; j < i; ++j) s -= lu[i * w + (j - i + r)] * x[j];
    x[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    const int j1 = (i + r < n - 1) ? i + r : n - 1;
    double s = x[i];
    for (int j = i + 1; j <= j1; ++j) s -= lu[i * w + (j - i + r)] * x[j];
    x[i] = s / lu[i * w + r];
  }
}

/* Dense m x m solve with partial pivoting, in place (a is destroyed). */
static int dense_solve(int m, double *a, double *x) {
  double amax = 0.0;
  for (int i = 0; i < m * m; ++i) amax = fmax(amax, fabs(a[i]));
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (fabs(a[i * m + k]) > fabs(a[p * m + k])) p = i;
    /* numerically singular: pivot at rounding level of the matrix scale */
    if (!(fabs(a[p * m + k]) > 1e-12 * amax)) return ORC_SINGULAR;
    if (p != k) {
      for (int j = 0; j < m; ++j) {
        double t = a[k * m + j]; a[k * m + j] = a[p * m + j]; a[p * m + j] = t;
      }
      double t = x[k]; x[k] = x[p]; x[p] = t;
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
  return ORC_OK;
}

static double band_at(const double *bands, int per_row, int r, int j, int o) {
  return bands[(per_row ? j * (2 * r + 1) : 0) + o + r];
}

/* A factorised line operator: band LU plus, for a cyclic A, the Woodbury
 * pieces Z = B^{-1} U (n x 2r) and the LU-free capacitance matrix K. */
typedef struct {
  int n, r, cyclic, m; /* m = 2r corner rows when cyclic, else 0 */
  double *lu;          /* n*(2r+1) */
  int *crow;           /* corner row indices, m */
  double *cval;        /* m x n dense rows of the corner part C = A - B */
  double *z;           /* n x m, column-major: z[c*n + i] */
  double *kmat;        /* m x m capacitance I + V^T Z */
} line_op;

static void op_free(line_op *op) {
  free(op->lu); free(op->crow); free(op->cval); free(op->z); free(op->kmat);
  memset(op, 0, sizeof(*op));
}

static int op_build(line_op *op, int r, int n, const double *bands, int per_row,
                    int cyclic) {
  memset(op, 0, sizeof(*op));
  if (r < 1 || r > 4 || n < 1) return ORC_BAD_ARG;
  if (cyclic && n < 2 * r + 1) return ORC_BAD_ARG;
  const int w = 2 * r + 1;
  op->n = n; op->r = r; op->cyclic = cyclic;
  op->lu = (double *)calloc((size_t)n * w, sizeof(double));
  if (!op->lu) return ORC_BAD_ARG;
  /* B: the acyclic band part; entries whose column wraps go to C. */
  for (int j = 0; j < n; ++j)
    for (int o = -r; o <= r; ++o) {
      const int c = j + o;
      if (c >= 0 && c < n) op->lu[j * w + o + r] = band_at(bands, per_row, r, j, o);
    }
  int st = band_lu(n, r, op->lu);
  if (st) { op_free(op); return st; }
  if (!cyclic) return ORC_OK;

  const int m = 2 * r;
  op->m = m;
  op->crow = (int *)malloc(sizeof(int) * m);
  op->cval = (double *)calloc((size_t)m * n, sizeof(double));
  op->z = (double *)calloc((size_t)m * n, sizeof(double));
  op->kmat = (double *)calloc((size_t)m * m, sizeof(double));
  /* corner rows: the first r rows (wrap to the end) and the last r rows
   * (wrap to the start) */
  for (int k = 0; k < r; ++k) { op->crow[k] = k; op->crow[r + k] = n - r + k; }
  for (int k = 0; k < m; ++k) {
    const int j = op->crow[k];
    for (int o = -r; o <= r; ++o) {
      const int c = j + o;
      if (c < 0 || c >= n) op->cval[k * n + ((c % n) + n) % n] += band_at(bands, per_row, r, j, o);
    }
  }
  /* Z = B^{-1} U with U = [e_crow[k]] */
  for (int k = 0; k < m; ++k) {
    double *zc = &op->z[k * n];
    zc[op->crow[k]] = 1.0;
    band_lu_solve(n, r, op->lu, zc);
  }
  /* K = I + V^T Z where row k of V^T is cval[k] */
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k) {
      double s = (i == k) ? 1.0 : 0.0;
      for (int c = 0; c < n; ++c) s += op->cval[i * n + c] * op->z[k * n + c];
      op->kmat[i * m + k] = s;
    }
  return ORC_OK;
}

/* x = A^{-1} b for one line (x may alias b).  tmp needs 2*m*m + m doubles. */
static int op_apply(const line_op *op, const double *b, double *x, double *tmp) {
  const int n = op->n;
  if (x != b) memcpy(x, b, sizeof(double) * n);
  band_lu_solve(n, op->r, op->lu, x);
  if (!op->cyclic) return ORC_OK;
  const int m = op->m;
  double *kcopy = tmp, *t = tmp + m * m;
  memcpy(kcopy, op->kmat, sizeof(double) * m * m);
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int c = 0; c < n; ++c) s += op->cval[i * n + c] * x[c];
    t[i] = s;
  }
  if (dense_solve(m, kcopy, t)) return ORC_SINGULAR;
  for (int k = 0; k < m; ++k)
    for (int i = 0; i < n; ++i) x[i] -= op->z[k * n + i] * t[k];
  return ORC_OK;
}

/* ---- public: one or many lines of a contiguous (lines x n) array ------- */
/* x = A^{-1} b per line: the system the compact scheme's left-hand side
 * defines (Sec. 1 Eq. (1)-(2); cyclic corners as in Sec. 3). */
int orc_solve_lines(int r, int n, const double *bands, int per_row, int cyclic,
                    int64_t nlines, const double *b, double *x) {
  line_op op;
  int st = op_build(&op, r, n, bands, per_row, cyclic);
  if (st) return st;
  int bad = 0;
  #pragma omp parallel reduction(|:bad)
  {
    double tmp[2 * 8 * 8 + 8];
    #pragma omp for schedule(static)
    for (int64_t l = 0; l < nlines; ++l)
      bad |= op_apply(&op, b + l * n, x + l * n, tmp);
  }
  op_free(&op);
  return bad ? ORC_SINGULAR : ORC_OK;
}

/* ---- 3D arrays: lines along one axis ----------------------------------- */
/* Layout: C order (nz, ny, nx), x unit stride; dims[0]=nx, dims[1]=ny,
 * dims[2]=nz.  Lines run along `axis` (0 = x, 1 = y, 2 = z). */
static void axis_geometry(const int64_t dims[3], int axis, int64_t *n,
                          int64_t *stride, int64_t *nl, int64_t *du, int64_t *su,
                          int64_t *sv) {
  const int64_t st[3] = {1, dims[0], dims[0] * dims[1]};
  const int u = (axis == 0) ? 1 : 0;
  const int v = (axis == 2) ? 1 : 2;
  *n = dims[axis]; *stride = st[axis];
  *du = dims[u]; *su = st[u]; *sv = st[v];
  *nl = dims[u] * dims[v];
}

/* b = B f along an axis: the right-hand side of Eq. (1) / Eq. (2) (App. A.2
 * for the staggered stencils), periodic. */
int orc_stencil_axis(const int64_t dims[3], int axis, int lo, int hi,
                     const double *coef, const double *f, double *out) {
  int64_t n, s, nl, du, su, sv;
  if (axis < 0 || axis > 2 || hi < lo) return ORC_BAD_ARG;
  axis_geometry(dims, axis, &n, &s, &nl, &du, &su, &sv);
  #pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < nl; ++l) {
    const int64_t base = (l % du) * su + (l / du) * sv;
    for (int64_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int q = lo; q <= hi; ++q) {
        const int64_t jj = ((j + q) % n + n) % n;
        acc += coef[q - lo] * f[base + jj * s];
      }
      out[base + j * s] = acc;
    }
  }
  return ORC_OK;
}

/* x = A^{-1} b for every line along an axis (Sec. 5: lines along each index
 * of a 3D array). */
int orc_solve_axis(const int64_t dims[3], int axis, int r, const double *bands,
                   int per_row, int cyclic, const double *b, double *x) {
  int64_t n, s, nl, du, su, sv;
  if (axis < 0 || axis > 2) return ORC_BAD_ARG;
  axis_geometry(dims, axis, &n, &s, &nl, &du, &su, &sv);
  line_op op;
  int st = op_build(&op, r, (int)n, bands, per_row, cyclic);
  if (st) return st;
  int bad = 0;
  #pragma omp parallel reduction(|:bad)
  {
    double tmp[2 * 8 * 8 + 8];
    double *line = (double *)malloc(sizeof(double) * n);
    #pragma omp for schedule(static)
    for (int64_t l = 0; l < nl; ++l) {
      const int64_t base = (l % du) * su + (l / du) * sv;
      for (int64_t j = 0; j < n; ++j) line[j] = b[base + j * s];
      bad |= op_apply(&op, line, line, tmp);
      for (int64_t j = 0; j < n; ++j) x[base + j * s] = line[j];
    }
    free(line);
  }
  op_free(&op);
  return bad ? ORC_SINGULAR : ORC_OK;
}

/* Stencil then solve: the compact derivative / interpolation f -> A^{-1} B f
 * (Eq. (1), Eq. (2)).  `out` must not alias `f`. */
int orc_apply_axis(const int64_t dims[3], int axis, int r, const double *bands,
                   int cyclic, int lo, int hi, const double *coef,
                   const double *f, double *out) {
  int st = orc_stencil_axis(dims, axis, lo, hi, coef, f, out);
  if (st) return st;
  return orc_solve_axis(dims, axis, r, bands, 0, cyclic, out, out);
}

/* Banded matvec y = A x along an axis, A the left-hand side of Eq. (1) /
 * Eq. (2) (used by tests for residuals). */
int orc_matvec_axis(const int64_t dims[3], int axis, int r, const double *bands,
                    int per_row, int cyclic, const double *x, double *y) {
  int64_t n, s, nl, du, su, sv;
  if (axis < 0 || axis > 2) return ORC_BAD_ARG;
  axis_geometry(dims, axis, &n, &s, &nl, &du, &su, &sv);
  #pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < nl; ++l) {
    const int64_t base = (l % du) * su + (l / du) * sv;
    for (int64_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int o = -r; o <= r; ++o) {
        int64_t c = j + o;
        if (!cyclic && (c < 0 || c >= n)) continue;
        c = (c % n + n) % n;
        acc += band_at(bands, per_row, r, (int)j, o) * x[base + c * s];
      }
      y[base + j * s] = acc;
    }
  }
  return ORC_OK;
}

int orc_num_threads(void) {
  int t = 1;
  #pragma omp parallel
  {
    #pragma omp single
    {
#ifdef _OPENMP
      t = omp_get_num_threads();
#endif
    }
  }
  return t;
}
