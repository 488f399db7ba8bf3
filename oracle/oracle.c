/*
 * Plain FP64 CPU oracle (TEST INFRASTRUCTURE: only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark use it).  See oracle.h.
 *
 * Paper: Mueller, Scheichl & Vainikko, arXiv:1402.3545.
 *
 * Everything here follows the plain definitions: A is assembled explicitly in
 * compressed sparse row form, products are row loops, the line solve is the
 * textbook Thomas algorithm applied to the tridiagonal diagonal blocks read out
 * of the CSR rows, and the V-cycle and CG loops are written in the paper's
 * order.  Loops are parallelised with plain OpenMP pragmas only.
 *
 * Discrete operator (volume-integrated cell-centred finite volumes; Sec. 2.1.1
 * "Discretisation" gives the column-block form  (Au)^(T) = A_T u^(T) +
 * sum_{T'} A_TT' u^(T'), Sec. 3.1 "Matrix-free implementation" the tensor-
 * product stencil  A_TT' = alpha_TT' diag(d),  A_T = |T| diag(a) - alpha_T
 * diag(d) + |T| tridiag(-(b+c), b, c)).  With area |T| = hx*hy, dz_k the
 * thickness of layer k and t_k the vertical transmissibility of face k
 * (between layers k-1 and k):
 *
 *   (Au)_{T,k} = |T| [ sigma dz_k u_{T,k} + t_k (u_{T,k} - u_{T,k-1})
 *                                        + t_{k+1} (u_{T,k} - u_{T,k+1}) ]
 *              + dz_k sum_{T'} C_TT' (u_{T,k} - u_{T',k})
 *
 * with u_{T,-1} = u_{T,nz} = 0.  C_TT' is the horizontal face coupling
 * (harmonic mean of K_T, K_T' times the face-length / distance ratio), so
 * a = sigma dz, d = dz, alpha_TT' = -C_TT', alpha_T = sum alpha_TT',
 * b_k = -t_k, c_k = -t_{k+1}.  On a uniform grid with constant K, dividing a
 * row by the cell volume gives the flat-box stencil of Sec. 2.1.1.
 *
 * Horizontal boundaries: doubly periodic, or the homogeneous Dirichlet walls
 * of Sec. 2.1.1.  At a wall the sum over T' includes the wall itself as a
 * neighbour with value 0 and coupling 2 K_T times the face ratio (the wall is
 * half a cell away), and no face crosses the domain edge.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int nx, ny, nz;
  double hx, hy, area;
  double *K;   /* per-column coefficient, j*nx+i */
  double *cx;  /* coupling of face (i+1/2, j): columns (i,j) and (i+1 mod nx, j) */
  double *cy;  /* coupling of face (i, j+1/2): columns (i,j) and (i, j+1 mod ny) */
  int bch;     /* 0 doubly periodic, 1 homogeneous Dirichlet at the four walls */
  double *wall; /* per column: couplings of its wall faces (Dirichlet only) */
  int64_t n;   /* rows */
  int64_t nnz;
  int64_t *rowptr;
  int32_t *col;
  double *val;
  double *u, *f, *r, *t; /* level work vectors for the V-cycle */
} level_t;

struct or_problem {
  int nlevels, bc_h, bc_v, ncoarse, nz;
  double kv, sigma, rho;
  double *zf;    /* nz+1 faces */
  double *dz;    /* nz layer thicknesses */
  double *tf;    /* nz+1 face transmissibilities */
  level_t *lev;
  double *w1, *w2, *w3, *w4, *w5; /* finest-size scratch for the solvers */
};

static __thread char g_err[256];

static void set_err(const char *msg) {
  strncpy(g_err, msg, sizeof(g_err) - 1);
  g_err[sizeof(g_err) - 1] = 0;
}

const char *or_last_error(void) { return g_err; }

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static void *xcalloc(size_t n, size_t sz) {
  void *q = calloc(n ? n : 1, sz);
  return q;
}

static int64_t gidx(const level_t *L, int i, int j, int k) {
  return ((int64_t)j * L->nx + i) * L->nz + k;
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* ---------------------------------------------------------------------------
 * Vertical profiles.  Cell centres zeta_k = (z_k + z_{k+1})/2.  Interior face
 * k (1..nz-1) has transmissibility K_v / (zeta_k - zeta_{k-1}).  A Dirichlet
 * end face sits half a layer from the cell centre: 2 K_v / dz; a Neumann end
 * face carries no flux.
 * ------------------------------------------------------------------------- */
static void build_profiles(or_problem *p) {
  int nz = p->nz;
  for (int k = 0; k < nz; ++k) p->dz[k] = p->zf[k + 1] - p->zf[k];
  for (int k = 1; k < nz; ++k) {
    double zc_lo = 0.5 * (p->zf[k - 1] + p->zf[k]);
    double zc_hi = 0.5 * (p->zf[k] + p->zf[k + 1]);
    p->tf[k] = p->kv / (zc_hi - zc_lo);
  }
  if (p->bc_v == 0) {
    p->tf[0] = 2.0 * p->kv / p->dz[0];
    p->tf[nz] = 2.0 * p->kv / p->dz[nz - 1];
  } else {
    p->tf[0] = 0.0;
    p->tf[nz] = 0.0;
  }
}

/* Face couplings of one level from its per-column K: harmonic mean per face,
 * computed once per face so that A is exactly symmetric.  With Dirichlet
 * walls (the paper's horizontal boundary condition, Sec. 2.1.1) the faces
 * across the domain edge do not exist; a wall face lies half a cell from the
 * column centre and couples the column to the zero boundary value with
 * 2 K_T (face length over half the spacing), which only enters the diagonal. */
static void build_faces(level_t *L) {
  int nx = L->nx, ny = L->ny;
  double fx = L->hy / L->hx, fy = L->hx / L->hy;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int64_t c = (int64_t)j * nx + i;
      double kc = L->K[c];
      double ke = L->K[(int64_t)j * nx + wrap(i + 1, nx)];
      double kn = L->K[(int64_t)wrap(j + 1, ny) * nx + i];
      L->cx[c] = fx * 2.0 * kc * ke / (kc + ke);
      L->cy[c] = fy * 2.0 * kc * kn / (kc + kn);
      L->wall[c] = 0.0;
      if (L->bch) {
        if (i == nx - 1) L->cx[c] = 0.0;
        if (j == ny - 1) L->cy[c] = 0.0;
        if (i == 0) L->wall[c] += fx * 2.0 * kc;
        if (i == nx - 1) L->wall[c] += fx * 2.0 * kc;
        if (j == 0) L->wall[c] += fy * 2.0 * kc;
        if (j == ny - 1) L->wall[c] += fy * 2.0 * kc;
      }
    }
}

/* Insert (c, v) into a row buffer, merging duplicate column indices. */
static int row_add(int32_t *cols, double *vals, int n, int32_t c, double v) {
  for (int q = 0; q < n; ++q)
    if (cols[q] == c) {
      vals[q] += v;
      return n;
    }
  cols[n] = c;
  vals[n] = v;
  return n + 1;
}

static void row_sort(int32_t *cols, double *vals, int n) {
  for (int a = 1; a < n; ++a) {
    int32_t c = cols[a];
    double v = vals[a];
    int b = a - 1;
    while (b >= 0 && cols[b] > c) {
      cols[b + 1] = cols[b];
      vals[b + 1] = vals[b];
      --b;
    }
    cols[b + 1] = c;
    vals[b + 1] = v;
  }
}

/* Assemble one row (T,k) of A: returns the number of entries. */
static int assemble_row(const or_problem *p, const level_t *L, int i, int j, int k,
                        int32_t *cols, double *vals) {
  int nx = L->nx, ny = L->ny, nz = L->nz;
  const double *dz = p->dz, *tf = p->tf;
  int64_t g = gidx(L, i, j, k);
  int n = 0;
  int iw = wrap(i - 1, nx), ie = wrap(i + 1, nx);
  int js = wrap(j - 1, ny), jn = wrap(j + 1, ny);
  double ce = L->cx[(int64_t)j * nx + i], cw = L->cx[(int64_t)j * nx + iw];
  double cn = L->cy[(int64_t)j * nx + i], cs = L->cy[(int64_t)js * nx + i];
  double wall = L->wall[(int64_t)j * nx + i];
  /* diagonal: zero-order term, both vertical faces, the four horizontal faces
   * (wall faces included) */
  double diag = L->area * (p->sigma * dz[k] + tf[k] + tf[k + 1]) +
                dz[k] * (ce + cw + cn + cs + wall);
  n = row_add(cols, vals, n, (int32_t)g, diag);
  if (k > 0) n = row_add(cols, vals, n, (int32_t)(g - 1), -L->area * tf[k]);
  if (k < nz - 1) n = row_add(cols, vals, n, (int32_t)(g + 1), -L->area * tf[k + 1]);
  /* faces across a Dirichlet wall have zero coupling and no entry */
  if (ce != 0.0) n = row_add(cols, vals, n, (int32_t)gidx(L, ie, j, k), -dz[k] * ce);
  if (cw != 0.0) n = row_add(cols, vals, n, (int32_t)gidx(L, iw, j, k), -dz[k] * cw);
  if (cn != 0.0) n = row_add(cols, vals, n, (int32_t)gidx(L, i, jn, k), -dz[k] * cn);
  if (cs != 0.0) n = row_add(cols, vals, n, (int32_t)gidx(L, i, js, k), -dz[k] * cs);
  row_sort(cols, vals, n);
  return n;
}

static int assemble_level(const or_problem *p, level_t *L) {
  int64_t n = L->n;
  L->rowptr = (int64_t *)xcalloc((size_t)n + 1, sizeof(int64_t));
  if (!L->rowptr) return -1;
  /* pass 1: row lengths */
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    int32_t cols[8];
    double vals[8];
    int k = (int)(g % L->nz);
    int64_t col = g / L->nz;
    int i = (int)(col % L->nx), j = (int)(col / L->nx);
    L->rowptr[g + 1] = assemble_row(p, L, i, j, k, cols, vals);
  }
  for (int64_t g = 0; g < n; ++g) L->rowptr[g + 1] += L->rowptr[g];
  L->nnz = L->rowptr[n];
  L->col = (int32_t *)xcalloc((size_t)L->nnz, sizeof(int32_t));
  L->val = (double *)xcalloc((size_t)L->nnz, sizeof(double));
  if (!L->col || !L->val) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    int32_t cols[8];
    double vals[8];
    int k = (int)(g % L->nz);
    int64_t col = g / L->nz;
    int i = (int)(col % L->nx), j = (int)(col / L->nx);
    int m = assemble_row(p, L, i, j, k, cols, vals);
    memcpy(L->col + L->rowptr[g], cols, (size_t)m * sizeof(int32_t));
    memcpy(L->val + L->rowptr[g], vals, (size_t)m * sizeof(double));
  }
  return 0;
}

void or_destroy(or_problem *p) {
  if (!p) return;
  if (p->lev)
    for (int d = 0; d < p->nlevels; ++d) {
      level_t *L = &p->lev[d];
      free(L->K); free(L->cx); free(L->cy); free(L->wall);
      free(L->rowptr); free(L->col); free(L->val);
      free(L->u); free(L->f); free(L->r); free(L->t);
    }
  free(p->lev);
  free(p->zf); free(p->dz); free(p->tf);
  free(p->w1); free(p->w2); free(p->w3); free(p->w4); free(p->w5);
  free(p);
}

static or_problem *create(int nx, int ny, int nz, int nlevels, int bc_h, int bc_v, double kv,
                          double sigma, const double *zfaces, const double *kh, double rho,
                          int ncoarse, int assemble) {
  if (nx < 2 || ny < 2 || nz < 2 || nlevels < 1) {
    set_err("need nx, ny, nz >= 2 and nlevels >= 1");
    return NULL;
  }
  if (bc_h != 0 && bc_h != 1) { set_err("bc_h must be 0 or 1"); return NULL; }
  if (bc_v != 0 && bc_v != 1) { set_err("bc_v must be 0 or 1"); return NULL; }
  if (!(sigma > 0.0) || !(kv >= 0.0)) { set_err("need sigma > 0, kv >= 0"); return NULL; }
  if (ncoarse < 1) { set_err("ncoarse >= 1"); return NULL; }
  int div = 1 << (nlevels - 1);
  if (nx % div || ny % div) {
    set_err("nx, ny must be divisible by 2^(nlevels-1)");
    return NULL;
  }
  if ((int64_t)nx * ny * nz > INT32_MAX) {
    set_err("too many rows for int32 column indices");
    return NULL;
  }
  or_problem *p = (or_problem *)xcalloc(1, sizeof(or_problem));
  p->nlevels = nlevels; p->bc_h = bc_h; p->bc_v = bc_v; p->ncoarse = ncoarse;
  p->nz = nz; p->kv = kv; p->sigma = sigma; p->rho = rho;
  p->zf = (double *)xcalloc((size_t)nz + 1, sizeof(double));
  p->dz = (double *)xcalloc((size_t)nz, sizeof(double));
  p->tf = (double *)xcalloc((size_t)nz + 1, sizeof(double));
  for (int k = 0; k <= nz; ++k)
    p->zf[k] = zfaces ? zfaces[k] : ((double)k / nz) * ((double)k / nz);
  for (int k = 0; k < nz; ++k)
    if (!(p->zf[k + 1] > p->zf[k])) {
      set_err("zfaces must be strictly increasing");
      or_destroy(p);
      return NULL;
    }
  build_profiles(p);
  p->lev = (level_t *)xcalloc((size_t)nlevels, sizeof(level_t));
  for (int d = 0; d < nlevels; ++d) {
    level_t *L = &p->lev[d];
    L->nx = nx >> d; L->ny = ny >> d; L->nz = nz;
    L->hx = 1.0 / L->nx; L->hy = 1.0 / L->ny;
    L->area = L->hx * L->hy;
    int64_t nc = (int64_t)L->nx * L->ny;
    L->n = nc * nz;
    L->K = (double *)xcalloc((size_t)nc, sizeof(double));
    L->cx = (double *)xcalloc((size_t)nc, sizeof(double));
    L->cy = (double *)xcalloc((size_t)nc, sizeof(double));
    L->wall = (double *)xcalloc((size_t)nc, sizeof(double));
    L->bch = bc_h;
    if (d == 0) {
      for (int64_t c = 0; c < nc; ++c) {
        L->K[c] = kh ? kh[c] : 1.0;
        if (!(L->K[c] > 0.0)) {
          set_err("kh must be positive");
          or_destroy(p);
          return NULL;
        }
      }
    } else {
      /* coarse coefficient: mean of the four children (the stencil is
       * rediscretised per level, Sec. 3.1: alpha depends on the level) */
      const level_t *F = &p->lev[d - 1];
      for (int J = 0; J < L->ny; ++J)
        for (int I = 0; I < L->nx; ++I) {
          double s = F->K[(int64_t)(2 * J) * F->nx + 2 * I] +
                     F->K[(int64_t)(2 * J) * F->nx + 2 * I + 1] +
                     F->K[(int64_t)(2 * J + 1) * F->nx + 2 * I] +
                     F->K[(int64_t)(2 * J + 1) * F->nx + 2 * I + 1];
          L->K[(int64_t)J * L->nx + I] = 0.25 * s;
        }
    }
    build_faces(L);
    if (!assemble) continue;
    if (assemble_level(p, L)) {
      set_err("out of memory assembling CSR");
      or_destroy(p);
      return NULL;
    }
    if (d > 0) {
      L->u = (double *)xcalloc((size_t)L->n, sizeof(double));
      L->f = (double *)xcalloc((size_t)L->n, sizeof(double));
    }
    L->r = (double *)xcalloc((size_t)L->n, sizeof(double));
    L->t = (double *)xcalloc((size_t)L->n, sizeof(double));
  }
  if (!assemble) return p;
  int64_t n0 = p->lev[0].n;
  p->w1 = (double *)xcalloc((size_t)n0, sizeof(double));
  p->w2 = (double *)xcalloc((size_t)n0, sizeof(double));
  p->w3 = (double *)xcalloc((size_t)n0, sizeof(double));
  p->w4 = (double *)xcalloc((size_t)n0, sizeof(double));
  p->w5 = (double *)xcalloc((size_t)n0, sizeof(double));
  if (!p->w5) {
    set_err("out of memory");
    or_destroy(p);
    return NULL;
  }
  return p;
}

or_problem *or_create(int nx, int ny, int nz, int nlevels, int bc_h, int bc_v, double kv,
                      double sigma, const double *zfaces, const double *kh, double rho,
                      int ncoarse) {
  return create(nx, ny, nz, nlevels, bc_h, bc_v, kv, sigma, zfaces, kh, rho, ncoarse, 1);
}

/* Same hierarchy without the CSR matrices: only the row-wise functions below
 * (and restriction / prolongation) are available.  For grids too large to
 * assemble, to check sampled rows and columns and full residual norms. */
or_problem *or_create_matfree(int nx, int ny, int nz, int nlevels, int bc_h, int bc_v, double kv,
                              double sigma, const double *zfaces, const double *kh, double rho,
                              int ncoarse) {
  return create(nx, ny, nz, nlevels, bc_h, bc_v, kv, sigma, zfaces, kh, rho, ncoarse, 0);
}

static int bad_depth(const or_problem *p, int d) {
  if (!p || d < 0 || d >= p->nlevels) {
    set_err("bad level");
    return 1;
  }
  return 0;
}

static int no_csr(const or_problem *p, int d) {
  if (!p->lev[d].rowptr) {
    set_err("this problem was created without CSR matrices");
    return 1;
  }
  return 0;
}

int or_shape(const or_problem *p, int d, int *nx, int *ny, int *nz) {
  if (bad_depth(p, d)) return -1;
  *nx = p->lev[d].nx; *ny = p->lev[d].ny; *nz = p->lev[d].nz;
  return 0;
}

int64_t or_nnz(const or_problem *p, int d) {
  if (bad_depth(p, d)) return -1;
  return p->lev[d].nnz;
}

int or_csr(const or_problem *p, int d, int64_t *rowptr, int32_t *col, double *val) {
  if (bad_depth(p, d) || no_csr(p, d)) return -1;
  const level_t *L = &p->lev[d];
  memcpy(rowptr, L->rowptr, (size_t)(L->n + 1) * sizeof(int64_t));
  memcpy(col, L->col, (size_t)L->nnz * sizeof(int32_t));
  memcpy(val, L->val, (size_t)L->nnz * sizeof(double));
  return 0;
}

int or_profiles(const or_problem *p, double *dz, double *tface) {
  memcpy(dz, p->dz, (size_t)p->nz * sizeof(double));
  memcpy(tface, p->tf, (size_t)(p->nz + 1) * sizeof(double));
  return 0;
}

int or_faces(const or_problem *p, int d, double *kcol, double *cx, double *cy) {
  if (bad_depth(p, d)) return -1;
  const level_t *L = &p->lev[d];
  size_t nc = (size_t)L->nx * L->ny;
  memcpy(kcol, L->K, nc * sizeof(double));
  memcpy(cx, L->cx, nc * sizeof(double));
  memcpy(cy, L->cy, nc * sizeof(double));
  return 0;
}

int or_walls(const or_problem *p, int d, double *wall) {
  if (bad_depth(p, d)) return -1;
  const level_t *L = &p->lev[d];
  memcpy(wall, L->wall, (size_t)L->nx * L->ny * sizeof(double));
  return 0;
}

/* ---------------------------------------------------------------------------
 * Level-1 operations
 * ------------------------------------------------------------------------- */
double or_dot(int64_t n, const double *x, const double *y) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t g = 0; g < n; ++g) s += x[g] * y[g];
  return s;
}

static double nrm2(int64_t n, const double *x) { return sqrt(or_dot(n, x, x)); }

/* y = A x, a plain CSR row loop (the SpMV of Sec. 2.2) */
static void csr_mv(const level_t *L, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < L->n; ++g) {
    double s = 0.0;
    for (int64_t q = L->rowptr[g]; q < L->rowptr[g + 1]; ++q) s += L->val[q] * x[L->col[q]];
    y[g] = s;
  }
}

int or_spmv(const or_problem *p, int d, const double *x, double *y) {
  if (bad_depth(p, d) || no_csr(p, d)) return -1;
  csr_mv(&p->lev[d], x, y);
  return 0;
}

static void residual(const level_t *L, const double *f, const double *u, double *r) {
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < L->n; ++g) {
    double s = 0.0;
    for (int64_t q = L->rowptr[g]; q < L->rowptr[g + 1]; ++q) s += L->val[q] * u[L->col[q]];
    r[g] = f[g] - s;
  }
}

int or_residual(const or_problem *p, int d, const double *f, const double *u, double *r) {
  if (bad_depth(p, d) || no_csr(p, d)) return -1;
  residual(&p->lev[d], f, u, r);
  return 0;
}

/* Entry (row, c) of the CSR matrix, 0 if absent. */
static double csr_entry(const level_t *L, int64_t row, int64_t c) {
  for (int64_t q = L->rowptr[row]; q < L->rowptr[row + 1]; ++q)
    if (L->col[q] == c) return L->val[q];
  return 0.0;
}

/* z = M^{-1} r with M = blockdiag(A_T), the vertical line relaxation of
 * Sec. 2.2.  Each diagonal block is tridiagonal (sub b, diagonal a, super c
 * read out of the CSR rows) and is solved by the textbook Thomas algorithm:
 * forward elimination, then back substitution, no pivoting. */
static void line_solve(const level_t *L, const double *r, double *z) {
  int nz = L->nz;
  int64_t ncol = (int64_t)L->nx * L->ny;
#pragma omp parallel
  {
    double *cp = (double *)malloc((size_t)nz * sizeof(double));
    double *dp = (double *)malloc((size_t)nz * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
      int64_t g0 = c * nz;
      for (int k = 0; k < nz; ++k) {
        int64_t g = g0 + k;
        double a = k > 0 ? csr_entry(L, g, g - 1) : 0.0;
        double b = csr_entry(L, g, g);
        double cc = k < nz - 1 ? csr_entry(L, g, g + 1) : 0.0;
        if (k == 0) {
          cp[0] = cc / b;
          dp[0] = r[g] / b;
        } else {
          double m = b - a * cp[k - 1];
          cp[k] = cc / m;
          dp[k] = (r[g] - a * dp[k - 1]) / m;
        }
      }
      z[g0 + nz - 1] = dp[nz - 1];
      for (int k = nz - 2; k >= 0; --k) z[g0 + k] = dp[k] - cp[k] * z[g0 + k + 1];
    }
    free(cp);
    free(dp);
  }
}

int or_line_solve(const or_problem *p, int d, const double *r, double *z) {
  if (bad_depth(p, d) || no_csr(p, d)) return -1;
  line_solve(&p->lev[d], r, z);
  return 0;
}

/* Block-Jacobi smoother, Sec. 2.2: u <- u + rho M^{-1} (f - A u). */
static void smooth(const level_t *L, const double *f, double *u, double rho, double *r,
                   double *z) {
  residual(L, f, u, r);
  line_solve(L, r, z);
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < L->n; ++g) u[g] += rho * z[g];
}

int or_smooth(or_problem *p, int d, const double *f, double *u, double rho) {
  if (bad_depth(p, d) || no_csr(p, d)) return -1;
  level_t *L = &p->lev[d];
  smooth(L, f, u, rho, L->r, L->t);
  return 0;
}

/* Restriction: the cell average of the residual density, which for the
 * volume-integrated residual is the sum over the four horizontal children
 * (horizontal-only semicoarsening, Sec. 2.2). */
static void restrict_sum(const level_t *F, const level_t *C, const double *rf, double *fc) {
  int nz = C->nz;
#pragma omp parallel for schedule(static)
  for (int64_t cc = 0; cc < (int64_t)C->nx * C->ny; ++cc) {
    int I = (int)(cc % C->nx), J = (int)(cc / C->nx);
    for (int k = 0; k < nz; ++k) {
      double s = rf[gidx(F, 2 * I, 2 * J, k)] + rf[gidx(F, 2 * I + 1, 2 * J, k)] +
                 rf[gidx(F, 2 * I, 2 * J + 1, k)] + rf[gidx(F, 2 * I + 1, 2 * J + 1, k)];
      fc[gidx(C, I, J, k)] = s;
    }
  }
}

int or_restrict(const or_problem *p, int dfine, const double *rf, double *fc) {
  if (bad_depth(p, dfine) || bad_depth(p, dfine + 1)) return -1;
  restrict_sum(&p->lev[dfine], &p->lev[dfine + 1], rf, fc);
  return 0;
}

/* Prolongation: cell-centred bilinear interpolation in the horizontal only
 * (Sec. 2.2, "(piecewise) linear").  Fine child (2I+a, 2J+b) takes weights
 * 9/16, 3/16, 3/16, 1/16 from its coarse parent, the parent's neighbour on
 * its side in x, in y, and the diagonal one; periodic wrap.  Behind a
 * Dirichlet wall the missing coarse cell is the mirror image of the parent
 * with opposite sign (the linear interpolant that vanishes on the wall). */
static void prolongate_add(const level_t *C, const level_t *F, const double *uc, double *uf) {
  int nz = F->nz;
#pragma omp parallel for schedule(static)
  for (int64_t fc = 0; fc < (int64_t)F->nx * F->ny; ++fc) {
    int i = (int)(fc % F->nx), j = (int)(fc / F->nx);
    int I = i / 2, J = j / 2;
    int I2 = I + ((i & 1) ? 1 : -1);
    int J2 = J + ((j & 1) ? 1 : -1);
    double sx = 1.0, sy = 1.0;
    if (C->bch) {
      if (I2 < 0 || I2 >= C->nx) { I2 = I; sx = -1.0; }
      if (J2 < 0 || J2 >= C->ny) { J2 = J; sy = -1.0; }
    } else {
      I2 = wrap(I2, C->nx);
      J2 = wrap(J2, C->ny);
    }
    for (int k = 0; k < nz; ++k) {
      double v = 9.0 * uc[gidx(C, I, J, k)] + 3.0 * sx * uc[gidx(C, I2, J, k)] +
                 3.0 * sy * uc[gidx(C, I, J2, k)] + sx * sy * uc[gidx(C, I2, J2, k)];
      uf[gidx(F, i, j, k)] += v / 16.0;
    }
  }
}

int or_prolongate_add(const or_problem *p, int dcoarse, const double *uc, double *uf) {
  if (bad_depth(p, dcoarse) || bad_depth(p, dcoarse - 1)) return -1;
  prolongate_add(&p->lev[dcoarse], &p->lev[dcoarse - 1], uc, uf);
  return 0;
}

/* RestrictSmooth (Sec. 3.1): f_c <- R r_f, then one smoothing step from a
 * zero initial guess, u_c <- rho M^{-1} f_c. */
static void restrict_smooth(const level_t *F, const level_t *C, const double *rf, double *fc,
                            double *uc, double rho) {
  restrict_sum(F, C, rf, fc);
  line_solve(C, fc, uc);
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < C->n; ++g) uc[g] *= rho;
}

int or_restrict_smooth(or_problem *p, int dc, const double *rf, double *fc, double *uc,
                       double rho) {
  if (bad_depth(p, dc) || bad_depth(p, dc - 1) || no_csr(p, dc)) return -1;
  restrict_smooth(&p->lev[dc - 1], &p->lev[dc], rf, fc, uc, rho);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Algorithm 1 (VCycle), one pre- and one post-smoothing step.  Depth d = 0 is
 * the finest level.  On the coarsest level the exact solve is replaced by the
 * restriction-smoothing step plus (ncoarse - 1) further smoothing steps
 * (Sec. 2.2: two smoother iterations suffice on the coarsest grid).  With a
 * single level the cycle is ncoarse smoothing steps.
 * ------------------------------------------------------------------------- */
static void vcycle(or_problem *p, int d, const double *f, double *u) {
  level_t *L = &p->lev[d];
  double rho = p->rho;
  if (d == p->nlevels - 1) {
    if (d == 0) {
      for (int s = 0; s < p->ncoarse; ++s) smooth(L, f, u, rho, L->r, L->t);
      return;
    }
    restrict_smooth(&p->lev[d - 1], L, p->lev[d - 1].r, L->f, L->u, rho);
    for (int s = 1; s < p->ncoarse; ++s) smooth(L, L->f, L->u, rho, L->r, L->t);
    return;
  }
  if (d == 0) {
    smooth(L, f, u, rho, L->r, L->t);
  } else {
    restrict_smooth(&p->lev[d - 1], L, p->lev[d - 1].r, L->f, L->u, rho);
    f = L->f;
    u = L->u;
  }
  residual(L, f, u, L->r);
  vcycle(p, d + 1, NULL, NULL);
  prolongate_add(&p->lev[d + 1], L, p->lev[d + 1].u, u);
  smooth(L, f, u, rho, L->r, L->t);
}

int or_vcycle(or_problem *p, const double *f, double *u) {
  if (!p || no_csr(p, 0)) return -1;
  vcycle(p, 0, f, u);
  return 0;
}

/* Multigrid iteration: repeated V-cycles until ||f - Au|| / ||f - Au_0|| < rtol
 * (Sec. 2.2, convergence test after each V-cycle).  history[it] holds the
 * relative residual after `it` cycles (history[0] = 1).  Returns 0 when
 * converged, 1 when maxit was reached. */
int or_mg_solve(or_problem *p, const double *f, double *u, double rtol, int maxit, int *iters,
                double *history) {
  if (!p || rtol <= 0.0 || maxit < 0) { set_err("bad arguments"); return -1; }
  if (no_csr(p, 0)) return -1;
  level_t *L = &p->lev[0];
  residual(L, f, u, p->w1);
  double r0 = nrm2(L->n, p->w1);
  if (history) history[0] = 1.0;
  *iters = 0;
  if (r0 == 0.0) return 0;
  for (int it = 1; it <= maxit; ++it) {
    vcycle(p, 0, f, u);
    residual(L, f, u, p->w1);
    double rr = nrm2(L->n, p->w1) / r0;
    if (history) history[it] = rr;
    *iters = it;
    if (!(rr == rr)) return 2;
    if (rr < rtol) return 0;
  }
  return 1;
}

/* Preconditioned CG (textbook form, e.g. Saad, Iterative Methods for Sparse
 * Linear Systems, Alg. 9.1) with the line preconditioner M.  Stops when the
 * recursively updated residual satisfies ||r_i|| / ||r_0|| < rtol; the true
 * relative residual at exit goes to *relres_true.  history[it] holds the
 * recursive relative residual after `it` iterations. */
int or_pcg_solve(or_problem *p, const double *f, double *u, double rtol, int maxit, int *iters,
                 double *history, double *relres_true) {
  if (!p || rtol <= 0.0 || maxit < 0) { set_err("bad arguments"); return -1; }
  if (no_csr(p, 0)) return -1;
  level_t *L = &p->lev[0];
  int64_t n = L->n;
  double *r = p->w1, *z = p->w2, *pp = p->w3, *q = p->w4;
  residual(L, f, u, r);
  double r0 = nrm2(n, r);
  if (history) history[0] = 1.0;
  *iters = 0;
  if (relres_true) *relres_true = 0.0;
  if (r0 == 0.0) return 0;
  line_solve(L, r, z);
  memcpy(pp, z, (size_t)n * sizeof(double));
  double rz = or_dot(n, r, z);
  int status = 1;
  for (int it = 1; it <= maxit; ++it) {
    csr_mv(L, pp, q);
    double alpha = rz / or_dot(n, pp, q);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
      u[g] += alpha * pp[g];
      r[g] -= alpha * q[g];
    }
    double rr = nrm2(n, r) / r0;
    if (history) history[it] = rr;
    *iters = it;
    if (!(rr == rr)) { status = 2; break; }
    if (rr < rtol) { status = 0; break; }
    line_solve(L, r, z);
    double rz_new = or_dot(n, r, z);
    double beta = rz_new / rz;
    rz = rz_new;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) pp[g] = z[g] + beta * pp[g];
  }
  if (relres_true) {
    residual(L, f, u, p->w5);
    *relres_true = nrm2(n, p->w5) / r0;
  }
  return status;
}

/* ---------------------------------------------------------------------------
 * Row-wise forms of the same definitions (no stored matrix): each row comes
 * from assemble_row, the routine that also fills the CSR arrays.
 * ------------------------------------------------------------------------- */
static void decode(const level_t *L, int64_t g, int *i, int *j, int *k) {
  *k = (int)(g % L->nz);
  int64_t c = g / L->nz;
  *i = (int)(c % L->nx);
  *j = (int)(c / L->nx);
}

/* y[q] = (A x)_{rows[q]} */
int or_apply_rows(const or_problem *p, int d, int64_t nrows, const int64_t *rows,
                  const double *x, double *y) {
  if (bad_depth(p, d)) return -1;
  const level_t *L = &p->lev[d];
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nrows; ++q) {
    int32_t cols[8];
    double vals[8];
    int i, j, k;
    decode(L, rows[q], &i, &j, &k);
    int m = assemble_row(p, L, i, j, k, cols, vals);
    double s = 0.0;
    for (int e = 0; e < m; ++e) s += vals[e] * x[cols[e]];
    y[q] = s;
  }
  return 0;
}

/* ||f - A u||_2^2 over all rows of level d */
double or_residual_norm2_rows(const or_problem *p, int d, const double *f, const double *u) {
  if (bad_depth(p, d)) return -1.0;
  const level_t *L = &p->lev[d];
  double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
  for (int64_t g = 0; g < L->n; ++g) {
    int32_t cols[8];
    double vals[8];
    int i, j, k;
    decode(L, g, &i, &j, &k);
    int m = assemble_row(p, L, i, j, k, cols, vals);
    double s = 0.0;
    for (int e = 0; e < m; ++e) s += vals[e] * u[cols[e]];
    double r = f[g] - s;
    acc += r * r;
  }
  return acc;
}

/* z = M^{-1} r on the listed columns (index j*nx+i) only: textbook Thomas on
 * the tridiagonal block of each column, read out of its assembled rows. */
int or_line_solve_columns(const or_problem *p, int d, int64_t ncols, const int64_t *colidx,
                          const double *r, double *z) {
  if (bad_depth(p, d)) return -1;
  const level_t *L = &p->lev[d];
  int nz = L->nz;
#pragma omp parallel
  {
    double *cp = (double *)malloc((size_t)nz * sizeof(double));
    double *dp = (double *)malloc((size_t)nz * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t q = 0; q < ncols; ++q) {
      int64_t c = colidx[q];
      int i = (int)(c % L->nx), j = (int)(c / L->nx);
      int64_t g0 = c * nz;
      for (int k = 0; k < nz; ++k) {
        int32_t cols[8];
        double vals[8];
        int m = assemble_row(p, L, i, j, k, cols, vals);
        int64_t g = g0 + k;
        double a = 0.0, b = 0.0, cc = 0.0;
        for (int e = 0; e < m; ++e) {
          if (cols[e] == g - 1) a = vals[e];
          else if (cols[e] == g) b = vals[e];
          else if (cols[e] == g + 1) cc = vals[e];
        }
        if (k == 0) {
          cp[0] = cc / b;
          dp[0] = r[g] / b;
        } else {
          double piv = b - a * cp[k - 1];
          cp[k] = cc / piv;
          dp[k] = (r[g] - a * dp[k - 1]) / piv;
        }
      }
      z[g0 + nz - 1] = dp[nz - 1];
      for (int k = nz - 2; k >= 0; --k) z[g0 + k] = dp[k] - cp[k] * z[g0 + k + 1];
    }
    free(cp);
    free(dp);
  }
  return 0;
}
