/*
 * FP64 CPU oracle of the multi-resolution SPH method for fluid-structure
 * interaction of Zhang, Rezavand & Hu (arXiv:1911.13255).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the GPU
 * library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.  It
 * shares no code, header or table with the GPU library.
 *
 * Everything is double precision.  Every neighbour sum runs over a neighbour
 * list kept in ascending original-index order (fluid, then walls, then solid),
 * with one OpenMP thread per particle and no reordering inside a sum.
 *
 * Readings of the paper where it is silent or garbled (numbered R1-R34 in the
 * design notes) are marked "reading" below.  Functions with no independent
 * check are marked "parity unpinned"; there are none at present: besides the
 * invariants (rigid motions, momentum exchange, hydrostatics), the magnitude
 * of every pair sum (continuity, pressure and viscous terms, the wall and
 * solid coupling terms, the solid stress divergence) is pinned to a closed
 * form on a lattice by the tests.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
  int dim, n_fluid, n_wall, n_solid, n_clamp;
  double dp_f, dp_s, h_ratio;
  double rho0_f, c_f, eta, gamma, g[3];
  double rho0_s, E, nu;
  double cfl_ac, cfl_ad, cfl_s, u_ref;
  double lo[3], hi[3];
  int periodic[3];
  double hydro_H;
  double inflow_U0, inflow_ts, inflow_H, inflow_len;
  const double *x_fluid, *v_fluid, *x_wall, *nrm_wall, *x_solid, *v_solid;
  int riemann, density_reinit;
  int material;    /* 0 Neo-Hookean, 1 linear elastic (Saint Venant-Kirchhoff) */
  int single_step; /* 1: the solid step is the one step of fluid and solid (kappa = 1) */
  int velocity_verlet; /* test contrast: 1 velocity-based Verlet instead of position-based */
} ora_scene;

typedef struct {
  int d, nf, nw, ns, nc;
  double dpf, dps, hf, hs;
  double rho0, c, eta, gam, g[3];
  double rho0s, E, nu, K, mu, lam, cs;
  double cfl_ac, cfl_ad, cfl_s, uref;
  double lo[3], hi[3], L[3];
  int per[3];
  double hydroH, inU0, ints, inH, inlen;
  int riemann, reinit, material, single, vv;
  double psi0;
  /* fluid, n x 3 vectors */
  double *x, *v, *rho, *drho, *m, *a, *p, *xr;
  double *sn_rho, *sn_p, *sn_v; /* mid-state snapshot used by the coupling on the solid */
  /* walls */
  double *xw, *wn;
  /* solid: 3 x 3 row-major tensors, 3-vectors */
  double *x0, *u, *vs, *as, *F, *dF, *B, *n0, *sn, *vbar, *abar, *fF, *xsr, *ms, *V0;
  double *fFp; /* pressure part of the coupling force on the solid */
  int *clamp;
  int *s_start, *s_idx;
  double *s_grad; /* grad_a W(r0_ab, h_s) for each reference pair */
  /* neighbour lists at the last rebuild */
  int *ff_start, *ff_idx, *fb_start, *fb_idx, *sf_start, *sf_idx;
  /* time */
  double t, dt_ac, dt_ad, dt_s, adv_accum;
  int kappa, need_rebuild;
  /* counters */
  long long n_ff, n_fb, n_sf, n_ss, steps, rebuilds, substeps, interactions;
} ora_ctx;

/* ------------------------------------------------------------------ helpers */

static double dot(int d, const double *a, const double *b) {
  double s = 0.0;
  for (int k = 0; k < d; ++k) s += a[k] * b[k];
  return s;
}

static double norm(int d, const double *a) { return sqrt(dot(d, a, a)); }

static void mat_eye(double *A) {
  memset(A, 0, 9 * sizeof(double));
  A[0] = A[4] = A[8] = 1.0;
}

/* C = A B on the leading d x d block of 3 x 3 row-major storage */
static void mat_mul(int d, const double *A, const double *B, double *C) {
  double T[9] = {0};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += A[3 * i + k] * B[3 * k + j];
      T[3 * i + j] = s;
    }
  memcpy(C, T, sizeof T);
}

static void mat_transpose(int d, const double *A, double *T) {
  double R[9] = {0};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) R[3 * i + j] = A[3 * j + i];
  memcpy(T, R, sizeof R);
}

static double mat_det(int d, const double *A) {
  if (d == 2) return A[0] * A[4] - A[1] * A[3];
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse by the adjugate; returns the determinant */
static double mat_inv(int d, const double *A, double *Ai) {
  double det = mat_det(d, A);
  double R[9] = {0};
  if (d == 2) {
    R[0] = A[4] / det;
    R[1] = -A[1] / det;
    R[3] = -A[3] / det;
    R[4] = A[0] / det;
  } else {
    R[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    R[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    R[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    R[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    R[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    R[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    R[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    R[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    R[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  }
  memcpy(Ai, R, sizeof R);
  return det;
}

/* ---------------------------------------------------- kernel (Section 4 preamble)
 * Reading: the "5th-order Wendland" kernel is Wendland C2 with support 2h,
 *   W(r, h) = alpha_d (1 - q/2)^4 (1 + 2q),  q = r/h < 2,
 *   alpha_2 = 7 / (4 pi h^2),  alpha_3 = 21 / (16 pi h^3).
 * The gradient is grad_i W_ij = e_ij dW/dr with e_ij = (r_i - r_j)/|r_ij|
 * (Section 2.2 prints an extra 1/r_ij, which is not dimensionally consistent). */
double ora_kernel_W(int d, double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double alpha = (d == 2) ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
  double t = 1.0 - 0.5 * q;
  return alpha * t * t * t * t * (1.0 + 2.0 * q);
}

double ora_kernel_dW(int d, double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double alpha = (d == 2) ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
  double t = 1.0 - 0.5 * q;
  return -5.0 * alpha * q * t * t * t / h;
}

/* ----------------------------------------------------- equation of state
 * Tait equation (Section 2.1): p = rho0 c^2 / gamma ((rho/rho0)^gamma - 1).
 * Inverse (used for the imaginary density of a wall or solid particle):
 *   rho = rho0 (1 + gamma p / (rho0 c^2))^(1/gamma); reading: the bracket is
 *   clipped at 0 so that a tension below -rho0 c^2 / gamma gives rho = 0. */
double ora_eos(double rho, double rho0, double c, double gam) {
  return rho0 * c * c / gam * (pow(rho / rho0, gam) - 1.0);
}

double ora_eos_inv(double p, double rho0, double c, double gam) {
  double s = 1.0 + gam * p / (rho0 * c * c);
  if (s < 0.0) s = 0.0;
  return rho0 * pow(s, 1.0 / gam);
}

/* ----------------------------------------------------- inter-particle Riemann problem
 * Section 2.2 names a low-dissipation Riemann solver without giving it; reading:
 * a linearised acoustic solver along the pair axis with a limited dissipation.
 * Left state i, right state j, e = e_ij:
 *   U_L = -v_i.e, U_R = -v_j.e, rho_bar = (rho_i + rho_j)/2, c_bar = c,
 *   U* = (U_L + U_R)/2 + (p_i - p_j) / (2 rho_bar c_bar),
 *   P* = (p_i + p_j)/2 + rho_bar beta (U_L - U_R)/2,  beta = min(3 max(U_L - U_R, 0), c_bar),
 *   v* = (v_i + v_j)/2 - (U* - (U_L + U_R)/2) e.
 * With riemann = 0 the simple averages P* = (p_i + p_j)/2, v* = (v_i + v_j)/2 are used. */
void ora_riemann(int d, int use_riemann, double c, double rho_i, double rho_j, double p_i,
                 double p_j, const double *vi, const double *vj, const double *e,
                 double *Pstar, double *vstar) {
  if (!use_riemann) {
    *Pstar = 0.5 * (p_i + p_j);
    for (int k = 0; k < d; ++k) vstar[k] = 0.5 * (vi[k] + vj[k]);
    return;
  }
  double UL = -dot(d, vi, e), UR = -dot(d, vj, e);
  double rb = 0.5 * (rho_i + rho_j);
  double Us = 0.5 * (UL + UR) + (p_i - p_j) / (2.0 * rb * c);
  double beta = fmin(3.0 * fmax(UL - UR, 0.0), c);
  *Pstar = 0.5 * (p_i + p_j) + 0.5 * rb * beta * (UL - UR);
  for (int k = 0; k < d; ++k) vstar[k] = 0.5 * (vi[k] + vj[k]) - (Us - 0.5 * (UL + UR)) * e[k];
}

/* ----------------------------------------------------- Neo-Hookean material
 * Strain energy (Section 2.1): W = mu tr(E) - mu ln J + lambda/2 (ln J)^2 with
 * E = (F^T F - I)/2 and J = det F.  Reading: S = dW/dE written out is
 *   S = mu (I - C^-1) + lambda ln(J) C^-1,  C = F^T F,
 * and P = F S.  In 2D the tensors are 2 x 2 (plane strain). */
void ora_nh_stress(int d, const double *F, double mu, double lam, double *P) {
  double Ft[9], C[9], Ci[9], S[9];
  mat_transpose(d, F, Ft);
  mat_mul(d, Ft, F, C);
  mat_inv(d, C, Ci);
  double J = mat_det(d, F);
  double lj = log(J);
  memset(S, 0, sizeof S);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) S[3 * i + j] = mu * ((i == j ? 1.0 : 0.0) - Ci[3 * i + j]) + lam * lj * Ci[3 * i + j];
  mat_mul(d, F, S, P);
}

double ora_nh_energy(int d, const double *F, double mu, double lam) {
  double Ft[9], C[9];
  mat_transpose(d, F, Ft);
  mat_mul(d, Ft, F, C);
  double trE = 0.0;
  for (int i = 0; i < d; ++i) trE += 0.5 * (C[4 * i] - 1.0);
  double lj = log(mat_det(d, F));
  return mu * trE - mu * lj + 0.5 * lam * lj * lj;
}

/* ------------------------------------------ linear elastic (Kirchhoff) material
 * Isotropic linear elasticity in the Green-Lagrange strain (Section 2.1):
 *   E = (F^T F - I)/2,  S = lambda tr(E) I + 2 mu E,  P = F S,
 * with strain energy W = lambda/2 tr(E)^2 + mu E:E.  Plane strain in 2D. */
void ora_svk_stress(int d, const double *F, double mu, double lam, double *P) {
  double Ft[9], C[9], E[9], S[9];
  mat_transpose(d, F, Ft);
  mat_mul(d, Ft, F, C);
  memset(E, 0, sizeof E);
  memset(S, 0, sizeof S);
  double trE = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) E[3 * i + j] = 0.5 * (C[3 * i + j] - (i == j ? 1.0 : 0.0));
  for (int i = 0; i < d; ++i) trE += E[4 * i];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) S[3 * i + j] = 2.0 * mu * E[3 * i + j] + (i == j ? lam * trE : 0.0);
  mat_mul(d, F, S, P);
}

double ora_svk_energy(int d, const double *F, double mu, double lam) {
  double Ft[9], C[9];
  mat_transpose(d, F, Ft);
  mat_mul(d, Ft, F, C);
  double trE = 0.0, EE = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double e = 0.5 * (C[3 * i + j] - (i == j ? 1.0 : 0.0));
      EE += e * e;
      if (i == j) trE += e;
    }
  return 0.5 * lam * trE * trE + mu * EE;
}

/* ----------------------------------------------------- particle number density
 * psi0: sum of dp^d W over an unbounded lattice of spacing dp at h = h_ratio dp,
 * self included (reference value for the density reinitialisation). */
double ora_psi0(int d, double h_ratio) {
  double dp = 1.0, h = h_ratio * dp, s = 0.0;
  int R = (int)ceil(2.0 * h_ratio) + 1;
  int kz0 = (d == 3) ? -R : 0, kz1 = (d == 3) ? R : 0;
  for (int i = -R; i <= R; ++i)
    for (int j = -R; j <= R; ++j)
      for (int k = kz0; k <= kz1; ++k) {
        double r = sqrt((double)(i * i + j * j + k * k)) * dp;
        if (r < 2.0 * h) s += pow(dp, d) * ora_kernel_W(d, r, h);
      }
  return s;
}

/* ------------------------------------------------------------ geometry */

/* r_a - r_b with the minimum image on periodic axes */
static void disp(const ora_ctx *c, const double *xa, const double *xb, double *out) {
  for (int k = 0; k < 3; ++k) {
    double dx = (k < c->d) ? xa[k] - xb[k] : 0.0;
    if (k < c->d && c->per[k]) dx -= c->L[k] * floor(dx / c->L[k] + 0.5);
    out[k] = dx;
  }
}

/* Simple uniform bin grid over the box [lo, hi) with cells no smaller than
 * the search radius; positions outside the box go to the nearest edge bin. */
typedef struct {
  int n[3];
  double cs[3];
  int *start, *items;
} bins;

static void bin_index(const ora_ctx *c, const bins *b, const double *x, int *ci) {
  for (int k = 0; k < 3; ++k) {
    if (k >= c->d) {
      ci[k] = 0;
      continue;
    }
    double s = x[k] - c->lo[k];
    if (c->per[k]) s -= c->L[k] * floor(s / c->L[k]);
    int q = (int)floor(s / b->cs[k]);
    if (q < 0) q = 0;
    if (q >= b->n[k]) q = b->n[k] - 1;
    ci[k] = q;
  }
}

static void bins_build(const ora_ctx *c, bins *b, const double *x, int n, double radius) {
  int ncell = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < c->d) {
      double ext = c->hi[k] - c->lo[k];
      b->n[k] = (int)floor(ext / radius);
      if (b->n[k] < 1) b->n[k] = 1;
      b->cs[k] = ext / b->n[k];
    } else {
      b->n[k] = 1;
      b->cs[k] = 1.0;
    }
    ncell *= b->n[k];
  }
  b->start = (int *)calloc((size_t)ncell + 1, sizeof(int));
  b->items = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *cell = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) {
    int ci[3];
    bin_index(c, b, x + 3 * i, ci);
    cell[i] = ci[0] + b->n[0] * (ci[1] + b->n[1] * ci[2]);
    b->start[cell[i] + 1]++;
  }
  for (int q = 0; q < ncell; ++q) b->start[q + 1] += b->start[q];
  int *fill = (int *)calloc((size_t)ncell, sizeof(int));
  for (int i = 0; i < n; ++i) b->items[b->start[cell[i]] + fill[cell[i]]++] = i;
  free(fill);
  free(cell);
}

static void bins_free(bins *b) {
  free(b->start);
  free(b->items);
}

static int cmp_int(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}

/* Neighbours of point q among points x[0..n) within radius (strictly less),
 * excluding index `self`; ascending index order.  Returns count; fills out if
 * non-null. */
static int query(const ora_ctx *c, const bins *b, const double *x, const double *q, int self,
                 double radius, int *out) {
  int ci[3];
  bin_index(c, b, q, ci);
  int cnt = 0;
  int lo2 = (c->d == 3) ? -1 : 0, hi2 = (c->d == 3) ? 1 : 0;
  /* visit each distinct neighbouring bin once (small periodic grids alias) */
  int seen[27], nseen = 0;
  for (int dz = lo2; dz <= hi2; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int nb[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
        int ok = 1;
        for (int k = 0; k < c->d; ++k) {
          if (c->per[k]) nb[k] = (nb[k] % b->n[k] + b->n[k]) % b->n[k];
          else if (nb[k] < 0 || nb[k] >= b->n[k]) ok = 0;
        }
        if (!ok) continue;
        int cell = nb[0] + b->n[0] * (nb[1] + b->n[1] * nb[2]);
        int dup = 0;
        for (int s = 0; s < nseen; ++s) dup |= (seen[s] == cell);
        if (dup) continue;
        seen[nseen++] = cell;
        for (int t = b->start[cell]; t < b->start[cell + 1]; ++t) {
          int j = b->items[t];
          if (j == self) continue;
          double r[3];
          disp(c, q, x + 3 * j, r);
          if (norm(c->d, r) < radius) {
            if (out) out[cnt] = j;
            cnt++;
          }
        }
      }
  if (out) qsort(out, (size_t)cnt, sizeof(int), cmp_int);
  return cnt;
}

/* CSR neighbour lists of the points q[0..nq) among x[0..n); self_same: skip
 * the same index (q and x the same set). */
static void build_csr(const ora_ctx *c, const double *q, int nq, const double *x, int n,
                      int self_same, double radius, int **start_out, int **idx_out) {
  bins b;
  bins_build(c, &b, x, n, radius);
  int *start = (int *)calloc((size_t)nq + 1, sizeof(int));
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nq; ++i) start[i + 1] = query(c, &b, x, q + 3 * i, self_same ? i : -1, radius, NULL);
  for (int i = 0; i < nq; ++i) start[i + 1] += start[i];
  int *idx = (int *)malloc(sizeof(int) * (size_t)(start[nq] > 0 ? start[nq] : 1));
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nq; ++i) query(c, &b, x, q + 3 * i, self_same ? i : -1, radius, idx + start[i]);
  bins_free(&b);
  *start_out = start;
  *idx_out = idx;
}

/* Brute-force O(N^2) neighbour lists (for the tests of the bin grid). */
int ora_brute_pairs(const ora_scene *sc, const double *x, int n, double radius, int *start,
                    int *idx) {
  ora_ctx c;
  memset(&c, 0, sizeof c);
  c.d = sc->dim;
  for (int k = 0; k < 3; ++k) {
    c.lo[k] = sc->lo[k];
    c.hi[k] = sc->hi[k];
    c.L[k] = sc->hi[k] - sc->lo[k];
    c.per[k] = sc->periodic[k];
  }
  double *x3 = (double *)calloc((size_t)n * 3 + 3, sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < c.d; ++k) x3[3 * i + k] = x[c.d * i + k];
  int cnt = 0;
  for (int i = 0; i < n; ++i) {
    if (start) start[i] = cnt;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3];
      disp(&c, x3 + 3 * i, x3 + 3 * j, r);
      if (norm(c.d, r) < radius) {
        if (idx) idx[cnt] = j;
        cnt++;
      }
    }
  }
  if (start) start[n] = cnt;
  free(x3);
  return cnt;
}

/* Same lists through the bin grid used by the oracle. */
int ora_grid_pairs(const ora_scene *sc, const double *x, int n, double radius, int *start,
                   int *idx) {
  ora_ctx c;
  memset(&c, 0, sizeof c);
  c.d = sc->dim;
  for (int k = 0; k < 3; ++k) {
    c.lo[k] = sc->lo[k];
    c.hi[k] = sc->hi[k];
    c.L[k] = sc->hi[k] - sc->lo[k];
    c.per[k] = sc->periodic[k];
  }
  double *x3 = (double *)calloc((size_t)n * 3 + 3, sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < c.d; ++k) x3[3 * i + k] = x[c.d * i + k];
  int *s = NULL, *ix = NULL;
  build_csr(&c, x3, n, x3, n, 1, radius, &s, &ix);
  int cnt = s[n];
  if (start) memcpy(start, s, sizeof(int) * (size_t)(n + 1));
  if (idx) memcpy(idx, ix, sizeof(int) * (size_t)cnt);
  free(s);
  free(ix);
  free(x3);
  return cnt;
}

/* ------------------------------------------------------------ context */

static double *zalloc(size_t n) { return (double *)calloc(n > 0 ? n : 1, sizeof(double)); }

static void load_vec(double *dst, const double *src, int n, int d) {
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < d; ++k) dst[3 * i + k] = src ? src[d * i + k] : 0.0;
}

void ora_destroy(ora_ctx *c);

ora_ctx *ora_create(const ora_scene *sc) {
  ora_ctx *c = (ora_ctx *)calloc(1, sizeof(ora_ctx));
  int d = c->d = sc->dim;
  c->nf = sc->n_fluid;
  c->nw = sc->n_wall;
  c->ns = sc->n_solid;
  c->nc = sc->n_clamp;
  c->dpf = sc->dp_f;
  c->dps = sc->dp_s;
  c->hf = sc->h_ratio * sc->dp_f;
  c->hs = sc->h_ratio * sc->dp_s;
  c->rho0 = sc->rho0_f;
  c->c = sc->c_f;
  c->eta = sc->eta;
  c->gam = sc->gamma;
  for (int k = 0; k < 3; ++k) {
    c->g[k] = (k < d) ? sc->g[k] : 0.0;
    c->lo[k] = sc->lo[k];
    c->hi[k] = sc->hi[k];
    c->L[k] = sc->hi[k] - sc->lo[k];
    c->per[k] = (k < d) ? sc->periodic[k] : 0;
  }
  /* Moduli (Section 2.1); reading: E = 2G(1 + nu) = 3K(1 - 2 nu), the printed
   * 2G(1 + 2 nu) being a typo; c_S = sqrt(K / rho0_S). */
  c->rho0s = sc->rho0_s;
  c->E = sc->E;
  c->nu = sc->nu;
  c->mu = sc->E / (2.0 * (1.0 + sc->nu));
  c->lam = sc->E * sc->nu / ((1.0 + sc->nu) * (1.0 - 2.0 * sc->nu));
  c->K = c->lam + 2.0 * c->mu / 3.0;
  c->cs = sqrt(c->K / c->rho0s);
  c->cfl_ac = sc->cfl_ac;
  c->cfl_ad = sc->cfl_ad;
  c->cfl_s = sc->cfl_s;
  c->uref = sc->u_ref;
  c->hydroH = sc->hydro_H;
  c->inU0 = sc->inflow_U0;
  c->ints = sc->inflow_ts;
  c->inH = sc->inflow_H;
  c->inlen = sc->inflow_len;
  c->riemann = sc->riemann;
  c->reinit = sc->density_reinit;
  c->material = sc->material;
  c->single = sc->single_step;
  c->vv = sc->velocity_verlet;
  c->psi0 = ora_psi0(d, sc->h_ratio);

  int nf = c->nf, nw = c->nw, ns = c->ns;
  c->x = zalloc(3 * (size_t)nf);
  c->v = zalloc(3 * (size_t)nf);
  c->a = zalloc(3 * (size_t)nf);
  c->xr = zalloc(3 * (size_t)nf);
  c->sn_v = zalloc(3 * (size_t)nf);
  c->rho = zalloc(nf);
  c->drho = zalloc(nf);
  c->m = zalloc(nf);
  c->p = zalloc(nf);
  c->sn_rho = zalloc(nf);
  c->sn_p = zalloc(nf);
  load_vec(c->x, sc->x_fluid, nf, d);
  load_vec(c->v, sc->v_fluid, nf, d);
  /* Initial fluid state (reading): hydrostatic pressure p = rho0 |g| (H - y)
   * along the vertical (last) axis, density from the inverse equation of
   * state, mass m = rho dp^d. */
  double gabs = norm(d, c->g);
  for (int i = 0; i < nf; ++i) {
    double pr = c->rho0 * gabs * (c->hydroH - c->x[3 * i + d - 1]);
    if (gabs == 0.0) pr = 0.0;
    c->rho[i] = ora_eos_inv(pr, c->rho0, c->c, c->gam);
    c->m[i] = c->rho[i] * pow(c->dpf, d);
  }
  c->xw = zalloc(3 * (size_t)nw);
  c->wn = zalloc(3 * (size_t)nw);
  load_vec(c->xw, sc->x_wall, nw, d);
  load_vec(c->wn, sc->nrm_wall, nw, d);

  c->x0 = zalloc(3 * (size_t)ns);
  c->u = zalloc(3 * (size_t)ns);
  c->vs = zalloc(3 * (size_t)ns);
  c->as = zalloc(3 * (size_t)ns);
  c->n0 = zalloc(3 * (size_t)ns);
  c->sn = zalloc(3 * (size_t)ns);
  c->vbar = zalloc(3 * (size_t)ns);
  c->abar = zalloc(3 * (size_t)ns);
  c->fF = zalloc(3 * (size_t)ns);
  c->fFp = zalloc(3 * (size_t)ns);
  c->xsr = zalloc(3 * (size_t)ns);
  c->F = zalloc(9 * (size_t)ns);
  c->dF = zalloc(9 * (size_t)ns);
  c->B = zalloc(9 * (size_t)ns);
  c->ms = zalloc(ns);
  c->V0 = zalloc(ns);
  c->clamp = (int *)calloc((size_t)ns + 1, sizeof(int));
  load_vec(c->x0, sc->x_solid, ns, d);
  for (int a = 0; a < ns; ++a) {
    c->clamp[a] = (a >= ns - c->nc);
    mat_eye(c->F + 9 * a);
    c->V0[a] = pow(c->dps, d);
    c->ms[a] = c->rho0s * c->V0[a];
    if (sc->v_solid && !c->clamp[a])
      for (int k = 0; k < d; ++k) c->vs[3 * a + k] = sc->v_solid[d * a + k];
  }
  /* Reference configuration (Section 2.2, correction matrix): neighbour sets
   * at |r0_ab| < 2 h_S, kernel gradients, and
   *   B_a = ( sum_b V_b (r0_b - r0_a) (x) grad_a W_ab )^-1;
   * reading: the volume V_b, missing in the printed formula, is included so
   * that B is dimensionless and the corrected gradient of a linear field is exact. */
  build_csr(c, c->x0, ns, c->x0, ns, 1, 2.0 * c->hs, &c->s_start, &c->s_idx);
  c->n_ss = c->s_start[ns];
  c->s_grad = zalloc(3 * (size_t)c->n_ss);
  for (int a = 0; a < ns; ++a) {
    double A[9] = {0}, nsum[3] = {0};
    for (int t = c->s_start[a]; t < c->s_start[a + 1]; ++t) {
      int b = c->s_idx[t];
      double r[3];
      disp(c, c->x0 + 3 * a, c->x0 + 3 * b, r);
      double rr = norm(d, r);
      double dW = ora_kernel_dW(d, rr, c->hs);
      for (int k = 0; k < d; ++k) c->s_grad[3 * t + k] = r[k] / rr * dW;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) A[3 * i + j] += c->V0[b] * (-r[i]) * c->s_grad[3 * t + j];
      for (int k = 0; k < d; ++k) nsum[k] -= c->V0[b] * c->s_grad[3 * t + k];
    }
    if (c->s_start[a + 1] > c->s_start[a]) mat_inv(d, A, c->B + 9 * a);
    else mat_eye(c->B + 9 * a);
    /* Surface normal (reading): n0 = normalise(-sum_b V_b grad_a W_ab), set to
     * zero where |sum| h_S < 0.01 (the mid-plane of a thin plate). */
    double nn = norm(d, nsum);
    if (nn * c->hs >= 0.01)
      for (int k = 0; k < d; ++k) c->n0[3 * a + k] = nsum[k] / nn;
    for (int k = 0; k < 3; ++k) c->sn[3 * a + k] = c->n0[3 * a + k];
  }
  c->need_rebuild = 1;
  return c;
}

void ora_destroy(ora_ctx *c) {
  if (!c) return;
  double *bufs[] = {c->x, c->v, c->rho, c->drho, c->m, c->a, c->p, c->xr, c->sn_rho, c->sn_p,
                    c->sn_v, c->xw, c->wn, c->x0, c->u, c->vs, c->as, c->F, c->dF, c->B,
                    c->n0, c->sn, c->vbar, c->abar, c->fF, c->xsr, c->ms, c->V0, c->s_grad, c->fFp};
  for (size_t k = 0; k < sizeof bufs / sizeof bufs[0]; ++k) free(bufs[k]);
  int *ibufs[] = {c->clamp, c->s_start, c->s_idx, c->ff_start, c->ff_idx, c->fb_start,
                  c->fb_idx, c->sf_start, c->sf_idx};
  for (size_t k = 0; k < sizeof ibufs / sizeof ibufs[0]; ++k) free(ibufs[k]);
  free(c);
}

/* ------------------------------------------------------------ pair terms */

/* Boundary particle k of the fluid-side lists: k < nw is wall k, otherwise the
 * solid particle k - nw.  Position at the last rebuild, averaged velocity and
 * acceleration, normal and volume. */
static void bnd_state(const ora_ctx *c, int k, const double **xb, const double **vb,
                      const double **ab, const double **nb, double *Vb) {
  static const double zero[3] = {0.0, 0.0, 0.0};
  if (k < c->nw) {
    *xb = c->xw + 3 * k;
    *vb = zero;
    *ab = zero;
    *nb = c->wn + 3 * k;
    *Vb = pow(c->dpf, c->d);
  } else {
    int a = k - c->nw;
    *xb = c->xsr + 3 * a;
    *vb = c->vbar + 3 * a;
    *ab = c->abar + 3 * a;
    *nb = c->sn + 3 * a;
    /* reading: a solid particle's volume in the coupling is its current
     * volume V0 J = m / rho */
    *Vb = c->V0[a] * mat_det(c->d, c->F + 9 * a);
  }
}

/* Force on fluid particle i from boundary particle a (Section 3.1, coupling
 * forces at h_F; Section 3.2, imaginary pressure and velocity from the
 * time-averaged solid velocity and acceleration):
 *   f = -2 V_i V_a (p_i rho_d + p_d rho_i)/(rho_i + rho_d) grad_i W_ia
 *       + 2 eta V_i V_a (v_i - v_d)/(|r_ia| + 0.01 h) dW/dr.
 * Readings: p_d = p_i + rho_i max(0, (abar_a - g).n_a)(r_ia.n_a) with n_a the
 * outward normal of the solid and r_ia = r_i - r_a (hydrostatic extrapolation;
 * the printed sign does not give it for either orientation of n), and
 * v_d = 2 vbar_a - v_i (the printed 2 v_i - vbar_a would be anti-viscous). */
static void coupling_pair(const ora_ctx *c, double rho_i, double p_i, const double *v_i,
                          double V_i, const double *xi, int k, double *f, double *fp) {
  const double *xb, *vb, *ab, *nb;
  double Va;
  bnd_state(c, k, &xb, &vb, &ab, &nb, &Va);
  int d = c->d;
  double r[3];
  disp(c, xi, xb, r);
  double rr = norm(d, r);
  double dW = ora_kernel_dW(d, rr, c->hf);
  double e[3] = {0};
  for (int q = 0; q < d; ++q) e[q] = r[q] / rr;
  double amg[3];
  for (int q = 0; q < 3; ++q) amg[q] = ab[q] - c->g[q];
  double s = fmax(0.0, dot(d, amg, nb));
  double pd = p_i + rho_i * s * dot(d, r, nb);
  double rhod = ora_eos_inv(pd, c->rho0, c->c, c->gam);
  double pf = (p_i * rhod + pd * rho_i) / (rho_i + rhod);
  for (int q = 0; q < 3; ++q) f[q] = 0.0;
  for (int q = 0; q < d; ++q) {
    double vd = 2.0 * vb[q] - v_i[q];
    double fpress = -2.0 * V_i * Va * pf * dW * e[q];
    f[q] = fpress + 2.0 * c->eta * V_i * Va * (v_i[q] - vd) / (rr + 0.01 * c->hf) * dW;
    if (fp) fp[q] = fpress;
  }
}

/* ------------------------------------------------------------ O2 rebuild */

static double vmax_fluid(const ora_ctx *c) {
  double m = 0.0;
  for (int i = 0; i < c->nf; ++i) m = fmax(m, norm(c->d, c->v + 3 * i));
  return m;
}

/* Start of an advection step (Algorithm 1, outer loop): advection time step,
 * neighbour lists and frozen pair geometry, density reinitialisation, normals. */
void ora_rebuild(ora_ctx *c) {
  int d = c->d, nf = c->nf, nw = c->nw, ns = c->ns;
  /* Advection criterion (Section 3.2).  Readings: |v|max is floored at U_ref
   * (c_F / 10) so that the step is finite at rest; the viscous bound uses
   * h^2 rho0 / eta (eta is a dynamic viscosity) and is dropped for eta = 0. */
  double vm = fmax(vmax_fluid(c), c->uref);
  double dt = c->cfl_ad * c->hf / vm;
  if (c->eta > 0.0) dt = fmin(dt, c->cfl_ad * c->hf * c->hf * c->rho0 / c->eta);
  c->dt_ad = dt;
  c->adv_accum = 0.0;
  /* Frozen geometry (reading): kernel values and gradients are updated only
   * here, from the positions at this rebuild. */
  memcpy(c->xr, c->x, sizeof(double) * 3 * (size_t)nf);
  for (int a = 0; a < ns; ++a)
    for (int k = 0; k < 3; ++k) c->xsr[3 * a + k] = c->x0[3 * a + k] + c->u[3 * a + k];
  /* boundary set for the fluid: walls, then free solid particles */
  int nfree = ns - c->nc;
  int nb = nw + nfree;
  double *xb = zalloc(3 * (size_t)nb);
  memcpy(xb, c->xw, sizeof(double) * 3 * (size_t)nw);
  memcpy(xb + 3 * (size_t)nw, c->xsr, sizeof(double) * 3 * (size_t)nfree);
  free(c->ff_start);
  free(c->ff_idx);
  free(c->fb_start);
  free(c->fb_idx);
  free(c->sf_start);
  free(c->sf_idx);
  double rad = 2.0 * c->hf;
  build_csr(c, c->xr, nf, c->xr, nf, 1, rad, &c->ff_start, &c->ff_idx);
  build_csr(c, c->xr, nf, xb, nb, 0, rad, &c->fb_start, &c->fb_idx);
  build_csr(c, c->xsr, nfree, c->xr, nf, 0, rad, &c->sf_start, &c->sf_idx);
  free(xb);
  c->n_ff = c->ff_start[nf];
  c->n_fb = c->fb_start[nf];
  c->n_sf = c->sf_start[nfree];
  /* Density reinitialisation (reading): psi_i = sum_j V_j W_ij over fluid,
   * wall and free-solid neighbours and self, with V_j = dp^d of j's phase;
   * mode 1: rho_i = rho0 max(1, psi_i / psi0);
   * mode 2: rho_i = max(rho_i, rho0 psi_i / psi0) (keeps a compressed
   * continuity density, lifts under-dense free-surface particles). */
  if (c->reinit) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nf; ++i) {
      double psi = pow(c->dpf, d) * ora_kernel_W(d, 0.0, c->hf);
      for (int t = c->ff_start[i]; t < c->ff_start[i + 1]; ++t) {
        double r[3];
        disp(c, c->xr + 3 * i, c->xr + 3 * c->ff_idx[t], r);
        psi += pow(c->dpf, d) * ora_kernel_W(d, norm(d, r), c->hf);
      }
      for (int t = c->fb_start[i]; t < c->fb_start[i + 1]; ++t) {
        int k = c->fb_idx[t];
        const double *xk = (k < nw) ? c->xw + 3 * k : c->xsr + 3 * (k - nw);
        double Vk = (k < nw) ? pow(c->dpf, d) : pow(c->dps, d);
        double r[3];
        disp(c, c->xr + 3 * i, xk, r);
        psi += Vk * ora_kernel_W(d, norm(d, r), c->hf);
      }
      if (c->reinit == 2) c->rho[i] = fmax(c->rho[i], c->rho0 * psi / c->psi0);
      else c->rho[i] = c->rho0 * fmax(1.0, psi / c->psi0);
    }
    c->interactions += c->n_ff + c->n_fb;
  }
  /* Normal update (reading): n = normalise(F^-T n0), zero stays zero. */
  for (int a = 0; a < ns; ++a) {
    double Fi[9], Fit[9], nn[3] = {0};
    mat_inv(d, c->F + 9 * a, Fi);
    mat_transpose(d, Fi, Fit);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) nn[i] += Fit[3 * i + j] * c->n0[3 * a + j];
    double l = norm(d, nn);
    for (int k = 0; k < 3; ++k) c->sn[3 * a + k] = (l > 0.0) ? nn[k] / l : 0.0;
  }
  c->rebuilds++;
  c->need_rebuild = 0;
}

/* ------------------------------------------------------------ O3-O7 fluid step */

static double inflow_speed(const ora_ctx *c, double y, double t) {
  /* Section 4.1 inflow.  Reading: U(y) = 6 Ubar y (H - y) / H^2 (peak 1.5 Ubar,
   * mean Ubar; the printed 1.5 factor drops a 4), Ubar ramped by
   * 0.5 U0 (1 - cos(pi t / 2)) up to t_s. */
  double Ub = (t <= c->ints) ? 0.5 * c->inU0 * (1.0 - cos(0.5 * M_PI * t)) : c->inU0;
  if (y <= 0.0 || y >= c->inH) return 0.0;
  return 6.0 * Ub * y * (c->inH - y) / (c->inH * c->inH);
}

static double solid_dt(const ora_ctx *c);

/* Pressure from the density and the snapshot the coupling on the solid reads
 * (the state at which the fluid forces are evaluated). */
static void fluid_snapshot(ora_ctx *c) {
  for (int i = 0; i < c->nf; ++i) {
    c->p[i] = ora_eos(c->rho[i], c->rho0, c->c, c->gam);
    c->sn_rho[i] = c->rho[i];
    c->sn_p[i] = c->p[i];
    for (int k = 0; k < 3; ++k) c->sn_v[3 * i + k] = c->v[3 * i + k];
  }
}

/* Momentum equation (Section 3.1) at the current density, pressure and
 * velocity: Riemann pressure, viscous term, coupling forces from walls and
 * solid, gravity. */
static void fluid_accel(ora_ctx *c) {
  int d = c->d, nf = c->nf;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nf; ++i) {
    double acc[3] = {0.0, 0.0, 0.0};
    double Vi = c->m[i] / c->rho[i];
    for (int t = c->ff_start[i]; t < c->ff_start[i + 1]; ++t) {
      int j = c->ff_idx[t];
      double r[3];
      disp(c, c->xr + 3 * i, c->xr + 3 * j, r);
      double rr = norm(d, r);
      double dW = ora_kernel_dW(d, rr, c->hf);
      double e[3] = {0};
      for (int q = 0; q < d; ++q) e[q] = r[q] / rr;
      double Vj = c->m[j] / c->rho[j];
      double Ps, vs[3];
      ora_riemann(d, c->riemann, c->c, c->rho[i], c->rho[j], c->p[i], c->p[j], c->v + 3 * i,
                  c->v + 3 * j, e, &Ps, vs);
      for (int q = 0; q < d; ++q)
        acc[q] += (-2.0 * Vi * Vj * Ps * dW * e[q] +
                   2.0 * c->eta * Vi * Vj * (c->v[3 * i + q] - c->v[3 * j + q]) / rr * dW) /
                  c->m[i];
    }
    for (int t = c->fb_start[i]; t < c->fb_start[i + 1]; ++t) {
      double f[3];
      coupling_pair(c, c->rho[i], c->p[i], c->v + 3 * i, Vi, c->xr + 3 * i, c->fb_idx[t], f, NULL);
      for (int q = 0; q < d; ++q) acc[q] += f[q] / c->m[i];
    }
    /* reading: body force enters as m_i g */
    for (int q = 0; q < d; ++q) c->a[3 * i + q] = acc[q] + c->g[q];
  }
}

/* Continuity (Section 3.1) at the current density and velocity.
 * Reading: walls and solid add rho_i sum_a V_a (v_i - vbar_a).grad_i W_ia. */
static void fluid_drho(const ora_ctx *c, double *drho) {
  int d = c->d, nf = c->nf;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nf; ++i) {
    double s = 0.0;
    for (int t = c->ff_start[i]; t < c->ff_start[i + 1]; ++t) {
      int j = c->ff_idx[t];
      double r[3];
      disp(c, c->xr + 3 * i, c->xr + 3 * j, r);
      double rr = norm(d, r);
      double dW = ora_kernel_dW(d, rr, c->hf);
      double e[3] = {0};
      for (int q = 0; q < d; ++q) e[q] = r[q] / rr;
      double Vj = c->m[j] / c->rho[j];
      double Ps, vs[3];
      ora_riemann(d, c->riemann, c->c, c->rho[i], c->rho[j], c->p[i], c->p[j], c->v + 3 * i,
                  c->v + 3 * j, e, &Ps, vs);
      double dv[3] = {0};
      for (int q = 0; q < d; ++q) dv[q] = c->v[3 * i + q] - vs[q];
      s += 2.0 * c->rho[i] * Vj * dot(d, dv, e) * dW;
    }
    for (int t = c->fb_start[i]; t < c->fb_start[i + 1]; ++t) {
      const double *xb, *vb, *ab, *nb;
      double Va;
      bnd_state(c, c->fb_idx[t], &xb, &vb, &ab, &nb, &Va);
      double r[3];
      disp(c, c->xr + 3 * i, xb, r);
      double rr = norm(d, r);
      double dW = ora_kernel_dW(d, rr, c->hf);
      double e[3] = {0}, dv[3] = {0};
      for (int q = 0; q < d; ++q) {
        e[q] = r[q] / rr;
        dv[q] = c->v[3 * i + q] - vb[q];
      }
      s += c->rho[i] * Va * dot(d, dv, e) * dW;
    }
    drho[i] = s;
  }
}

/* periodic wrap and inflow buffer (Section 4.1; reading: periodic channel
 * whose first inflow_len of length is reset to the inflow profile) */
static void fluid_wrap_inflow(ora_ctx *c, double tn) {
  int d = c->d;
  for (int i = 0; i < c->nf; ++i) {
    for (int k = 0; k < d; ++k)
      if (c->per[k]) {
        double s = c->x[3 * i + k] - c->lo[k];
        c->x[3 * i + k] = c->lo[k] + s - c->L[k] * floor(s / c->L[k]);
      }
    if (c->inlen > 0.0 && c->x[3 * i] - c->lo[0] < c->inlen) {
      c->v[3 * i] = inflow_speed(c, c->x[3 * i + 1], tn);
      for (int k = 1; k < d; ++k) c->v[3 * i + k] = 0.0;
    }
  }
}

/* The velocity-based Verlet scheme that Section 3.3 contrasts with its own
 * (test contrast only): half a step of velocity with the acceleration of the
 * last evaluation, a full step of position and density, the forces and the
 * density rate evaluated at the new state, another half step of velocity.
 * The accelerations and rates start at zero before the first evaluation. */
static void fluid_step_velocity_verlet(ora_ctx *c, double dt) {
  int d = c->d, nf = c->nf;
  for (int i = 0; i < nf; ++i) {
    for (int k = 0; k < d; ++k) c->v[3 * i + k] += 0.5 * dt * c->a[3 * i + k];
    c->rho[i] += dt * c->drho[i];
    for (int k = 0; k < d; ++k) c->x[3 * i + k] += dt * c->v[3 * i + k];
  }
  fluid_snapshot(c);
  fluid_accel(c);
  fluid_drho(c, c->drho);
  for (int i = 0; i < nf; ++i)
    for (int k = 0; k < d; ++k) c->v[3 * i + k] += 0.5 * dt * c->a[3 * i + k];
  fluid_wrap_inflow(c, c->t + dt);
  c->interactions += 2 * (c->n_ff + c->n_fb);
}

/* One fluid acoustic step with the position-based Verlet scheme (Section 3.3). */
void ora_fluid_step(ora_ctx *c) {
  int d = c->d, nf = c->nf;
  /* Acoustic criterion (Section 3.2) with the scene's CFL number. */
  c->dt_ac = c->cfl_ac * c->hf / (c->c + vmax_fluid(c));
  /* The contrast to the multiple time steps (Section 3.2): the solid step,
   * when smaller, is the single step of both fluid and structure. */
  if (c->single && c->ns > c->nc) c->dt_ac = fmin(c->dt_ac, solid_dt(c));
  double dt = c->dt_ac;
  if (c->vv) {
    fluid_step_velocity_verlet(c, dt);
    return;
  }
  /* first half: density and position to the mid-point */
  for (int i = 0; i < nf; ++i) {
    c->rho[i] += 0.5 * dt * c->drho[i];
    for (int k = 0; k < d; ++k) c->x[3 * i + k] += 0.5 * dt * c->v[3 * i + k];
  }
  /* forces at the mid-point */
  fluid_snapshot(c);
  fluid_accel(c);
  /* velocity: full step */
  for (int i = 0; i < nf; ++i)
    for (int k = 0; k < d; ++k) c->v[3 * i + k] += dt * c->a[3 * i + k];
  /* continuity with the new velocity at the mid-point density */
  double *drho = zalloc(nf);
  fluid_drho(c, drho);
  /* second half: position with the new velocity, density with the new rate */
  for (int i = 0; i < nf; ++i) {
    c->drho[i] = drho[i];
    c->rho[i] += 0.5 * dt * drho[i];
    for (int k = 0; k < d; ++k) c->x[3 * i + k] += 0.5 * dt * c->v[3 * i + k];
  }
  free(drho);
  fluid_wrap_inflow(c, c->t + dt);
  c->interactions += 2 * (c->n_ff + c->n_fb);
}

/* ------------------------------------------------------------ O8 coupling on the solid */

/* f^F_a: the exact negatives of the fluid-side coupling pair terms, evaluated
 * from the same mid-state snapshot (reading of Algorithm 1's ordering, which
 * makes the momentum exchange of every pair exact). */
void ora_couple(ora_ctx *c) {
  int d = c->d, nfree = c->ns - c->nc;
#pragma omp parallel for schedule(static)
  for (int a = 0; a < c->ns; ++a) {
    double fa[3] = {0.0, 0.0, 0.0}, fap[3] = {0.0, 0.0, 0.0};
    if (a < nfree)
      for (int t = c->sf_start[a]; t < c->sf_start[a + 1]; ++t) {
        int i = c->sf_idx[t];
        double Vi = c->m[i] / c->sn_rho[i];
        double f[3], fp[3];
        coupling_pair(c, c->sn_rho[i], c->sn_p[i], c->sn_v + 3 * i, Vi, c->xr + 3 * i, c->nw + a, f, fp);
        for (int q = 0; q < d; ++q) {
          fa[q] -= f[q];
          fap[q] -= fp[q];
        }
      }
    for (int q = 0; q < 3; ++q) {
      c->fF[3 * a + q] = fa[q];
      c->fFp[3 * a + q] = fap[q];
    }
  }
  c->interactions += c->n_sf;
}

/* ------------------------------------------------------------ O9 solid sub-steps */

/* Solid time step (Section 3.2) over free particles at the step start;
 * the acceleration bound is dropped while |a|max = 0. */
static double solid_dt(const ora_ctx *c) {
  int d = c->d;
  double vm = 0.0, am = 0.0;
  for (int a = 0; a < c->ns; ++a)
    if (!c->clamp[a]) {
      vm = fmax(vm, norm(d, c->vs + 3 * a));
      am = fmax(am, norm(d, c->as + 3 * a));
    }
  double dts = c->cfl_s * c->hs / (c->cs + vm);
  if (am > 0.0) dts = fmin(dts, c->cfl_s * sqrt(c->hs / am));
  return dts;
}

/* P B of every solid particle at its current deformation gradient. */
static void solid_PB(const ora_ctx *c, double *PB) {
  int d = c->d;
#pragma omp parallel for schedule(static)
  for (int a = 0; a < c->ns; ++a) {
    double P[9];
    if (c->material == 1) ora_svk_stress(d, c->F + 9 * a, c->mu, c->lam, P);
    else ora_nh_stress(d, c->F + 9 * a, c->mu, c->lam, P);
    mat_mul(d, P, c->B + 9 * a, PB + 9 * a);
  }
}

/* Momentum (Section 2.2, corrected total-Lagrangian form at h_S):
 *   m_a dv/dt = sum_b V_a V_b (P_a B_a + P_b B_b) grad0_a W_ab + f^F_a + m_a g. */
static void solid_accel(ora_ctx *c, const double *PB) {
  int d = c->d;
#pragma omp parallel for schedule(static)
  for (int a = 0; a < c->ns; ++a) {
    if (c->clamp[a]) continue;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int t = c->s_start[a]; t < c->s_start[a + 1]; ++t) {
      int b = c->s_idx[t];
      for (int i = 0; i < d; ++i) {
        double s = 0.0;
        for (int j = 0; j < d; ++j) s += (PB[9 * a + 3 * i + j] + PB[9 * b + 3 * i + j]) * c->s_grad[3 * t + j];
        acc[i] += c->V0[a] * c->V0[b] * s;
      }
    }
    for (int q = 0; q < d; ++q) c->as[3 * a + q] = (acc[q] + c->fF[3 * a + q]) / c->ms[a] + c->g[q];
  }
}

/* Reading: dF/dt = sum_b V_b (v_b - v_a) (x) (B_a grad0_a W_ab), the
 * corrected gradient of the velocity. */
static void solid_rate(ora_ctx *c) {
  int d = c->d;
#pragma omp parallel for schedule(static)
  for (int a = 0; a < c->ns; ++a) {
    double G[9] = {0};
    if (!c->clamp[a])
      for (int t = c->s_start[a]; t < c->s_start[a + 1]; ++t) {
        int b = c->s_idx[t];
        double bg[3] = {0};
        for (int i = 0; i < d; ++i)
          for (int j = 0; j < d; ++j) bg[i] += c->B[9 * a + 3 * i + j] * c->s_grad[3 * t + j];
        for (int i = 0; i < d; ++i)
          for (int j = 0; j < d; ++j)
            G[3 * i + j] += c->V0[b] * (c->vs[3 * b + i] - c->vs[3 * a + i]) * bg[j];
      }
    memcpy(c->dF + 9 * a, G, sizeof G);
  }
}

/* Reading: the clamp block is held at u = 0, v = 0, F = I. */
static void solid_hold_clamp(ora_ctx *c, int a) {
  for (int q = 0; q < 3; ++q) c->u[3 * a + q] = c->vs[3 * a + q] = c->as[3 * a + q] = 0.0;
  mat_eye(c->F + 9 * a);
  memset(c->dF + 9 * a, 0, 9 * sizeof(double));
}

/* kappa solid steps with the position-based Verlet scheme (Section 3.3), the
 * fluid force held constant; then the time averages of Section 3.2. */
void ora_solid_substeps(ora_ctx *c) {
  int d = c->d, ns = c->ns;
  double dts = solid_dt(c);
  c->dt_s = dts;
  /* Reading: kappa = floor(dt_ac / dt_s) + 1 equal sub-steps of dt_ac / kappa,
   * so that they sum to dt_ac exactly.  With one shared step (the contrast of
   * Section 3.2) dt_ac <= dt_s already and the solid takes one step. */
  c->kappa = c->single ? 1 : (int)floor(c->dt_ac / dts) + 1;
  double del = c->dt_ac / c->kappa;
  double *u0 = zalloc(3 * (size_t)ns), *v0 = zalloc(3 * (size_t)ns);
  memcpy(u0, c->u, sizeof(double) * 3 * (size_t)ns);
  memcpy(v0, c->vs, sizeof(double) * 3 * (size_t)ns);
  double *PB = zalloc(9 * (size_t)ns);
  for (int sub = 0; sub < c->kappa; ++sub) {
    if (c->vv) {
      /* velocity-based contrast: half kick with the last evaluation, full
       * step of F (rate from the half-kicked velocity) and position, the
       * stress and acceleration at the new state, second half kick */
      for (int a = 0; a < ns; ++a) {
        if (c->clamp[a]) continue;
        for (int q = 0; q < d; ++q) c->vs[3 * a + q] += 0.5 * del * c->as[3 * a + q];
      }
      solid_rate(c);
      for (int a = 0; a < ns; ++a) {
        if (c->clamp[a]) continue;
        for (int q = 0; q < 9; ++q) c->F[9 * a + q] += del * c->dF[9 * a + q];
        for (int q = 0; q < d; ++q) c->u[3 * a + q] += del * c->vs[3 * a + q];
      }
      solid_PB(c, PB);
      solid_accel(c, PB);
      for (int a = 0; a < ns; ++a) {
        if (c->clamp[a]) {
          solid_hold_clamp(c, a);
          continue;
        }
        for (int q = 0; q < d; ++q) c->vs[3 * a + q] += 0.5 * del * c->as[3 * a + q];
      }
      c->interactions += 2 * c->n_ss;
      c->substeps++;
      continue;
    }
    /* first half: deformation gradient, density (rho0 / J), position */
    for (int a = 0; a < ns; ++a) {
      if (c->clamp[a]) continue;
      for (int q = 0; q < 9; ++q) c->F[9 * a + q] += 0.5 * del * c->dF[9 * a + q];
      for (int q = 0; q < d; ++q) c->u[3 * a + q] += 0.5 * del * c->vs[3 * a + q];
    }
    solid_PB(c, PB);
    solid_accel(c, PB);
    for (int a = 0; a < ns; ++a) {
      if (c->clamp[a]) continue;
      for (int q = 0; q < d; ++q) c->vs[3 * a + q] += del * c->as[3 * a + q];
    }
    /* deformation rate with the new velocity */
    solid_rate(c);
    /* second half: deformation gradient and position */
    for (int a = 0; a < ns; ++a) {
      if (c->clamp[a]) {
        solid_hold_clamp(c, a);
        continue;
      }
      for (int q = 0; q < 9; ++q) c->F[9 * a + q] += 0.5 * del * c->dF[9 * a + q];
      for (int q = 0; q < d; ++q) c->u[3 * a + q] += 0.5 * del * c->vs[3 * a + q];
    }
    c->interactions += 2 * c->n_ss;
    c->substeps++;
  }
  /* Time averages over the acoustic step (reading): vbar = (u_end - u_start)
   * / dt_ac, abar = (v_end - v_start) / dt_ac. */
  for (int a = 0; a < ns; ++a)
    for (int q = 0; q < d; ++q) {
      c->vbar[3 * a + q] = (c->u[3 * a + q] - u0[3 * a + q]) / c->dt_ac;
      c->abar[3 * a + q] = (c->vs[3 * a + q] - v0[3 * a + q]) / c->dt_ac;
    }
  free(u0);
  free(v0);
  free(PB);
  /* Advance time; the acoustic loop ends once the accumulated acoustic steps
   * reach the advection step (reading of the "while sum <= dt_ad" loop). */
  c->t += c->dt_ac;
  c->adv_accum += c->dt_ac;
  if (c->adv_accum >= c->dt_ad) c->need_rebuild = 1;
  c->steps++;
}

/* One acoustic step of Algorithm 1, with the rebuild at advection-step starts. */
void ora_step(ora_ctx *c) {
  if (c->need_rebuild) ora_rebuild(c);
  ora_fluid_step(c);
  ora_couple(c);
  ora_solid_substeps(c);
}

void ora_advance(ora_ctx *c, int n) {
  for (int s = 0; s < n; ++s) ora_step(c);
}

/* ------------------------------------------------------------ state I/O */

enum {
  F_X = 0, F_V, F_RHO, F_DRHO, F_A, F_P, /* fluid */
  S_U = 10, S_V, S_A, S_F, S_DF, S_FF, S_VBAR, S_ABAR, S_N, S_B, S_N0, S_X0, S_FFP /* solid */
};

static int field_shape(const ora_ctx *c, int f, double **buf, int *n, int *w, int *stride) {
  int d = c->d;
  *stride = 3;
  switch (f) {
  case F_X: *buf = c->x; *n = c->nf; *w = d; return 0;
  case F_V: *buf = c->v; *n = c->nf; *w = d; return 0;
  case F_A: *buf = c->a; *n = c->nf; *w = d; return 0;
  case F_RHO: *buf = c->rho; *n = c->nf; *w = 1; *stride = 1; return 0;
  case F_DRHO: *buf = c->drho; *n = c->nf; *w = 1; *stride = 1; return 0;
  case F_P: *buf = c->p; *n = c->nf; *w = 1; *stride = 1; return 0;
  case S_U: *buf = c->u; *n = c->ns; *w = d; return 0;
  case S_V: *buf = c->vs; *n = c->ns; *w = d; return 0;
  case S_A: *buf = c->as; *n = c->ns; *w = d; return 0;
  case S_FF: *buf = c->fF; *n = c->ns; *w = d; return 0;
  case S_VBAR: *buf = c->vbar; *n = c->ns; *w = d; return 0;
  case S_ABAR: *buf = c->abar; *n = c->ns; *w = d; return 0;
  case S_N: *buf = c->sn; *n = c->ns; *w = d; return 0;
  case S_N0: *buf = c->n0; *n = c->ns; *w = d; return 0;
  case S_X0: *buf = c->x0; *n = c->ns; *w = d; return 0;
  case S_FFP: *buf = c->fFp; *n = c->ns; *w = d; return 0;
  case S_F: *buf = c->F; *n = c->ns; *w = -d; *stride = 9; return 0;
  case S_DF: *buf = c->dF; *n = c->ns; *w = -d; *stride = 9; return 0;
  case S_B: *buf = c->B; *n = c->ns; *w = -d; *stride = 9; return 0;
  }
  return -1;
}

/* Copy a field out in index order: vectors n x d, tensors n x d x d. */
int ora_get(const ora_ctx *c, int f, double *out) {
  double *buf;
  int n, w, st;
  if (field_shape(c, f, &buf, &n, &w, &st)) return -1;
  int d = c->d;
  for (int i = 0; i < n; ++i) {
    if (w > 0)
      for (int k = 0; k < w; ++k) out[w * i + k] = buf[st * i + k];
    else
      for (int r = 0; r < d; ++r)
        for (int q = 0; q < d; ++q) out[d * d * i + d * r + q] = buf[9 * i + 3 * r + q];
  }
  return 0;
}

int ora_set(ora_ctx *c, int f, const double *in) {
  double *buf;
  int n, w, st;
  if (field_shape(c, f, &buf, &n, &w, &st)) return -1;
  int d = c->d;
  for (int i = 0; i < n; ++i) {
    if (w > 0)
      for (int k = 0; k < w; ++k) buf[st * i + k] = in[w * i + k];
    else
      for (int r = 0; r < d; ++r)
        for (int q = 0; q < d; ++q) buf[9 * i + 3 * r + q] = in[d * d * i + d * r + q];
  }
  return 0;
}

/* scalars: t, dt_ac, dt_ad, dt_s, adv_accum, kappa, need_rebuild, psi0,
 * K, mu, lambda, c_s */
void ora_scalars(const ora_ctx *c, double *out) {
  out[0] = c->t;
  out[1] = c->dt_ac;
  out[2] = c->dt_ad;
  out[3] = c->dt_s;
  out[4] = c->adv_accum;
  out[5] = c->kappa;
  out[6] = c->need_rebuild;
  out[7] = c->psi0;
  out[8] = c->K;
  out[9] = c->mu;
  out[10] = c->lam;
  out[11] = c->cs;
}

void ora_set_scalars(ora_ctx *c, const double *in) {
  c->t = in[0];
  c->dt_ac = in[1];
  c->dt_ad = in[2];
  c->dt_s = in[3];
  c->adv_accum = in[4];
  c->kappa = (int)in[5];
  c->need_rebuild = (int)in[6];
}

/* counters: ff, fb, sf, ss pairs; steps, rebuilds, substeps, interactions */
void ora_counters(const ora_ctx *c, long long *out) {
  out[0] = c->n_ff;
  out[1] = c->n_fb;
  out[2] = c->n_sf;
  out[3] = c->n_ss;
  out[4] = c->steps;
  out[5] = c->rebuilds;
  out[6] = c->substeps;
  out[7] = c->interactions;
}

/* totals (index order sums): fluid momentum (3), solid momentum (3), fluid
 * kinetic energy, solid kinetic energy, solid strain energy, sum of the
 * coupling force on the solid (3) */
void ora_totals(const ora_ctx *c, double *out) {
  int d = c->d;
  memset(out, 0, 12 * sizeof(double));
  for (int i = 0; i < c->nf; ++i) {
    for (int k = 0; k < d; ++k) out[k] += c->m[i] * c->v[3 * i + k];
    out[6] += 0.5 * c->m[i] * dot(d, c->v + 3 * i, c->v + 3 * i);
  }
  for (int a = 0; a < c->ns; ++a) {
    for (int k = 0; k < d; ++k) {
      out[3 + k] += c->ms[a] * c->vs[3 * a + k];
      out[9 + k] += c->fF[3 * a + k];
    }
    out[7] += 0.5 * c->ms[a] * dot(d, c->vs + 3 * a, c->vs + 3 * a);
    out[8] += c->V0[a] * (c->material == 1 ? ora_svk_energy(d, c->F + 9 * a, c->mu, c->lam)
                                           : ora_nh_energy(d, c->F + 9 * a, c->mu, c->lam));
  }
}

/* Sum over fluid particles of the force exerted on them by free solid
 * particles (walls excluded), from the current snapshot: the fluid-side half
 * of the coupling momentum exchange. */
void ora_fluid_side_coupling(const ora_ctx *c, double *out) {
  int d = c->d;
  out[0] = out[1] = out[2] = 0.0;
  for (int i = 0; i < c->nf; ++i) {
    double Vi = c->m[i] / c->sn_rho[i];
    for (int t = c->fb_start[i]; t < c->fb_start[i + 1]; ++t) {
      int k = c->fb_idx[t];
      if (k < c->nw) continue;
      double f[3];
      coupling_pair(c, c->sn_rho[i], c->sn_p[i], c->sn_v + 3 * i, Vi, c->xr + 3 * i, k, f, NULL);
      for (int q = 0; q < d; ++q) out[q] += f[q];
    }
  }
}

/* threads the oracle's parallel loops use */
int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the following parallel loops (timing only) */
void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* fluid masses (index order) */
void ora_masses(const ora_ctx *c, double *mf, double *ms) {
  if (mf) memcpy(mf, c->m, sizeof(double) * (size_t)c->nf);
  if (ms) memcpy(ms, c->ms, sizeof(double) * (size_t)c->ns);
}

/* the neighbour lists at the last rebuild: which = 0 fluid-fluid,
 * 1 fluid-boundary, 2 solid-fluid, 3 solid-solid reference */
int ora_pairs(const ora_ctx *c, int which, int *start, int *idx) {
  int *s, *ix, n;
  switch (which) {
  case 0: s = c->ff_start; ix = c->ff_idx; n = c->nf; break;
  case 1: s = c->fb_start; ix = c->fb_idx; n = c->nf; break;
  case 2: s = c->sf_start; ix = c->sf_idx; n = c->ns - c->nc; break;
  case 3: s = c->s_start; ix = c->s_idx; n = c->ns; break;
  default: return -1;
  }
  if (!s) return -2;
  if (start) memcpy(start, s, sizeof(int) * (size_t)(n + 1));
  if (idx) memcpy(idx, ix, sizeof(int) * (size_t)s[n]);
  return s[n];
}
