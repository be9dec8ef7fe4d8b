/*
 * Host-side driver that runs the FP64 oracle on small synthetic scenes under
 * AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
 * tests/test_oracle_sanitized.py with gcc; no GPU code involved).
 *
 * Scenes: a periodic 2D box with a free solid block (every pair loop, the
 * coupling, rebuilds), the same with the linear elastic law, one shared time
 * step and the velocity-based Verlet contrast; a 2D floor with a clamped solid
 * post and gravity (walls, clamp, density reinitialisation); a periodic 3D box
 * with a free solid block.  Prints one checksum line per scene and exits 0
 * when every run stays finite.
 */
#include "../oracle/oracle.c"

#include <stdio.h>

static uint64_t lcg = 0x9e3779b97f4a7c15ull;
static double urand(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

/* lattice of cell-centred points in [lo, hi) with spacing dp */
static int lattice(int d, const double *lo, const double *hi, double dp, double *out, int cap) {
  int n[3] = {1, 1, 1}, m = 0;
  for (int k = 0; k < d; ++k) n[k] = (int)floor((hi[k] - lo[k]) / dp + 0.5);
  for (int i = 0; i < n[0]; ++i)
    for (int j = 0; j < n[1]; ++j)
      for (int l = 0; l < n[2]; ++l) {
        if (m >= cap) return m;
        double p[3] = {lo[0] + (i + 0.5) * dp, lo[1] + (j + 0.5) * dp, d == 3 ? lo[2] + (l + 0.5) * dp : 0.0};
        for (int k = 0; k < d; ++k) out[d * m + k] = p[k];
        ++m;
      }
  return m;
}

static int inside(int d, const double *p, const double *lo, const double *hi) {
  for (int k = 0; k < d; ++k)
    if (!(p[k] > lo[k] && p[k] < hi[k])) return 0;
  return 1;
}

static int run(const char *name, ora_scene *sc, int steps) {
  ora_ctx *c = ora_create(sc);
  ora_advance(c, steps);
  double tot[12], s = 0.0;
  ora_totals(c, tot);
  for (int k = 0; k < 12; ++k) s += fabs(tot[k]);
  double sc8[12];
  ora_scalars(c, sc8);
  long long cnt[8];
  ora_counters(c, cnt);
  int ok = isfinite(s) && isfinite(sc8[0]);
  printf("%s: t %.6e checksum %.12e rebuilds %lld substeps %lld %s\n", name, sc8[0], s, cnt[5], cnt[6],
         ok ? "ok" : "NOT FINITE");
  ora_destroy(c);
  return ok ? 0 : 1;
}

/* periodic box of side 12 dp with a free solid block (dp_s = dp / 2) */
static int periodic_box(int d, int material, int single, int vv) {
  const double dp = 0.01, L = 12 * dp;
  double lo[3] = {0, 0, 0}, hi[3] = {L, L, d == 3 ? L : 1.0};
  double blo[3] = {0.375 * L, 0.375 * L, 0.375 * L}, bhi[3] = {0.625 * L, 0.625 * L, 0.625 * L};
  int capf = 4096, caps = 4096;
  double *xf = calloc((size_t)capf * 3, sizeof(double)), *vf = calloc((size_t)capf * 3, sizeof(double));
  double *xs = calloc((size_t)caps * 3, sizeof(double)), *vs = calloc((size_t)caps * 3, sizeof(double));
  double *tmp = calloc((size_t)capf * 3, sizeof(double));
  int nt = lattice(d, lo, hi, dp, tmp, capf), nf = 0;
  for (int i = 0; i < nt; ++i)
    if (!inside(d, tmp + d * i, blo, bhi)) {
      for (int k = 0; k < d; ++k) {
        xf[d * nf + k] = tmp[d * i + k];
        vf[d * nf + k] = (2.0 * urand() - 1.0) * 0.3;
      }
      ++nf;
    }
  int ns = lattice(d, blo, bhi, dp / 2, xs, caps);
  for (int i = 0; i < ns * d; ++i) vs[i] = (2.0 * urand() - 1.0) * 0.3;
  ora_scene sc = {.dim = d, .n_fluid = nf, .n_wall = 0, .n_solid = ns, .n_clamp = 0, .dp_f = dp, .dp_s = dp / 2,
                  .h_ratio = 1.3, .rho0_f = 1000.0, .c_f = 10.0, .eta = 0.5, .gamma = 7.0, .g = {0, 0, 0},
                  .rho0_s = 1200.0, .E = 2e5, .nu = 0.35, .cfl_ac = 0.25, .cfl_ad = 0.25, .cfl_s = 0.6,
                  .u_ref = 1.0, .periodic = {1, 1, d == 3}, .x_fluid = xf, .v_fluid = vf, .x_wall = NULL,
                  .nrm_wall = NULL, .x_solid = xs, .v_solid = vs, .riemann = 1, .density_reinit = 1,
                  .material = material, .single_step = single, .velocity_verlet = vv};
  for (int k = 0; k < 3; ++k) {
    sc.lo[k] = lo[k];
    sc.hi[k] = hi[k];
  }
  char name[96];
  snprintf(name, sizeof name, "periodic box %dD material %d single %d velocity-Verlet %d", d, material, single, vv);
  int rc = run(name, &sc, d == 3 ? 4 : 25);
  free(xf);
  free(vf);
  free(xs);
  free(vs);
  free(tmp);
  return rc;
}

/* water layer on a three-layer floor around a solid post clamped below the floor */
static int floor_with_post(void) {
  const double dp = 0.01, W = 0.2, H = 0.1;
  double flo[3] = {0, 0, 0}, fhi[3] = {W, H, 1};
  double plo[3] = {0.09, 0, 0}, phi[3] = {0.11, 0.06, 1};
  double clo[3] = {0.09, -0.015, 0}, chi[3] = {0.11, 0, 1};
  double wlo[3] = {0, -0.03, 0}, whi[3] = {W, 0, 1};
  int cap = 8192;
  double *xf = calloc((size_t)cap * 2, sizeof(double)), *tmp = calloc((size_t)cap * 2, sizeof(double));
  double *xw = calloc((size_t)cap * 2, sizeof(double)), *nw = calloc((size_t)cap * 2, sizeof(double));
  double *xs = calloc((size_t)cap * 2, sizeof(double));
  int nt = lattice(2, flo, fhi, dp, tmp, cap), nf = 0;
  for (int i = 0; i < nt; ++i)
    if (!inside(2, tmp + 2 * i, plo, phi)) {
      xf[2 * nf] = tmp[2 * i];
      xf[2 * nf + 1] = tmp[2 * i + 1];
      ++nf;
    }
  int nw_ = lattice(2, wlo, whi, dp, xw, cap);
  for (int i = 0; i < nw_; ++i) {
    nw[2 * i] = 0.0;
    nw[2 * i + 1] = 1.0;
  }
  int ns = lattice(2, plo, phi, dp / 2, xs, cap);
  int nc = lattice(2, clo, chi, dp / 2, xs + 2 * ns, cap - ns);
  double g = 9.81, c0 = 10.0 * sqrt(2.0 * g * H);
  ora_scene sc = {.dim = 2, .n_fluid = nf, .n_wall = nw_, .n_solid = ns + nc, .n_clamp = nc, .dp_f = dp,
                  .dp_s = dp / 2, .h_ratio = 1.3, .rho0_f = 1000.0, .c_f = c0, .eta = 0.0, .gamma = 7.0,
                  .g = {0, -g, 0}, .rho0_s = 1100.0, .E = 1e6, .nu = 0.4, .cfl_ac = 0.25, .cfl_ad = 0.25,
                  .cfl_s = 0.6, .u_ref = c0 / 10.0, .lo = {-0.05, -0.05, 0}, .hi = {W + 0.05, H + 0.1, 1},
                  .periodic = {0, 0, 0}, .hydro_H = H, .x_fluid = xf, .v_fluid = NULL, .x_wall = xw,
                  .nrm_wall = nw, .x_solid = xs, .v_solid = NULL, .riemann = 1, .density_reinit = 2};
  int rc = run("floor with a clamped post", &sc, 12);
  free(xf);
  free(tmp);
  free(xw);
  free(nw);
  free(xs);
  return rc;
}

int main(void) {
  int rc = 0;
  rc |= periodic_box(2, 0, 0, 0);
  rc |= periodic_box(2, 1, 0, 0);
  rc |= periodic_box(2, 0, 1, 0);
  rc |= periodic_box(2, 0, 0, 1);
  rc |= floor_with_post();
  rc |= periodic_box(3, 1, 1, 0);
  return rc;
}
