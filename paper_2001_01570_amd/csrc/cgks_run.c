/* cgks_run: drive the library through its C ABI alone (no Python, no torch).
 *
 *   cgks_run CONFIG STATE_IN STEPS STATE_OUT
 *
 * CONFIG: one line of numbers, in order
 *   dim nx ny x0 x1 y0 y1 gamma cfl bc0 bc1 bc2 bc3
 *   inflow_prim (16 values, side-major) weno_eps tau_eps tau_C fixed_dt mu
 *   [gauss_points [recon_vars [side_slopes [tang_weno]]]]  (optional; 2, CGKS_CONSERVATIVE, 0 and 0 when absent)
 * STATE_IN / STATE_OUT: the fields as raw native doubles in the layout of
 * cgks.h (6*nx values in 1D, 12*ny*nx in 2D).  The state is loaded from host
 * memory, advanced STEPS steps of the configured rule on the null stream and
 * written back; t and the step count go to stdout.  Exit status 0 on success,
 * 1 on a usage or I/O error, 2 on a library error (its message on stderr). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cgks.h"

static int fail(const char *what, int rc) {
  fprintf(stderr, "cgks_run: %s: %s (%d)\n", what, cgks_strerror(rc), rc);
  return 2;
}

int main(int argc, char **argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: cgks_run CONFIG STATE_IN STEPS STATE_OUT\n");
    return 1;
  }
  cgks_config cfg;
  memset(&cfg, 0, sizeof cfg);
  FILE *f = fopen(argv[1], "r");
  if (!f) { perror(argv[1]); return 1; }
  int ok = fscanf(f, "%d %d %d %lf %lf %lf %lf %lf %lf %d %d %d %d", &cfg.dim, &cfg.nx, &cfg.ny, &cfg.x0,
                  &cfg.x1, &cfg.y0, &cfg.y1, &cfg.gamma, &cfg.cfl, &cfg.bc[0], &cfg.bc[1], &cfg.bc[2],
                  &cfg.bc[3]) == 13;
  for (int s = 0; ok && s < 4; ++s)
    for (int q = 0; ok && q < 4; ++q) ok = fscanf(f, "%lf", &cfg.inflow_prim[s][q]) == 1;
  ok = ok && fscanf(f, "%lf %lf %lf %lf %lf", &cfg.weno_eps, &cfg.tau_eps, &cfg.tau_C, &cfg.fixed_dt, &cfg.mu) == 5;
  if (ok && fscanf(f, "%d", &cfg.gauss_points) != 1) cfg.gauss_points = 2;
  else if (ok && fscanf(f, "%d", &cfg.recon_vars) != 1) cfg.recon_vars = CGKS_CONSERVATIVE;
  else if (ok && fscanf(f, "%d", &cfg.side_slopes) != 1) cfg.side_slopes = 0;
  else if (ok && fscanf(f, "%d", &cfg.tang_weno) != 1) cfg.tang_weno = 0;
  fclose(f);
  if (!ok) { fprintf(stderr, "cgks_run: malformed configuration %s\n", argv[1]); return 1; }
  cfg.storage = CGKS_FP64;
  const long steps = atol(argv[3]);
  const size_t n = cfg.dim == 2 ? (size_t)12 * cfg.ny * cfg.nx : (size_t)6 * cfg.nx;
  if (cfg.nx < 1 || (cfg.dim == 2 && cfg.ny < 1) || steps < 0) { fprintf(stderr, "cgks_run: bad sizes\n"); return 1; }

  double *fields = (double *)malloc(n * sizeof(double));
  if (!fields) { fprintf(stderr, "cgks_run: out of memory\n"); return 1; }
  f = fopen(argv[2], "rb");
  if (!f) { perror(argv[2]); free(fields); return 1; }
  const size_t got = fread(fields, sizeof(double), n, f);
  fclose(f);
  if (got != n) { fprintf(stderr, "cgks_run: %s holds %zu of %zu values\n", argv[2], got, n); free(fields); return 1; }

  cgks_ctx *ctx = NULL;
  int rc = cgks_create(&cfg, NULL, &ctx);
  if (rc) { free(fields); return fail("cgks_create", rc); }
  rc = cgks_set_state(ctx, fields, 0, 0.0);
  if (!rc) rc = cgks_run_steps(ctx, steps);
  double t = 0.0;
  long done = 0;
  if (!rc) rc = cgks_get_state(ctx, fields, 0, &t, &done);
  cgks_destroy(ctx);
  if (rc) { free(fields); return fail("stepping", rc); }

  f = fopen(argv[4], "wb");
  if (!f || fwrite(fields, sizeof(double), n, f) != n) {
    perror(argv[4]);
    if (f) fclose(f);
    free(fields);
    return 1;
  }
  fclose(f);
  free(fields);
  printf("t %.17g steps %ld\n", t, done);
  return 0;
}
