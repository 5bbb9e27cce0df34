/* Internal declarations of the oracle (test infrastructure only). */
#ifndef CGKS_ORACLE_INTERNAL_H
#define CGKS_ORACLE_INTERNAL_H

int orc_solve(int n, double *A, double *b);
int orc_invert(int n, const double *A, double *Ainv);
void orc_recon_init(void);

/* Moments of a Maxwellian g = rho (lambda/pi)^((K+d)/2) exp(-lambda((u-U)^2 + (v-V)^2 + xi^2)),
 * normalised by rho: mu[n] = <u^n> (full space or one half space), mv[n] = <v^n>,
 * mx[k] = <xi^(2k)>. */
typedef struct {
  int dim;
  double K, rho, U, V, lam;
  double mu[9], mv[9], mx[3];
} orc_maxw;

/* Returns 0, or -1 when W is not an admissible state (rho<=0, p<=0, non-finite). */
int orc_maxw_init(int dim, double gamma, const double *W, int half, orc_maxw *g);
int orc_admissible(int dim, double gamma, const double *W);
double orc_pressure(int dim, double gamma, const double *W);

#endif
