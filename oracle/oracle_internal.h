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

/* one interface point; returns 1 when the equilibrium-state guard fired */
int orc_gks_point_g(int dim, double gamma, double tau_eps, double tau_C, double mu, double dt,
                    const double *W0, const double *W0n, const double *W0t,
                    const double *W0nn, const double *W0nt, const double *W0tt,
                    const double *Wl, const double *Wr,
                    double *F, double *Ft, double *Wt, double *Wtt,
                    double *Nh, double *Nf, double *tau, double *W0used);

#endif
