/*
 * cgks_oracle.h -- plain FP64 CPU oracle of the compact 8th-order gas-kinetic
 * scheme (Zhao, Ji, Shyy, Xu, "An acoustic and shock wave capturing compact
 * high-order gas-kinetic scheme with spectral-like resolution", arXiv 2001.01570).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant with the GPU
 * library, and the GPU library never calls it.
 *
 * Field layout (structure of arrays, x fastest): 1D has 6 fields
 *   [rho, rhoU, rhoE, (rho)_x, (rhoU)_x, (rhoE)_x]  each of length nx,
 * 2D has 12 fields
 *   [W(4), W_x(4), W_y(4)],  W = (rho, rhoU, rhoV, rhoE), each ny*nx.
 * W are cell averages, W_x / W_y cell-averaged gradients (Sec. 3.1).
 *
 * All arithmetic is IEEE double, compiled without contraction or fast-math.
 */
#ifndef CGKS_ORACLE_H
#define CGKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_FREE = 1, ORC_WALL = 2, ORC_INFLOW = 3, ORC_NOSLIP = 4 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENONPHYS = -4 };

typedef struct {
  int dim, nx, ny;
  double x0, x1, y0, y1, gamma, cfl;
  int bc[4];                 /* xlo, xhi, ylo, yhi */
  double inflow_prim[4][4];  /* (rho, U, V, p) per side with ORC_INFLOW */
  double weno_eps, tau_eps, tau_C;
  double fixed_dt;           /* 0 -> CFL rule, >0 -> fixed step */
  double mu;                 /* dynamic viscosity: 0 -> Euler, > 0 -> Navier-Stokes */
  int gauss_points;          /* 2D: Gauss-Legendre points per face segment, 2 (0 means 2;
                                3 segments with the tangential gradients) or 4 (sextic through
                                7 segment averages, three ghost layers) */
  int side_slopes;           /* slopes of the two non-equilibrium sides: 0 the linear
                                reconstruction's derivatives (the scheme as read); 1 (an
                                evaluated variant) the WENO-weighted derivatives of the
                                candidate polynomials of each side, in 2D taken to the
                                Gauss point like the normal derivative */
  int char_vars;             /* variables of the nonlinear (WENO-Z) reconstruction: 0
                                conservative, 1 characteristic (Sec. 3.2: the eigenvectors
                                of the normal flux Jacobian at the mean of the two cells
                                beside the face, per stencil line) */
  int tang_weno;             /* tangential assembly of the WENO-Z states (2D, conservative
                                variables, linear side slopes; an evaluated variant): 0 as
                                the linear quantities; 1 a WENO-Z of the three
                                average-interpolating quadratics on the five nearest
                                segments (orc_tang_weno, orc_tang_weno_eta) */
} orc_config;

typedef struct orc_ctx orc_ctx;

typedef struct {
  long steps;
  long guard_w0;     /* linear equilibrium state inadmissible -> kinetic state */
  long guard_weno;   /* WENO point state inadmissible -> adjacent cell average */
  double last_dt;
} orc_counters;

int  orc_create(const orc_config *cfg, orc_ctx **out);
void orc_destroy(orc_ctx *c);
int  orc_set_state(orc_ctx *c, const double *fields, double t0);
int  orc_get_state(const orc_ctx *c, double *fields, double *t, long *step);
double orc_cfl_dt(const orc_ctx *c);      /* CFL step of the current state (unclamped) */
int  orc_step(orc_ctx *c, double dt, double *dt_used);   /* dt<=0 -> rule in cfg */
int  orc_advance_to(orc_ctx *c, double t_end, long max_steps, long *steps_taken);
int  orc_counters_get(const orc_ctx *c, orc_counters *out);
long orc_last_bad_cell(const orc_ctx *c);
void orc_set_threads(int n);

/* ---- building blocks exposed for unit tests (scaled cell width h = 1) ---- */
/* Linear compact reconstruction at x_{i+1/2}, eq. (recons-8th-val):
 * Q[0..3] = Q_{i-1..i+2}, D[0..3] = h Q'_{i-1..i+2}; out = (P7, h P7_x, h^2 P7_xx). */
void orc_p7(const double *Q, const double *D, double *out);
/* Left WENO-Z value at x_{i+1/2} (Sec. 3.3): returns value; cand[7], beta[7],
 * weights[7] receive the candidate values, smoothness indicators and weights. */
double orc_weno_left(const double *Q, const double *D, double eps,
                     double *cand, double *beta, double *weights);
double orc_weno_right(const double *Q, const double *D, double eps);
/* The same with *dval = h * d/dx at x_{i+1/2} of the WENO combination of the
 * candidate polynomials (their slopes combined with the nonlinear weights). */
double orc_weno_left_d(const double *Q, const double *D, double eps, double *dval);
double orc_weno_right_d(const double *Q, const double *D, double eps, double *dval);
/* Moments <u^n v^m xi^(2k)> of a (half-)Maxwellian; half = 0 full, +1 u>0, -1 u<0. */
double orc_moment(int dim, double gamma, double U, double V, double lambda,
                  int half, int n, int m, int k);
/* Solve <psi a>_g = b for the expansion coefficients a of g (dim+2 unknowns). */
void orc_slope(int dim, double gamma, const double *W, const double *b, double *a);
/* Exact Euler second time derivative at a point (Cauchy-Kowalewski), 2D form:
 * inputs are conservative W and its first and second derivatives. */
void orc_euler_wtt(double gamma, const double *W, const double *Wx, const double *Wy,
                   const double *Wxx, const double *Wxy, const double *Wyy, double *Wtt);
/* One interface point of the gas-kinetic evolution (Sec. 2.1-2.2).
 * in: W0, W0_n, W0_t, W0_nn, W0_nt, W0_tt, Wl, Wr (dim+2 each, normal = x);
 * out: F[nc], Ft[nc], Wt[nc], Wtt[nc], N_half[nc], N_full[nc], tau. */
void orc_gks_point(int dim, double gamma, double tau_eps, double tau_C, double mu, double dt,
                   const double *W0, const double *W0n, const double *W0t,
                   const double *W0nn, const double *W0nt, const double *W0tt,
                   const double *Wl, const double *Wr,
                   double *F, double *Ft, double *Wt, double *Wtt,
                   double *Nh, double *Nf, double *tau);
/* orc_gks_point with the positivity guard of the equilibrium state reported:
 * returns 1 when W0 was inadmissible and the kinetic collision state of the
 * two sides took its place; W0used (nc) receives the state actually used.
 * Wln, Wrn: normal slopes of the two non-equilibrium sides (NULL: W0n, the
 * scheme as read). */
int orc_gks_point_g(int dim, double gamma, double tau_eps, double tau_C, double mu, double dt,
                    const double *W0, const double *W0n, const double *W0t,
                    const double *W0nn, const double *W0nt, const double *W0tt,
                    const double *Wl, const double *Wr,
                    double *F, double *Ft, double *Wt, double *Wtt,
                    double *Nh, double *Nf, double *tau, double *W0used,
                    const double *Wln, const double *Wrn);
/* One 1D face of a stage as the scheme evaluates it (Sec. 2.2, 3.2, 3.3), for
 * the face between cells 1 and 2 of a 4-cell line: cells[f * 4 + m] is field
 * f (the 6 fields of the 1D layout) of cell m.  The reference state of the
 * face is cell 1.  out (12): F, F_t, A, B in blocks of 3 -- A, B the stage's
 * interface-state terms (stage 1: at t + dt/2 and the stage-n part at
 * t + dt; stage 2, final = 1: W_tt and 0), as deviations from cell 1.
 * guards[0]: equilibrium-state guard fired (0/1); guards[1]: inadmissible
 * WENO point states replaced by the adjacent cell average (0..2). */
void orc_face_1d(const orc_config *cfg, const double *cells, double dt, int final,
                 double *out, long *guards);
/* Characteristic variables (Sec. 3.2).  orc_char_basis: right eigenvectors
 * R[i * nc + j] (component i of wave j; waves u - c, u (, u), u + c) of the
 * Jacobian of the Euler flux in the first direction at W, and L = R^-1 (row
 * major); -1 if W is not admissible.  orc_weno_char: the WENO-Z left and
 * right states of one line reconstructed in the characteristic variables of
 * Wm; Q[k * 4 + m], D[k * 4 + m] as for orc_weno_left per component k; the
 * states as deviations, per component; returns 0 (conservative variables
 * used) when Wm is not admissible, else 1. */
int orc_char_basis(int dim, double gamma, const double *W, double *L, double *R);
int orc_weno_char(int dim, double gamma, double eps, const double *Wm, const double *Q, const double *D,
                  double *wl, double *wr);
/* The same evolution evaluated as the time integral of the interface flux over
 * [0, delta]: Fhat(delta), with tau in the exponentials and tau_ce in the
 * Chapman-Enskog term (exposed for the extraction tests). */
void orc_flux_integral(int dim, double gamma, double tau, double tau_ce, double delta,
                       const double *W0, const double *W0n, const double *W0t,
                       const double *Wl, const double *Wr, double *Fhat);
/* The sextic through 7 unit-cell averages s[0..6] (offsets -3..3), at eta:
 * (value, d/deta, d2/deta2). */
void orc_sextic(const double *s, double eta, double *out3);
/* The quadratic through 3 unit-cell averages s[0..2] (offsets -1..1), at eta. */
void orc_quadratic3(const double *s, double eta, double *out3);
/* Point value at the first Gauss node eta = -1/(2 sqrt 3) (unit segment
 * width) from the averages s[0..4] of the segments -2..2: WENO-Z of the
 * three average-interpolating quadratics on segments (-2..0), (-1..1),
 * (0..2); the second node is reached by reversing s.  Test infrastructure:
 * the tangential-WENO variant of the 2D assembly. */
double orc_tang_weno(const double *s, double eps, double *cand, double *beta, double *weights);
/* The same at any node eta (the four-point nodes), linear weights from the
 * quartic through the five averages. */
double orc_tang_weno_eta(const double *s, double eta, double eps, double *cand, double *beta, double *weights);
/* The quintic fixed by 3 unit-cell averages s[0..2] (offsets -1..1) and by the
 * averages of its derivative over the same cells, d[0..2] (for a unit cell the
 * average of the derivative is the difference of the end values), at eta:
 * (value, d/deta, d2/deta2). */
void orc_hermite3(const double *s, const double *d, double eta, double *out3);
/* The cubic through the averages a[0..3] of 4 unit cells, cells 1 and 2 on
 * either side of eta = 1/2 (the cells of the normal stencil of a face): its
 * value and first derivative at the face. */
void orc_cubic_face(const double *a, double *out2);

#ifdef __cplusplus
}
#endif
#endif
