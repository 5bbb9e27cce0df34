/* Compact reconstructions of Sec. 3 (test infrastructure only, see cgks_oracle.h).
 *
 * Coordinates are scaled by the cell width h: cell I_i is [-1/2, 1/2], the
 * stencil cells I_{i-1}, I_i, I_{i+1}, I_{i+2} are indexed 0..3, the interface
 * x_{i+1/2} sits at 1/2.  Q[m] are cell averages, D[m] = h Q'_m cell-averaged
 * slopes times h (so D[m] = q(right edge) - q(left edge) for the cell's
 * polynomial).
 */
#include <math.h>
#include <string.h>
#include "oracle_internal.h"
#include "cgks_oracle.h"

/* Eq. (recons-8th-val): value, h*d/dx and h^2*d2/dx2 of P^7 at x_{i+1/2}. */
void orc_p7(const double *Q, const double *D, double *out) {
  out[0] = (25.0 * Q[0] + 185.0 * Q[1] + 185.0 * Q[2] + 25.0 * Q[3]
            + 6.0 * D[0] + 102.0 * D[1] - 102.0 * D[2] - 6.0 * D[3]) / 420.0;
  out[1] = (-14.0 * Q[0] - 270.0 * Q[1] + 270.0 * Q[2] + 14.0 * Q[3]
            - 3.0 * D[0] - 99.0 * D[1] - 99.0 * D[2] - 3.0 * D[3]) / 108.0;
  out[2] = (-4.0 * Q[0] + 4.0 * Q[1] + 4.0 * Q[2] - 4.0 * Q[3]
            - D[0] - 9.0 * D[1] + 9.0 * D[2] + D[3]) / 4.0;
}

/* Candidate values q_k(x_{i+1/2}) of eq. (sub-stencil). */
static void candidates(const double *Q, const double *D, double *q) {
  q[0] = (-7.0 * Q[0] + 13.0 * Q[1] - 4.0 * D[0]) / 6.0;
  q[1] = (-Q[0] + 5.0 * Q[1] + 2.0 * Q[2]) / 6.0;
  q[2] = (5.0 * Q[1] + 32.0 * Q[2] - 13.0 * Q[3] + 6.0 * D[3]) / 24.0;
  q[3] = (-Q[0] + 5.0 * Q[1] + 2.0 * Q[2]) / 6.0;
  q[4] = (2.0 * Q[1] + 5.0 * Q[2] - Q[3]) / 6.0;
  q[5] = (10.0 * Q[0] + 19.0 * Q[1] + Q[2] + 3.0 * D[0] + 21.0 * D[1]) / 30.0;
  q[6] = (Q[1] + 19.0 * Q[2] + 10.0 * Q[3] - 21.0 * D[2] - 3.0 * D[3]) / 30.0;
}

/* Linear weights d_k of the 8th-order reconstruction (Sec. 3.3). */
static const double DK[7] = {3.0 / 98.0, 5.0 / 98.0, 4.0 / 49.0, 7.0 / 98.0,
                             7.0 / 98.0, 17.0 / 49.0, 17.0 / 49.0};

/* ---- smoothness indicators from their definition, eq. (smooth-indicator) ----
 * Each sub-stencil polynomial is built explicitly: its monomial coefficients on
 * I_i are the solution of the stencil's averaging/slope conditions (inverted
 * once), and beta = sum_r int_{I_i} (q^(r))^2 (h = 1 after scaling). */
typedef struct { int kind; int cell; } cond_t;   /* kind 0: average, 1: slope */
typedef struct { int deg; int n; cond_t c[5]; } stencil_t;

/* beta_0..beta_6 use S_0, S~_1 (cubic on Q_{i-1},Q_i,Q_{i+1},Q'_{i-1}, the
 * symmetric replacement of Sec. 3.3), S_2, S_3, S_4, S_5, S_6. */
static const stencil_t STENCIL[7] = {
  {2, 3, {{0, 0}, {0, 1}, {1, 0}}},
  {3, 4, {{0, 0}, {0, 1}, {0, 2}, {1, 0}}},
  {3, 4, {{0, 1}, {0, 2}, {0, 3}, {1, 3}}},
  {2, 3, {{0, 0}, {0, 1}, {0, 2}}},
  {2, 3, {{0, 1}, {0, 2}, {0, 3}}},
  {4, 5, {{0, 0}, {0, 1}, {0, 2}, {1, 0}, {1, 1}}},
  {4, 5, {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}}},
};
static double STENCIL_INV[7][25];
static double SEXTIC_INV[49];
static double QUADRATIC_INV[9];
static double HERMITE3_INV[36];
static double CUBIC_INV[16];
static int recon_ready = 0;

static double ipow(double x, int p) { double r = 1.0; for (int i = 0; i < p; ++i) r *= x; return r; }

static double cell_lo(int m) { return (double)m - 1.5; }   /* cell m spans [m-3/2, m-1/2] */

__attribute__((constructor)) void orc_recon_init(void) {
  if (recon_ready) return;
  for (int k = 0; k < 7; ++k) {
    const stencil_t *s = &STENCIL[k];
    double A[25];
    for (int r = 0; r < s->n; ++r) {
      double lo = cell_lo(s->c[r].cell), hi = lo + 1.0;
      for (int p = 0; p < s->n; ++p) {
        if (s->c[r].kind == 0) A[r * s->n + p] = (ipow(hi, p + 1) - ipow(lo, p + 1)) / (p + 1);
        else A[r * s->n + p] = ipow(hi, p) - ipow(lo, p);
      }
    }
    orc_invert(s->n, A, STENCIL_INV[k]);
  }
  {
    double B7[49];               /* cell r spans [r-7/2, r-5/2]: offsets -3..3 */
    for (int r = 0; r < 7; ++r) {
      double lo = r - 3.5, hi = r - 2.5;
      for (int p = 0; p < 7; ++p) B7[r * 7 + p] = (ipow(hi, p + 1) - ipow(lo, p + 1)) / (p + 1);
    }
    orc_invert(7, B7, SEXTIC_INV);
  }
  {
    /* quadratic through 3 averages on segments offsets -1..1 */
    double B3[9];
    for (int r = 0; r < 3; ++r) {
      double lo = r - 1.5, hi = r - 0.5;
      for (int p = 0; p < 3; ++p) B3[r * 3 + p] = (ipow(hi, p + 1) - ipow(lo, p + 1)) / (p + 1);
    }
    orc_invert(3, B3, QUADRATIC_INV);
  }
  {
    /* quintic fixed by the averages of the polynomial and of its derivative on
     * the segments at offsets -1..1: rows 0-2 average, rows 3-5 the average of
     * the derivative times the width, i.e. p(hi) - p(lo) */
    double H[36];
    for (int r = 0; r < 3; ++r) {
      double lo = r - 1.5, hi = r - 0.5;
      for (int p = 0; p < 6; ++p) {
        H[r * 6 + p] = (ipow(hi, p + 1) - ipow(lo, p + 1)) / (p + 1);
        H[(r + 3) * 6 + p] = ipow(hi, p) - ipow(lo, p);
      }
    }
    orc_invert(6, H, HERMITE3_INV);
  }
  {
    /* cubic through the averages of 4 unit cells spanning [m-3/2, m-1/2], m = 0..3 */
    double Cb[16];
    for (int r = 0; r < 4; ++r) {
      double lo = cell_lo(r), hi = lo + 1.0;
      for (int p = 0; p < 4; ++p) Cb[r * 4 + p] = (ipow(hi, p + 1) - ipow(lo, p + 1)) / (p + 1);
    }
    orc_invert(4, Cb, CUBIC_INV);
  }
  recon_ready = 1;
}

/* int_{-1/2}^{1/2} xi^p dxi */
static double mono_int(int p) {
  if (p % 2) return 0.0;
  return 2.0 * ipow(0.5, p + 1) / (p + 1);
}

static double falling(int m, int r) { double f = 1.0; for (int i = 0; i < r; ++i) f *= (m - i); return f; }

static double beta_of(int k, const double *Q, const double *D) {
  const stencil_t *s = &STENCIL[k];
  double rhs[5], coef[5];
  for (int r = 0; r < s->n; ++r) rhs[r] = s->c[r].kind == 0 ? Q[s->c[r].cell] : D[s->c[r].cell];
  for (int p = 0; p < s->n; ++p) {
    double acc = 0.0;
    for (int r = 0; r < s->n; ++r) acc += STENCIL_INV[k][p * s->n + r] * rhs[r];
    coef[p] = acc;
  }
  double beta = 0.0;
  for (int r = 1; r <= s->deg; ++r)
    for (int m = r; m <= s->deg; ++m)
      for (int mm = r; mm <= s->deg; ++mm)
        beta += coef[m] * coef[mm] * falling(m, r) * falling(mm, r) * mono_int(m + mm - 2 * r);
  return beta;
}

/* h * d/dx at x_{i+1/2} of the polynomial of candidate k (the sub-stencils of
 * eq. (sub-stencil); candidate 1 is the quadratic on Q_{i-1}, Q_i, Q_{i+1}, the
 * same polynomial as candidate 3). */
static double candidate_slope(int k, const double *Q, const double *D) {
  const int ks = k == 1 ? 3 : k;
  const stencil_t *s = &STENCIL[ks];
  double rhs[5];
  for (int r = 0; r < s->n; ++r) rhs[r] = s->c[r].kind == 0 ? Q[s->c[r].cell] : D[s->c[r].cell];
  double d = 0.0;
  for (int p = 1; p < s->n; ++p) {
    double acc = 0.0;
    for (int r = 0; r < s->n; ++r) acc += STENCIL_INV[ks][p * s->n + r] * rhs[r];
    d += acc * p * ipow(0.5, p - 1);
  }
  return d;
}

/* Left value of the WENO-Z reconstruction, eqs. (right-left), (WENO-Z-w), (tau).
 * The data are first shifted by Q_i: the reconstruction commutes with adding a
 * constant, and the shift keeps the indicators free of cancellation.  dval
 * (may be NULL): the candidates' slopes h * q_k'(x_{i+1/2}) combined with the
 * same nonlinear weights (the evaluated variant of the side slopes). */
static double weno_left_impl(const double *Qin, const double *D, double eps,
                             double *cand, double *beta, double *weights, double *dval) {
  double Q[4], q[7], b[7], w[7];
  const double ref = Qin[1];
  for (int m = 0; m < 4; ++m) Q[m] = Qin[m] - ref;
  candidates(Q, D, q);
  for (int k = 0; k < 7; ++k) b[k] = beta_of(k, Q, D);
  const double zref = fabs(3.0 * (b[0] - b[4]) + (b[4] - b[3]));
  double asum = 0.0;
  for (int k = 0; k < 7; ++k) { w[k] = DK[k] * (1.0 + zref / (b[k] + eps)); asum += w[k]; }
  double val = 0.0;
  for (int k = 0; k < 7; ++k) { w[k] /= asum; val += w[k] * q[k]; }
  if (dval) {
    double d = 0.0;
    for (int k = 0; k < 7; ++k) d += w[k] * candidate_slope(k, Q, D);
    *dval = d;
  }
  if (cand) for (int k = 0; k < 7; ++k) cand[k] = q[k] + ref;
  if (beta) memcpy(beta, b, sizeof b);
  if (weights) memcpy(weights, w, sizeof w);
  return val + ref;
}

double orc_weno_left(const double *Qin, const double *D, double eps,
                     double *cand, double *beta, double *weights) {
  return weno_left_impl(Qin, D, eps, cand, beta, weights, 0);
}

double orc_weno_left_d(const double *Q, const double *D, double eps, double *dval) {
  return weno_left_impl(Q, D, eps, 0, 0, 0, dval);
}

/* Right value at x_{i+1/2}: the left procedure applied to the stencil mirrored
 * about the interface (cells reversed, slopes negated); its slope changes sign
 * with the mirror. */
double orc_weno_right(const double *Q, const double *D, double eps) {
  double Qm[4], Dm[4];
  for (int m = 0; m < 4; ++m) { Qm[m] = Q[3 - m]; Dm[m] = -D[3 - m]; }
  return weno_left_impl(Qm, Dm, eps, 0, 0, 0, 0);
}

double orc_weno_right_d(const double *Q, const double *D, double eps, double *dval) {
  double Qm[4], Dm[4], d;
  for (int m = 0; m < 4; ++m) { Qm[m] = Q[3 - m]; Dm[m] = -D[3 - m]; }
  const double v = weno_left_impl(Qm, Dm, eps, 0, 0, 0, &d);
  *dval = -d;
  return v;
}

void orc_sextic(const double *s, double eta, double *out3) {
  double c[7];
  for (int p = 0; p < 7; ++p) {
    double acc = 0.0;
    for (int r = 0; r < 7; ++r) acc += SEXTIC_INV[p * 7 + r] * s[r];
    c[p] = acc;
  }
  double v = 0.0, d1 = 0.0, d2 = 0.0;
  for (int p = 0; p < 7; ++p) {
    v += c[p] * ipow(eta, p);
    if (p >= 1) d1 += c[p] * p * ipow(eta, p - 1);
    if (p >= 2) d2 += c[p] * p * (p - 1) * ipow(eta, p - 2);
  }
  out3[0] = v; out3[1] = d1; out3[2] = d2;
}


/* value, first and second derivative at eta of the polynomial whose monomial
 * coefficients are Minv * rhs (n unknowns) */
static void poly_eval(int n, const double *Minv, const double *rhs, double eta, double *out3) {
  double c[8];
  for (int p = 0; p < n; ++p) {
    double acc = 0.0;
    for (int r = 0; r < n; ++r) acc += Minv[p * n + r] * rhs[r];
    c[p] = acc;
  }
  double v = 0.0, d1 = 0.0, d2 = 0.0;
  for (int p = 0; p < n; ++p) {
    v += c[p] * ipow(eta, p);
    if (p >= 1) d1 += c[p] * p * ipow(eta, p - 1);
    if (p >= 2) d2 += c[p] * p * (p - 1) * ipow(eta, p - 2);
  }
  out3[0] = v; out3[1] = d1; out3[2] = d2;
}

void orc_quadratic3(const double *s, double eta, double *out3) {
  poly_eval(3, QUADRATIC_INV, s, eta, out3);
}

void orc_hermite3(const double *s, const double *d, double eta, double *out3) {
  const double rhs[6] = {s[0], s[1], s[2], d[0], d[1], d[2]};
  poly_eval(6, HERMITE3_INV, rhs, eta, out3);
}

void orc_cubic_face(const double *a, double *out2) {
  double o[3];
  poly_eval(4, CUBIC_INV, a, 0.5, o);
  out2[0] = o[0]; out2[1] = o[1];
}

/* Tangential WENO-Z of the WENO-Z states (the evaluated variant tang_weno):
 * each of the three quadratics has the segment averages A, B, C on the unit
 * segments centred at c - 1, c, c + 1 (c = -1, 0, 1):
 *   p(y) = B - (A - 2B + C)/24 + (C - A)/2 (y - c) + (A - 2B + C)/2 (y - c)^2,
 * its smoothness on the centre segment is the Jiang-Shu indicator of the
 * three averages, and the nonlinear weights have the form of the normal
 * reconstruction's WENO-Z (eq. WENO-Z-w) with tau = |beta_0 - beta_2|.  The
 * linear weights are the ones for which the combination equals the quartic
 * through the five averages at eta = -1/(2 sqrt 3): solving the five
 * coefficient equations gives 7/36 + sqrt(3)/1080, 11/18 and
 * 7/36 - sqrt(3)/1080 (all positive). */
double orc_tang_weno(const double *s, double eps, double *cand, double *beta, double *weights) {
  const double eta = -0.5 / sqrt(3.0);
  const double d[3] = {7.0 / 36.0 + sqrt(3.0) / 1080.0, 11.0 / 18.0, 7.0 / 36.0 - sqrt(3.0) / 1080.0};
  double q[3], b[3], w[3];
  for (int k = 0; k < 3; ++k) {
    const double A = s[k], B = s[k + 1], C = s[k + 2], y = eta - (k - 1.0);
    const double curv = A - 2.0 * B + C;
    q[k] = B - curv / 24.0 + 0.5 * (C - A) * y + 0.5 * curv * y * y;
  }
  {
    const double a0 = s[0] - 2.0 * s[1] + s[2], c0 = s[0] - 4.0 * s[1] + 3.0 * s[2];
    const double a1 = s[1] - 2.0 * s[2] + s[3], c1 = s[1] - s[3];
    const double a2 = s[2] - 2.0 * s[3] + s[4], c2 = 3.0 * s[2] - 4.0 * s[3] + s[4];
    b[0] = 13.0 / 12.0 * a0 * a0 + 0.25 * c0 * c0;
    b[1] = 13.0 / 12.0 * a1 * a1 + 0.25 * c1 * c1;
    b[2] = 13.0 / 12.0 * a2 * a2 + 0.25 * c2 * c2;
  }
  const double tau = fabs(b[0] - b[2]);
  double wsum = 0.0;
  for (int k = 0; k < 3; ++k) { w[k] = d[k] * (1.0 + tau / (b[k] + eps)); wsum += w[k]; }
  double v = 0.0;
  for (int k = 0; k < 3; ++k) {
    w[k] /= wsum;
    v += w[k] * q[k];
    if (cand) cand[k] = q[k];
    if (beta) beta[k] = b[k];
    if (weights) weights[k] = w[k];
  }
  return v;
}

/* The same WENO-Z at any node eta in (-1/2, 1/2) (the four-point nodes): the
 * linear weights follow from matching the quartic through the five averages
 * at eta, whose weight of each average comes from the inverse of the 5 x 5
 * matrix of the monomials' segment averages.  s_0 enters only the first
 * quadratic and s_4 only the third, which fixes d_0 and d_2; s_1 then fixes
 * d_1 (the other two equations hold by construction). */
double orc_tang_weno_eta(const double *s, double eta, double eps, double *cand, double *beta, double *weights) {
  double A[25], Ainv[25];
  for (int m = 0; m < 5; ++m)
    for (int p = 0; p < 5; ++p) {
      const double lo = m - 2.5, hi = m - 1.5;
      A[m * 5 + p] = (ipow(hi, p + 1) - ipow(lo, p + 1)) / (p + 1);
    }
  if (orc_invert(5, A, Ainv) != 0) return NAN;
  double P[5];   /* weight of average i in the quartic at eta */
  for (int i = 0; i < 5; ++i) {
    P[i] = 0.0;
    for (int p = 0; p < 5; ++p) P[i] += Ainv[p * 5 + i] * ipow(eta, p);
  }
  /* each quadratic's weights of its three averages (A, B, C) at eta */
  double qa[3], qb[3], qc[3];
  for (int k = 0; k < 3; ++k) {
    const double y = eta - (k - 1.0), w2 = -1.0 / 24.0 + 0.5 * y * y;
    qa[k] = w2 - 0.5 * y;
    qb[k] = 1.0 - 2.0 * w2;
    qc[k] = w2 + 0.5 * y;
  }
  double d[3];
  d[0] = P[0] / qa[0];
  d[2] = P[4] / qc[2];
  d[1] = (P[1] - d[0] * qb[0]) / qa[1];
  double q[3], b[3], w[3];
  for (int k = 0; k < 3; ++k) q[k] = qa[k] * s[k] + qb[k] * s[k + 1] + qc[k] * s[k + 2];
  {
    const double a0 = s[0] - 2.0 * s[1] + s[2], c0 = s[0] - 4.0 * s[1] + 3.0 * s[2];
    const double a1 = s[1] - 2.0 * s[2] + s[3], c1 = s[1] - s[3];
    const double a2 = s[2] - 2.0 * s[3] + s[4], c2 = 3.0 * s[2] - 4.0 * s[3] + s[4];
    b[0] = 13.0 / 12.0 * a0 * a0 + 0.25 * c0 * c0;
    b[1] = 13.0 / 12.0 * a1 * a1 + 0.25 * c1 * c1;
    b[2] = 13.0 / 12.0 * a2 * a2 + 0.25 * c2 * c2;
  }
  const double tau = fabs(b[0] - b[2]);
  double wsum = 0.0;
  for (int k = 0; k < 3; ++k) { w[k] = d[k] * (1.0 + tau / (b[k] + eps)); wsum += w[k]; }
  double v = 0.0;
  for (int k = 0; k < 3; ++k) {
    w[k] /= wsum;
    v += w[k] * q[k];
    if (cand) cand[k] = q[k];
    if (beta) beta[k] = b[k];
    if (weights) weights[k] = w[k];
  }
  return v;
}
