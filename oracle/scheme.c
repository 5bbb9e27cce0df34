/* The compact GKS time step in 1D and 2D (test infrastructure only, see
 * cgks_oracle.h): ghost cells, the two stages of the two-stage fourth-order
 * method for the cell averages (eq. step-hyper-1) and, along the same line,
 * for the interface states that update the cell-averaged gradients through
 * the Gauss theorem (eq. compact-deriv-1), and the CFL time step. */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle_internal.h"
#include "cgks_oracle.h"

struct orc_ctx {
  orc_config cfg;
  int nc, nf, gx, gy;
  int ng;                /* ghost layers: 2, or 3 for the 7-segment tangential stencil */
  int nl, npts;          /* 2D: tangential stencil lines (3 or 7) and Gauss points (2 or 4) */
  double dx, dy;
  double *U, *Us, *Un;   /* ghosted state, ghosted intermediate state, next state */
  double *P;             /* W + dt L + dt^2/6 L_t and the matching gradient part */
  double *xf, *yf;       /* per-face results, 4 blocks of nc */
  double t;
  long step, bad_cell;
  orc_counters cnt;
};

#define NF_FACE 4  /* blocks per face: F, Ft, A, B */

static int nthreads_req = 0;
void orc_set_threads(int n) { nthreads_req = n; }

static size_t fsize(const orc_ctx *c) { return (size_t)c->gx * c->gy; }
static double *fld(const orc_ctx *c, double *base, int f) { return base + (size_t)f * fsize(c); }
static size_t gidx(const orc_ctx *c, int i, int j) {
  return c->cfg.dim == 2 ? (size_t)(j + c->ng) * c->gx + (i + c->ng) : (size_t)(i + c->ng);
}

int orc_create(const orc_config *cfg, orc_ctx **out) {
  if (!cfg || !out) return ORC_EINVAL;
  if (cfg->dim != 1 && cfg->dim != 2) return ORC_EINVAL;
  if (cfg->nx < 1 || (cfg->dim == 2 && cfg->ny < 1)) return ORC_EINVAL;
  if (!(cfg->gamma > 1.0) || !(cfg->x1 > cfg->x0)) return ORC_EINVAL;
  if (cfg->dim == 2 && !(cfg->y1 > cfg->y0)) return ORC_EINVAL;
  for (int s = 0; s < 2 * cfg->dim; ++s) if (cfg->bc[s] < 0 || cfg->bc[s] > 4) return ORC_EINVAL;
  if ((cfg->bc[0] == ORC_PERIODIC) != (cfg->bc[1] == ORC_PERIODIC)) return ORC_EINVAL;
  if (cfg->dim == 2 && (cfg->bc[2] == ORC_PERIODIC) != (cfg->bc[3] == ORC_PERIODIC)) return ORC_EINVAL;
  if (!(cfg->mu >= 0.0) || !isfinite(cfg->mu)) return ORC_EINVAL;
  const int gp = cfg->gauss_points ? cfg->gauss_points : 2;
  if (cfg->side_slopes != 0 && cfg->side_slopes != 1) return ORC_EINVAL;
  if (cfg->char_vars != 0 && (cfg->char_vars != 1 || cfg->side_slopes)) return ORC_EINVAL;
  if (cfg->tang_weno != 0 && (cfg->tang_weno != 1 || cfg->dim != 2 || cfg->char_vars || cfg->side_slopes))
    return ORC_EINVAL;
  if (gp != 2 && !(gp == 4 && cfg->dim == 2)) return ORC_EINVAL;
  /* the 7-segment stencil reaches 3 cells across a side: a wall mirrors 3 cells */
  if (gp == 4)
    for (int s = 0; s < 4; ++s)
      if ((cfg->bc[s] == ORC_WALL || cfg->bc[s] == ORC_NOSLIP) && (s < 2 ? cfg->nx : cfg->ny) < 3) return ORC_EINVAL;
  orc_recon_init();
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof *c);
  if (!c) return ORC_ENOMEM;
  c->cfg = *cfg;
  if (cfg->dim == 1) c->cfg.ny = 1;
  c->nc = cfg->dim + 2;
  c->nf = cfg->dim == 2 ? 12 : 6;
  c->cfg.gauss_points = gp;
  c->npts = cfg->dim == 2 ? gp : 1;
  c->nl = gp == 4 ? 7 : (cfg->tang_weno ? 5 : 3);   /* tangential WENO: 5 segments */
  c->ng = gp == 4 ? 3 : 2;
  c->gx = c->cfg.nx + 2 * c->ng;
  c->gy = cfg->dim == 2 ? c->cfg.ny + 2 * c->ng : 1;
  c->dx = (cfg->x1 - cfg->x0) / cfg->nx;
  c->dy = cfg->dim == 2 ? (cfg->y1 - cfg->y0) / cfg->ny : 1.0;
  const size_t n = (size_t)c->nf * fsize(c);
  c->U = (double *)calloc(n, sizeof(double));
  c->Us = (double *)calloc(n, sizeof(double));
  c->Un = (double *)calloc(n, sizeof(double));
  c->P = (double *)calloc(n, sizeof(double));
  const size_t nxf = (size_t)(c->cfg.nx + 1) * c->cfg.ny * NF_FACE * c->nc;
  const size_t nyf = (size_t)c->cfg.nx * (c->cfg.ny + 1) * NF_FACE * c->nc;
  c->xf = (double *)calloc(nxf, sizeof(double));
  c->yf = cfg->dim == 2 ? (double *)calloc(nyf, sizeof(double)) : NULL;
  if (!c->U || !c->Us || !c->Un || !c->P || !c->xf || (cfg->dim == 2 && !c->yf)) {
    orc_destroy(c);
    return ORC_ENOMEM;
  }
  c->bad_cell = -1;
  *out = c;
  return ORC_OK;
}

void orc_destroy(orc_ctx *c) {
  if (!c) return;
  free(c->U); free(c->Us); free(c->Un); free(c->P); free(c->xf); free(c->yf);
  free(c);
}

int orc_set_state(orc_ctx *c, const double *fields, double t0) {
  const int nx = c->cfg.nx, ny = c->cfg.ny;
  for (int f = 0; f < c->nf; ++f)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        fld(c, c->U, f)[gidx(c, i, j)] = fields[((size_t)f * ny + j) * nx + i];
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double W[4];
      for (int k = 0; k < c->nc; ++k) W[k] = fld(c, c->U, k)[gidx(c, i, j)];
      if (!orc_admissible(c->cfg.dim, c->cfg.gamma, W)) { c->bad_cell = (long)j * nx + i; return ORC_ENONPHYS; }
    }
  c->t = t0;
  c->step = 0;
  return ORC_OK;
}

int orc_get_state(const orc_ctx *c, double *fields, double *t, long *step) {
  const int nx = c->cfg.nx, ny = c->cfg.ny;
  if (fields)
    for (int f = 0; f < c->nf; ++f)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
          fields[((size_t)f * ny + j) * nx + i] = fld(c, c->U, f)[gidx(c, i, j)];
  if (t) *t = c->t;
  if (step) *step = c->step;
  return ORC_OK;
}

int orc_counters_get(const orc_ctx *c, orc_counters *out) { *out = c->cnt; out->steps = c->step; return ORC_OK; }
long orc_last_bad_cell(const orc_ctx *c) { return c->bad_cell; }

/* ---- ghost cells (two layers) -------------------------------------------
 * periodic: wrap; free: copy the boundary cell average, zero gradients;
 * wall: mirror (normal momentum odd; the normal gradient has the opposite
 * parity of its variable, the tangential gradient the same); inflow: fixed
 * state with zero gradients.  x ghosts first, then y ghosts over all columns. */
static void inflow_state(const orc_ctx *c, int side, double *W) {
  const double *q = c->cfg.inflow_prim[side];
  const double g1 = c->cfg.gamma - 1.0;
  if (c->cfg.dim == 2) {
    W[0] = q[0]; W[1] = q[0] * q[1]; W[2] = q[0] * q[2];
    W[3] = q[3] / g1 + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2]);
  } else {
    W[0] = q[0]; W[1] = q[0] * q[1]; W[2] = q[3] / g1 + 0.5 * q[0] * q[1] * q[1];
  }
}

/* copy one ghost cell dst from src following the side's rule; axis 0 = x, 1 = y */
static void ghost_copy(orc_ctx *c, double *G, size_t dst, size_t src, int side, int axis) {
  const int nc = c->nc, bc = c->cfg.bc[side];
  if (bc == ORC_PERIODIC) {
    for (int f = 0; f < c->nf; ++f) fld(c, G, f)[dst] = fld(c, G, f)[src];
  } else if (bc == ORC_FREE) {
    for (int k = 0; k < nc; ++k) fld(c, G, k)[dst] = fld(c, G, k)[src];
    for (int f = nc; f < c->nf; ++f) fld(c, G, f)[dst] = 0.0;
  } else if (bc == ORC_INFLOW) {
    double W[4];
    inflow_state(c, side, W);
    for (int k = 0; k < nc; ++k) fld(c, G, k)[dst] = W[k];
    for (int f = nc; f < c->nf; ++f) fld(c, G, f)[dst] = 0.0;
  } else {  /* wall: mirror; slip wall: the normal momentum is odd, no-slip
             * (viscous, adiabatic) wall: both momenta are odd */
    const int vel = 1 + axis;     /* momentum component normal to the wall */
    for (int k = 0; k < nc; ++k) {
      const int odd = k == vel || (bc == ORC_NOSLIP && k >= 1 && k <= c->cfg.dim);
      const double par = odd ? -1.0 : 1.0;
      fld(c, G, k)[dst] = par * fld(c, G, k)[src];
      for (int a = 0; a < c->cfg.dim; ++a) {
        const double gpar = (a == axis) ? -par : par;
        fld(c, G, c->nc * (1 + a) + k)[dst] = gpar * fld(c, G, c->nc * (1 + a) + k)[src];
      }
    }
  }
}

static void fill_ghosts(orc_ctx *c, double *G) {
  const int nx = c->cfg.nx, ny = c->cfg.ny;
  for (int j = 0; j < ny; ++j)
    for (int k = 1; k <= c->ng; ++k) {
      int src_lo, src_hi;
      switch (c->cfg.bc[0]) {
        case ORC_PERIODIC: src_lo = ((-k) % nx + nx) % nx; break;
        case ORC_WALL: case ORC_NOSLIP: src_lo = k - 1 < nx ? k - 1 : nx - 1; break;
        default: src_lo = 0;
      }
      switch (c->cfg.bc[1]) {
        case ORC_PERIODIC: src_hi = (nx - 1 + k) % nx; break;
        case ORC_WALL: case ORC_NOSLIP: src_hi = nx - k >= 0 ? nx - k : 0; break;
        default: src_hi = nx - 1;
      }
      ghost_copy(c, G, gidx(c, -k, j), gidx(c, src_lo, j), 0, 0);
      ghost_copy(c, G, gidx(c, nx - 1 + k, j), gidx(c, src_hi, j), 1, 0);
    }
  if (c->cfg.dim == 1) return;
  for (int i = -c->ng; i < nx + c->ng; ++i)
    for (int k = 1; k <= c->ng; ++k) {
      int src_lo, src_hi;
      switch (c->cfg.bc[2]) {
        case ORC_PERIODIC: src_lo = ((-k) % ny + ny) % ny; break;
        case ORC_WALL: case ORC_NOSLIP: src_lo = k - 1 < ny ? k - 1 : ny - 1; break;
        default: src_lo = 0;
      }
      switch (c->cfg.bc[3]) {
        case ORC_PERIODIC: src_hi = (ny - 1 + k) % ny; break;
        case ORC_WALL: case ORC_NOSLIP: src_hi = ny - k >= 0 ? ny - k : 0; break;
        default: src_hi = ny - 1;
      }
      ghost_copy(c, G, gidx(c, i, -k), gidx(c, i, src_lo), 2, 1);
      ghost_copy(c, G, gidx(c, i, ny - 1 + k), gidx(c, i, src_hi), 3, 1);
    }
}

/* ---- CFL (Sec. 4): dt = CFL * min over cells of min(dx/(|U|+c), dy/(|V|+c)) */
double orc_cfl_dt(const orc_ctx *c) {
  const int nx = c->cfg.nx, ny = c->cfg.ny, dim = c->cfg.dim;
  double lmax = 0.0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double W[4];
      for (int k = 0; k < c->nc; ++k) W[k] = fld(c, c->U, k)[gidx(c, i, j)];
      const double p = orc_pressure(dim, c->cfg.gamma, W);
      const double snd = sqrt(c->cfg.gamma * p / W[0]);
      double l = (fabs(W[1] / W[0]) + snd) / c->dx;
      if (dim == 2) {
        const double ly = (fabs(W[2] / W[0]) + snd) / c->dy;
        if (ly > l) l = ly;
      }
      if (l > lmax) lmax = l;
    }
  return c->cfg.cfl / lmax;
}

/* ---- one face: normal reconstruction of 5 stencil lines, tangential
 * reconstruction to the Gauss points, gas-kinetic evolution at each point -- */

/* Normal reconstruction on one line (Sec. 3.2, 3.3): Q shifted by the face's
 * reference state, D = h Q'.  Output: P7, P7_n, P7_nn, left and right values. */
static void normal_line(const double *Q, const double *D, double h, double eps, double *o5, double *sd) {
  double p[3];
  orc_p7(Q, D, p);
  o5[0] = p[0];
  o5[1] = p[1] / h;
  o5[2] = p[2] / (h * h);
  if (sd) {   /* the side-slope variant: the WENO-weighted slopes of both sides too */
    double dl, dr;
    o5[3] = orc_weno_left_d(Q, D, eps, &dl);
    o5[4] = orc_weno_right_d(Q, D, eps, &dr);
    sd[0] = dl / h;
    sd[1] = dr / h;
  } else {
    o5[3] = orc_weno_left(Q, D, eps, 0, 0, 0);
    o5[4] = orc_weno_right(Q, D, eps);
  }
}

static void swap12(double *v) { double t = v[1]; v[1] = v[2]; v[2] = t; }

/* All components of one stencil line.  Q[k][m], D[k][m]: component k of cell
 * m (cells i-1..i+2 of the line, face between i and i+1) as the deviation
 * from the face's reference state and h times the normal derivative.
 * o5[q][k]: the normal_line outputs of component k; sd[s][k] the side slopes
 * of the evaluated variant (sd != NULL).  With characteristic variables the
 * WENO-Z states are reconstructed in the characteristic variables of the
 * mean Wm of cells i and i+1 (rot: y face, whose normal momentum is
 * component 2). */
static void line_all(const orc_config *cfg, int nc, double Q[4][4], double D[4][4], double h, const double *Wm,
                     int rot, double o5[5][4], double (*sd)[4]) {
  for (int k = 0; k < nc; ++k) {
    double o[5], s2[2] = {0.0, 0.0};
    normal_line(Q[k], D[k], h, cfg->weno_eps, o, sd ? s2 : 0);
    for (int q = 0; q < 5; ++q) o5[q][k] = o[q];
    if (sd) { sd[0][k] = s2[0]; sd[1][k] = s2[1]; }
  }
  if (cfg->char_vars) {
    double Qc[16], Dc[16], Wr[4], wl[4], wr[4];
    const int dim = nc - 2;
    for (int k = 0; k < nc; ++k) {
      Wr[k] = Wm[k];
      for (int m = 0; m < 4; ++m) { Qc[4 * k + m] = Q[k][m]; Dc[4 * k + m] = D[k][m]; }
    }
    if (rot) {
      swap12(Wr);
      for (int m = 0; m < 4; ++m) {
        double t = Qc[4 + m]; Qc[4 + m] = Qc[8 + m]; Qc[8 + m] = t;
        t = Dc[4 + m]; Dc[4 + m] = Dc[8 + m]; Dc[8 + m] = t;
      }
    }
    orc_weno_char(dim, cfg->gamma, cfg->weno_eps, Wr, Qc, Dc, wl, wr);
    if (rot) { swap12(wl); swap12(wr); }
    for (int k = 0; k < nc; ++k) { o5[3][k] = wl[k]; o5[4][k] = wr[k]; }
  }
}

typedef struct { long w0, weno; } guards_t;

/* Evaluate one face.  lines[l][q][c]: stencil line l (tangential offset
 * l - nl/2, only l=0 used in 1D), quantity q (P7, P7_n, P7_nn, W_l, W_r),
 * component c; the value quantities are deviations from ref.  tg[l][q][c]:
 * the line's tangential gradient reconstructed across the face from the
 * cells' own tangential gradients, q = 0 its value at the face, q = 1 its
 * normal derivative.  rot: y-face (swap momenta).  Writes F, Ft, A, B
 * (blocks of nc) averaged over the Gauss points with the Gauss-Legendre
 * weights.
 *
 * Tangential assembly (the 2D algorithm figure of Sec. 3 is not in the text):
 * the face sees the cells' cell-averaged tangential gradients, which the
 * compact scheme carries beside the averages.  Two Gauss points: every
 * quantity comes from the three nearest segments, the value quantities (and
 * the normal derivative) by the quintic that matches their segment averages
 * and the segment averages of their tangential derivative, W_nn by the
 * quadratic through its segment averages.  Four Gauss points: the sextic
 * through 7 segment averages for the values and the first derivatives; W_nt
 * and W_tt, which enter only the second time derivative, from the quintics
 * of the three nearest segments as with two points. */
static void face_eval(orc_ctx *c, double lines[7][5][4], double tg[7][2][4], const double *ref,
                      const double *Wleft, const double *Wright, double dt, int final, int rot, double ht,
                      double (*ss)[2][4], double *out, guards_t *gd) {
  const int dim = c->cfg.dim, nc = c->nc;
  const double gam = c->cfg.gamma;
  const int npts = c->npts, nl = c->nl;
  /* Gauss-Legendre nodes and weights on the segment [-1/2, 1/2] (weights sum to 1) */
  double eta[4], wgt[4];
  if (npts == 4) {
    const double a = 0.5 * sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double b = 0.5 * sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double wa = (18.0 + sqrt(30.0)) / 72.0, wb = (18.0 - sqrt(30.0)) / 72.0;
    eta[0] = -b; eta[1] = -a; eta[2] = a; eta[3] = b;
    wgt[0] = wb; wgt[1] = wa; wgt[2] = wa; wgt[3] = wb;
  } else if (npts == 2) {
    eta[0] = -0.5 / sqrt(3.0); eta[1] = 0.5 / sqrt(3.0);
    wgt[0] = wgt[1] = 0.5;
  } else {
    eta[0] = 0.0; wgt[0] = 1.0;
  }
  for (int k = 0; k < NF_FACE * nc; ++k) out[k] = 0.0;
  for (int g = 0; g < npts; ++g) {
    double W0d[4], W0[4], Wn[4], Wt_[4], Wnn[4], Wnt[4], Wtt_[4], Wl[4], Wr[4];
    for (int k = 0; k < nc; ++k) {
      if (dim == 2 && (nl == 3 || nl == 5)) {
        /* two points: the three nearest segments (with the tangential WENO
         * variant, nl = 5, the middle three of the five) */
        const int o = nl == 5;
        double s[3], d[3], dn[3], r3[3];
        for (int l = 0; l < 3; ++l) { d[l] = ht * tg[l + o][0][k]; dn[l] = ht * tg[l + o][1][k]; }
        for (int l = 0; l < 3; ++l) s[l] = lines[l + o][0][k];
        orc_hermite3(s, d, eta[g], r3);
        W0d[k] = r3[0]; Wt_[k] = r3[1] / ht; Wtt_[k] = r3[2] / (ht * ht);
        for (int l = 0; l < 3; ++l) s[l] = lines[l + o][1][k];
        orc_hermite3(s, dn, eta[g], r3);
        Wn[k] = r3[0]; Wnt[k] = r3[1] / ht;
        for (int l = 0; l < 3; ++l) s[l] = lines[l + o][2][k];
        orc_quadratic3(s, eta[g], r3);
        Wnn[k] = r3[0];
        if (nl == 5) {
          /* tangential WENO-Z of the five segments' states at the node (the
           * second node: the segments in reverse order) */
          double s5[5];
          for (int l = 0; l < 5; ++l) s5[l] = lines[g == 0 ? l : 4 - l][3][k];
          Wl[k] = ref[k] + orc_tang_weno(s5, c->cfg.weno_eps, 0, 0, 0);
          for (int l = 0; l < 5; ++l) s5[l] = lines[g == 0 ? l : 4 - l][4][k];
          Wr[k] = ref[k] + orc_tang_weno(s5, c->cfg.weno_eps, 0, 0, 0);
        } else {
          for (int l = 0; l < 3; ++l) s[l] = lines[l][3][k];
          orc_hermite3(s, d, eta[g], r3);
          Wl[k] = ref[k] + r3[0];
          for (int l = 0; l < 3; ++l) s[l] = lines[l][4][k];
          orc_hermite3(s, d, eta[g], r3);
          Wr[k] = ref[k] + r3[0];
        }
      } else if (dim == 2) {
        double s[7], r3[3], d[3];
        for (int l = 0; l < nl; ++l) s[l] = lines[l][0][k];
        orc_sextic(s, eta[g], r3);
        W0d[k] = r3[0]; Wt_[k] = r3[1] / ht;
        for (int l = 0; l < nl; ++l) s[l] = lines[l][1][k];
        orc_sextic(s, eta[g], r3);
        Wn[k] = r3[0];
        /* the tangential derivatives that enter only the second time
         * derivative come from the three nearest segments, as with two points */
        for (int l = 0; l < 3; ++l) { s[l] = lines[l + 2][0][k]; d[l] = ht * tg[l + 2][0][k]; }
        orc_hermite3(s, d, eta[g], r3);
        Wtt_[k] = r3[2] / (ht * ht);
        for (int l = 0; l < 3; ++l) { s[l] = lines[l + 2][1][k]; d[l] = ht * tg[l + 2][1][k]; }
        orc_hermite3(s, d, eta[g], r3);
        Wnt[k] = r3[1] / ht;
        for (int l = 0; l < nl; ++l) s[l] = lines[l][2][k];
        orc_sextic(s, eta[g], r3);
        Wnn[k] = r3[0];
        if (c->cfg.tang_weno) {
          /* the tangential-WENO variant: the middle five of the seven segments */
          double s5[5];
          for (int l = 0; l < 5; ++l) s5[l] = lines[l + 1][3][k];
          Wl[k] = ref[k] + orc_tang_weno_eta(s5, eta[g], c->cfg.weno_eps, 0, 0, 0);
          for (int l = 0; l < 5; ++l) s5[l] = lines[l + 1][4][k];
          Wr[k] = ref[k] + orc_tang_weno_eta(s5, eta[g], c->cfg.weno_eps, 0, 0, 0);
        } else {
          for (int l = 0; l < nl; ++l) s[l] = lines[l][3][k];
          orc_sextic(s, eta[g], r3);
          Wl[k] = ref[k] + r3[0];
          for (int l = 0; l < nl; ++l) s[l] = lines[l][4][k];
          orc_sextic(s, eta[g], r3);
          Wr[k] = ref[k] + r3[0];
        }
      } else {
        W0d[k] = lines[0][0][k]; Wn[k] = lines[0][1][k]; Wnn[k] = lines[0][2][k];
        Wl[k] = ref[k] + lines[0][3][k]; Wr[k] = ref[k] + lines[0][4][k];
        Wt_[k] = Wnt[k] = Wtt_[k] = 0.0;
      }
      W0[k] = ref[k] + W0d[k];
    }
    /* side slopes of the evaluated variant: the WENO-weighted slopes of each
     * line (ss[l][side][k]), in 2D taken to the point like the normal
     * derivative Wn (two points: the quintic of the three nearest segments
     * with the same tangential-derivative data; four points: the sextic
     * through the 7 segments); a side that falls back to the cell average
     * takes the linear slope */
    double Wln[4], Wrn[4];
    if (ss) {
      for (int k = 0; k < nc; ++k) {
        if (dim == 2 && nl == 3) {
          double sl[3], sr[3], dn[3], r3[3];
          for (int l = 0; l < 3; ++l) { sl[l] = ss[l][0][k]; sr[l] = ss[l][1][k]; dn[l] = ht * tg[l][1][k]; }
          orc_hermite3(sl, dn, eta[g], r3);
          Wln[k] = r3[0];
          orc_hermite3(sr, dn, eta[g], r3);
          Wrn[k] = r3[0];
        } else if (dim == 2) {
          double sl[7], sr[7], r3[3];
          for (int l = 0; l < nl; ++l) { sl[l] = ss[l][0][k]; sr[l] = ss[l][1][k]; }
          orc_sextic(sl, eta[g], r3);
          Wln[k] = r3[0];
          orc_sextic(sr, eta[g], r3);
          Wrn[k] = r3[0];
        } else {
          Wln[k] = ss[0][0][k];
          Wrn[k] = ss[0][1][k];
        }
      }
    }
    /* inadmissible nonlinear states fall back to the adjacent cell average */
    if (!orc_admissible(dim, gam, Wl)) {
      for (int k = 0; k < nc; ++k) { Wl[k] = Wleft[k]; Wln[k] = Wn[k]; }
      gd->weno++;
    }
    if (!orc_admissible(dim, gam, Wr)) {
      for (int k = 0; k < nc; ++k) { Wr[k] = Wright[k]; Wrn[k] = Wn[k]; }
      gd->weno++;
    }
    if (rot) {
      swap12(W0); swap12(Wn); swap12(Wt_); swap12(Wnn); swap12(Wnt); swap12(Wtt_);
      swap12(Wl); swap12(Wr); swap12(Wln); swap12(Wrn);
    }
    double F[4], Ft[4], Wt[4], Wtt[4], Nh[4], Nf[4], tau, W0u[4];
    const int fired = orc_gks_point_g(dim, gam, c->cfg.tau_eps, c->cfg.tau_C, c->cfg.mu, dt, W0, Wn, Wt_, Wnn,
                                      Wnt, Wtt_, Wl, Wr, F, Ft, Wt, Wtt, Nh, Nf, &tau, W0u,
                                      ss ? Wln : 0, ss ? Wrn : 0);
    if (rot) { swap12(F); swap12(Ft); swap12(Wt); swap12(Wtt); swap12(Nh); swap12(Nf); swap12(W0u); }
    if (fired) { gd->w0++; for (int k = 0; k < nc; ++k) W0d[k] = W0u[k] - ref[k]; }
    const double wg = wgt[g];
    for (int k = 0; k < nc; ++k) {
      double A, B;
      if (!final) {
        /* interface state at t + dt/2 and the stage-n part of the state at t + dt (Sec. 2.2) */
        A = W0d[k] + 0.5 * dt * Wt[k] + dt * dt / 8.0 * Wtt[k] + Nh[k];
        B = W0d[k] + dt * Wt[k] + dt * dt / 6.0 * Wtt[k] + Nf[k];
      } else {
        A = Wtt[k];
        B = 0.0;
      }
      out[k] += wg * F[k];
      out[nc + k] += wg * Ft[k];
      out[2 * nc + k] += wg * A;
      out[3 * nc + k] += wg * B;
    }
  }
}

void orc_face_1d(const orc_config *cfg, const double *cells, double dt, int final,
                 double *out, long *guards) {
  orc_ctx c;
  memset(&c, 0, sizeof c);
  c.cfg = *cfg;
  c.cfg.dim = 1;
  c.nc = 3;
  c.npts = 1;
  c.nl = 1;
  orc_recon_init();
  const double h = (cfg->x1 - cfg->x0) / cfg->nx;
  double ref[4] = {0, 0, 0, 0}, Wlc[4] = {0, 0, 0, 0}, Wrc[4] = {0, 0, 0, 0};
  double lines[7][5][4], tg[7][2][4], ss[1][2][4] = {{{0}}};
  memset(tg, 0, sizeof tg);
  double Q[4][4], D[4][4], Wm[4], o5[5][4];
  for (int k = 0; k < 3; ++k) {
    ref[k] = Wlc[k] = cells[k * 4 + 1];
    Wrc[k] = cells[k * 4 + 2];
    Wm[k] = 0.5 * (Wlc[k] + Wrc[k]);
    for (int m = 0; m < 4; ++m) {
      Q[k][m] = cells[k * 4 + m] - ref[k];
      D[k][m] = h * cells[(3 + k) * 4 + m];
    }
  }
  line_all(cfg, 3, Q, D, h, Wm, 0, o5, cfg->side_slopes ? ss[0] : 0);
  for (int q = 0; q < 5; ++q)
    for (int k = 0; k < 3; ++k) lines[0][q][k] = o5[q][k];
  guards_t gd = {0, 0};
  face_eval(&c, lines, tg, ref, Wlc, Wrc, dt, final, 0, 1.0, cfg->side_slopes ? ss : 0, out, &gd);
  guards[0] = gd.w0;
  guards[1] = gd.weno;
}

/* all faces of one stage on the ghosted state G */
static void stage_faces(orc_ctx *c, const double *G, double dt, int final, guards_t *gd_total) {
  const int nx = c->cfg.nx, ny = c->cfg.ny, nc = c->nc, dim = c->cfg.dim;
  long gw0 = 0, gwe = 0;
  /* x faces: face f between cells f-1 and f, reference = cell f-1 of the same row */
#pragma omp parallel for schedule(dynamic) reduction(+ : gw0, gwe) if (nthreads_req != 1 && ny > 1)
  for (int j = 0; j < ny; ++j) {
    guards_t gd = {0, 0};
    for (int f = 0; f <= nx; ++f) {
      double ref[4], Wlc[4], Wrc[4], lines[7][5][4], tg[7][2][4], ss[7][2][4];
      const int side = c->cfg.side_slopes;
      for (int k = 0; k < nc; ++k) {
        ref[k] = fld(c, (double *)G, k)[gidx(c, f - 1, j)];
        Wlc[k] = ref[k];
        Wrc[k] = fld(c, (double *)G, k)[gidx(c, f, j)];
      }
      const int nl = dim == 2 ? c->nl : 1;
      for (int l = 0; l < nl; ++l) {
        const int jj = dim == 2 ? j + l - nl / 2 : 0;
        double Q[4][4], D[4][4], Wm[4], o5[5][4];
        for (int k = 0; k < nc; ++k) {
          const double *Gk = fld(c, (double *)G, k);
          for (int m = 0; m < 4; ++m) {
            Q[k][m] = Gk[gidx(c, f - 2 + m, jj)] - ref[k];
            D[k][m] = c->dx * fld(c, (double *)G, nc + k)[gidx(c, f - 2 + m, jj)];
          }
          Wm[k] = 0.5 * (Gk[gidx(c, f - 1, jj)] + Gk[gidx(c, f, jj)]);
        }
        line_all(&c->cfg, nc, Q, D, c->dx, Wm, 0, o5, side ? ss[l] : 0);
        for (int k = 0; k < nc; ++k) {
          for (int q = 0; q < 5; ++q) lines[l][q][k] = o5[q][k];
          if (dim == 2) {
            double T[4], o2[2];
            for (int m = 0; m < 4; ++m) T[m] = fld(c, (double *)G, 2 * nc + k)[gidx(c, f - 2 + m, jj)];
            orc_cubic_face(T, o2);
            tg[l][0][k] = o2[0];
            tg[l][1][k] = o2[1] / c->dx;
          }
        }
      }
      double *out = c->xf + ((size_t)j * (nx + 1) + f) * NF_FACE * nc;
      face_eval(c, lines, tg, ref, Wlc, Wrc, dt, final, 0, c->dy, side ? ss : 0, out, &gd);
    }
    gw0 += gd.w0; gwe += gd.weno;
  }
  if (dim == 2) {
    /* y faces: face f between cells (i, f-1) and (i, f), reference = cell (i, f-1) */
#pragma omp parallel for schedule(dynamic) reduction(+ : gw0, gwe) if (nthreads_req != 1)
    for (int f = 0; f <= ny; ++f) {
      guards_t gd = {0, 0};
      for (int i = 0; i < nx; ++i) {
        double ref[4], Wlc[4], Wrc[4], lines[7][5][4], tg[7][2][4], ss[7][2][4];
        const int side = c->cfg.side_slopes;
        for (int k = 0; k < nc; ++k) {
          ref[k] = fld(c, (double *)G, k)[gidx(c, i, f - 1)];
          Wlc[k] = ref[k];
          Wrc[k] = fld(c, (double *)G, k)[gidx(c, i, f)];
        }
        for (int l = 0; l < c->nl; ++l) {
          const int ii = i + l - c->nl / 2;
          double Q[4][4], D[4][4], Wm[4], o5[5][4];
          for (int k = 0; k < nc; ++k) {
            const double *Gk = fld(c, (double *)G, k);
            for (int m = 0; m < 4; ++m) {
              Q[k][m] = Gk[gidx(c, ii, f - 2 + m)] - ref[k];
              D[k][m] = c->dy * fld(c, (double *)G, 2 * nc + k)[gidx(c, ii, f - 2 + m)];
            }
            Wm[k] = 0.5 * (Gk[gidx(c, ii, f - 1)] + Gk[gidx(c, ii, f)]);
          }
          line_all(&c->cfg, nc, Q, D, c->dy, Wm, 1, o5, side ? ss[l] : 0);
          for (int k = 0; k < nc; ++k) {
            double T[4], o2[2];
            for (int q = 0; q < 5; ++q) lines[l][q][k] = o5[q][k];
            for (int m = 0; m < 4; ++m) T[m] = fld(c, (double *)G, nc + k)[gidx(c, ii, f - 2 + m)];
            orc_cubic_face(T, o2);
            tg[l][0][k] = o2[0];
            tg[l][1][k] = o2[1] / c->dy;
          }
        }
        double *out = c->yf + ((size_t)f * nx + i) * NF_FACE * nc;
        face_eval(c, lines, tg, ref, Wlc, Wrc, dt, final, 1, c->dx, side ? ss : 0, out, &gd);
      }
      gw0 += gd.w0; gwe += gd.weno;
    }
  }
  gd_total->w0 += gw0;
  gd_total->weno += gwe;
}

/* Cell updates.  Stage 1 (final = 0): W* = W + dt/2 L + dt^2/8 L_t and the
 * partial P = W + dt L + dt^2/6 L_t (eq. step-hyper-1); gradients of the
 * intermediate state from the interface states at t + dt/2 by the Gauss
 * theorem (eq. compact-deriv-1), and their stage-n partial.
 * Stage 2 (final = 1): W^{n+1} = P + dt^2/3 L_t*, gradients likewise with
 * the second time derivative of the interface state at t*. */
static void stage_update(orc_ctx *c, const double *G, double dt, int final, double *dst) {
  const int nx = c->cfg.nx, ny = c->cfg.ny, nc = c->nc, dim = c->cfg.dim;
  const int B = NF_FACE * nc;
#pragma omp parallel for if (nthreads_req != 1 && ny > 1)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double *xl = c->xf + ((size_t)j * (nx + 1) + i) * B;
      const double *xr = xl + B;
      const double *yl = dim == 2 ? c->yf + ((size_t)j * nx + i) * B : NULL;
      const double *yr = dim == 2 ? c->yf + ((size_t)(j + 1) * nx + i) * B : NULL;
      const size_t id = gidx(c, i, j);
      for (int k = 0; k < nc; ++k) {
        double L = -(xr[k] - xl[k]) / c->dx;
        double Lt = -(xr[nc + k] - xl[nc + k]) / c->dx;
        if (dim == 2) {
          L += -(yr[k] - yl[k]) / c->dy;
          Lt += -(yr[nc + k] - yl[nc + k]) / c->dy;
        }
        const double W = fld(c, (double *)G, k)[id];
        /* the x-face values carry deviations from their left cells:
         * W(x_{i+1/2}) - W(x_{i-1/2}) = dev_{i+1/2} - dev_{i-1/2} + (W_i - W_{i-1}) */
        const double jx = W - fld(c, (double *)G, k)[gidx(c, i - 1, j)];
        const double jy = dim == 2 ? W - fld(c, (double *)G, k)[gidx(c, i, j - 1)] : 0.0;
        if (!final) {
          fld(c, dst, k)[id] = W + 0.5 * dt * L + dt * dt / 8.0 * Lt;
          fld(c, c->P, k)[id] = W + dt * L + dt * dt / 6.0 * Lt;
          fld(c, dst, nc + k)[id] = ((xr[2 * nc + k] - xl[2 * nc + k]) + jx) / c->dx;
          fld(c, c->P, nc + k)[id] = ((xr[3 * nc + k] - xl[3 * nc + k]) + jx) / c->dx;
          if (dim == 2) {
            fld(c, dst, 2 * nc + k)[id] = ((yr[2 * nc + k] - yl[2 * nc + k]) + jy) / c->dy;
            fld(c, c->P, 2 * nc + k)[id] = ((yr[3 * nc + k] - yl[3 * nc + k]) + jy) / c->dy;
          }
        } else {
          fld(c, dst, k)[id] = fld(c, c->P, k)[id] + dt * dt / 3.0 * Lt;
          fld(c, dst, nc + k)[id] = fld(c, c->P, nc + k)[id]
                                    + dt * dt / 3.0 * (xr[2 * nc + k] - xl[2 * nc + k]) / c->dx;
          if (dim == 2)
            fld(c, dst, 2 * nc + k)[id] = fld(c, c->P, 2 * nc + k)[id]
                                          + dt * dt / 3.0 * (yr[2 * nc + k] - yl[2 * nc + k]) / c->dy;
        }
      }
    }
}

static long first_bad(const orc_ctx *c, const double *G) {
  for (int j = 0; j < c->cfg.ny; ++j)
    for (int i = 0; i < c->cfg.nx; ++i) {
      double W[4];
      for (int k = 0; k < c->nc; ++k) W[k] = fld(c, (double *)G, k)[gidx(c, i, j)];
      if (!orc_admissible(c->cfg.dim, c->cfg.gamma, W)) return (long)j * c->cfg.nx + i;
    }
  return -1;
}

int orc_step(orc_ctx *c, double dt, double *dt_used) {
#ifdef _OPENMP
  if (nthreads_req > 0) omp_set_num_threads(nthreads_req);
#endif
  if (!(dt > 0.0)) dt = c->cfg.fixed_dt > 0.0 ? c->cfg.fixed_dt : orc_cfl_dt(c);
  if (!(dt > 0.0) || !isfinite(dt)) return ORC_EINVAL;
  guards_t gd = {0, 0};
  fill_ghosts(c, c->U);
  stage_faces(c, c->U, dt, 0, &gd);
  stage_update(c, c->U, dt, 0, c->Us);
  long bad = first_bad(c, c->Us);
  if (bad >= 0) { c->bad_cell = bad; return ORC_ENONPHYS; }
  fill_ghosts(c, c->Us);
  stage_faces(c, c->Us, dt, 1, &gd);
  stage_update(c, c->Us, dt, 1, c->Un);
  bad = first_bad(c, c->Un);
  if (bad >= 0) { c->bad_cell = bad; return ORC_ENONPHYS; }
  double *t = c->U; c->U = c->Un; c->Un = t;
  c->t += dt;
  c->step += 1;
  c->cnt.guard_w0 += gd.w0;
  c->cnt.guard_weno += gd.weno;
  c->cnt.last_dt = dt;
  if (dt_used) *dt_used = dt;
  return ORC_OK;
}

/* Advance to t_end: each step uses the CFL (or fixed) step, the last one is
 * clamped so that the run lands on t_end exactly. */
int orc_advance_to(orc_ctx *c, double t_end, long max_steps, long *steps_taken) {
  long n = 0;
  int rc = ORC_OK;
  while (c->t < t_end && (max_steps <= 0 || n < max_steps)) {
    double dt = c->cfg.fixed_dt > 0.0 ? c->cfg.fixed_dt : orc_cfl_dt(c);
    int last = 0;
    /* a step that reaches t_end to within round-off of the time sum is the last */
    if (dt * (1.0 + 1e-9) >= t_end - c->t) { dt = t_end - c->t; last = 1; }
    rc = orc_step(c, dt, NULL);
    if (rc) break;
    if (last) c->t = t_end;
    ++n;
  }
  if (steps_taken) *steps_taken = n;
  return rc;
}
