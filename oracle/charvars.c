/*
 * charvars.c -- characteristic variables of the Euler equations for the
 * nonlinear reconstruction (Sec. 3.2: the cell averages and slopes that the
 * compact reconstruction acts on may be conservative or characteristic
 * variables).  Part of the oracle: TEST INFRASTRUCTURE ONLY.
 *
 * The characteristic variables of a line are the coordinates of the
 * conservative variables in the right eigenvectors of the Jacobian of the
 * Euler flux normal to the face, evaluated at one reference state per face
 * and line (the mean of the two cells beside the face).  The linear
 * reconstruction P7 commutes with the constant change of variables, so only
 * the WENO-Z states change: project, reconstruct each characteristic
 * component, project back.
 */
#include <math.h>

#include "cgks_oracle.h"
#include "oracle_internal.h"

/* The flux Jacobian A = dF/dW of the Euler equations in the direction of the
 * first velocity component has, at a state with velocity (u, v), sound speed
 * c and total enthalpy H, the eigenvalues u - c, u (once per further
 * velocity component), u + c with right eigenvectors (columns)
 *   u - c : (1, u - c, v, H - u c)
 *   u     : (1, u, v, (u^2 + v^2)/2)
 *   u     : (0, 0, 1, v)                      (2D only)
 *   u + c : (1, u + c, v, H + u c)
 * (1D: drop the v component and the shear wave).  With g = gamma - 1,
 * q2 = u^2 + v^2 and b = g / c^2 the rows of the inverse are
 *   ( b q2/4 + u/(2c), -b u/2 - 1/(2c), -b v/2, b/2 )
 *   ( 1 - b q2/2,       b u,             b v,   -b  )
 *   ( -v,               0,               1,      0  )   (2D only)
 *   ( b q2/4 - u/(2c), -b u/2 + 1/(2c), -b v/2, b/2 ). */
int orc_char_basis(int dim, double gamma, const double *W, double *L, double *R) {
  if (!orc_admissible(dim, gamma, W)) return -1;
  const int nc = dim + 2;
  const double rho = W[0];
  const double u = W[1] / rho;
  const double v = dim == 2 ? W[2] / rho : 0.0;
  const double p = orc_pressure(dim, gamma, W);
  const double c = sqrt(gamma * p / rho);
  const double H = (W[nc - 1] + p) / rho;
  const double q2 = u * u + v * v;
  const double b = (gamma - 1.0) / (c * c);
  for (int i = 0; i < nc * nc; ++i) { L[i] = 0.0; R[i] = 0.0; }
  const int e = nc - 1;          /* energy row / column */
  const int a = nc - 1;          /* the u + c wave */
  /* right eigenvectors: R[i * nc + j], component i of wave j */
  R[0 * nc + 0] = 1.0; R[1 * nc + 0] = u - c; R[e * nc + 0] = H - u * c;
  R[0 * nc + 1] = 1.0; R[1 * nc + 1] = u;     R[e * nc + 1] = 0.5 * q2;
  R[0 * nc + a] = 1.0; R[1 * nc + a] = u + c; R[e * nc + a] = H + u * c;
  if (dim == 2) {
    R[2 * nc + 0] = v; R[2 * nc + 1] = v; R[2 * nc + a] = v;
    R[2 * nc + 2] = 1.0; R[e * nc + 2] = v;
  }
  /* left eigenvectors: L[j * nc + i], row j */
  L[0 * nc + 0] = 0.25 * b * q2 + 0.5 * u / c;
  L[0 * nc + 1] = -0.5 * b * u - 0.5 / c;
  L[0 * nc + e] = 0.5 * b;
  L[1 * nc + 0] = 1.0 - 0.5 * b * q2;
  L[1 * nc + 1] = b * u;
  L[1 * nc + e] = -b;
  L[a * nc + 0] = 0.25 * b * q2 - 0.5 * u / c;
  L[a * nc + 1] = -0.5 * b * u + 0.5 / c;
  L[a * nc + e] = 0.5 * b;
  if (dim == 2) {
    L[0 * nc + 2] = -0.5 * b * v;
    L[1 * nc + 2] = b * v;
    L[a * nc + 2] = -0.5 * b * v;
    L[2 * nc + 0] = -v;
    L[2 * nc + 2] = 1.0;
  }
  return 0;
}

/* The WENO-Z left and right states of one line in characteristic variables.
 * Q[k * 4 + m]: component k of cell m (cells i-1..i+2) minus the face's
 * reference state (cell i), D[k * 4 + m] = h times its normal derivative;
 * Wm: the reference state of the change of variables (the mean of cells i
 * and i+1).  Writes the states (as deviations from cell i) to wl, wr and
 * returns 1; when Wm is not admissible the line keeps the conservative
 * variables (wl, wr componentwise) and 0 is returned. */
int orc_weno_char(int dim, double gamma, double eps, const double *Wm, const double *Q, const double *D,
                  double *wl, double *wr) {
  const int nc = dim + 2;
  double L[16], R[16];
  if (orc_char_basis(dim, gamma, Wm, L, R) != 0) {
    for (int k = 0; k < nc; ++k) {
      wl[k] = orc_weno_left(Q + 4 * k, D + 4 * k, eps, 0, 0, 0);
      wr[k] = orc_weno_right(Q + 4 * k, D + 4 * k, eps);
    }
    return 0;
  }
  double cl[4], cr[4];
  for (int j = 0; j < nc; ++j) {
    double q[4], d[4];
    for (int m = 0; m < 4; ++m) {
      q[m] = 0.0;
      d[m] = 0.0;
      for (int k = 0; k < nc; ++k) {
        q[m] += L[j * nc + k] * Q[k * 4 + m];
        d[m] += L[j * nc + k] * D[k * 4 + m];
      }
    }
    cl[j] = orc_weno_left(q, d, eps, 0, 0, 0);
    cr[j] = orc_weno_right(q, d, eps);
  }
  for (int k = 0; k < nc; ++k) {
    wl[k] = 0.0;
    wr[k] = 0.0;
    for (int j = 0; j < nc; ++j) {
      wl[k] += R[k * nc + j] * cl[j];
      wr[k] += R[k * nc + j] * cr[j];
    }
  }
  return 1;
}
