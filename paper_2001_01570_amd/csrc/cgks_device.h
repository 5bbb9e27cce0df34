// Device arithmetic of the compact 8th-order gas-kinetic scheme for gfx950.
//
// Sec. 3.2-3.3 (compact linear and WENO-Z reconstruction), Sec. 2.1-2.2
// (gas-kinetic interface evolution, flux extraction, interface state) of
// Zhao, Ji, Shyy, Xu, arXiv 2001.01570.  All FP64.
//
// Data along one reconstruction line are shifted by the average of the cell
// left of the interface (Q_i): the reconstructions commute with adding a
// constant, and the shift keeps every derivative-type quantity and every
// smoothness indicator free of cancellation against the O(1) background.
#pragma once
#include <hip/hip_runtime.h>

// device functions are also host-callable so that their arithmetic can be
// exercised on the CPU
#define CGKS_HD __host__ __device__

// Register-pressure controls of the face-point evaluation (no effect on the
// arithmetic; no-ops on the host):
//   CGKS_PIN(x)   materialise x here (the compiler may not sink the arithmetic
//                 that produces it towards its later uses)
//   CGKS_BREAK()  compiler memory barrier + scheduling barrier: LDS values are
//                 re-read after it instead of being held in registers
#if defined(__HIP_DEVICE_COMPILE__)
#define CGKS_PIN(x) asm volatile("" : "+v"(x))
#define CGKS_BREAK()                    \
  do {                                  \
    asm volatile("" ::: "memory");      \
    __builtin_amdgcn_sched_barrier(0);  \
  } while (0)
#else
#define CGKS_PIN(x) ((void)0)
#define CGKS_BREAK() ((void)0)
#endif

namespace cgks {

// Reciprocal: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (each step squares the relative error), within about an
// ulp of 1/x for finite nonzero x.  The host build divides.
CGKS_HD __forceinline__ double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

// ----------------------------------------------------------------------------
// compact reconstruction on one line, one component (scaled cell width h = 1)
// inputs (shifted by Q_i): a = Q_{i-1}-Q_i, c = Q_{i+1}-Q_i, d = Q_{i+2}-Q_i,
// A..D = h Q'_{i-1..i+2}
// ----------------------------------------------------------------------------

struct Line5 {       // outputs of the normal reconstruction of one component
  double v;          // P7 value at x_{i+1/2} (shifted)
  double vn;         // h * dP7/dx
  double vnn;        // h^2 * d2P7/dx2
  double wl, wr;     // WENO-Z left / right values (shifted)
};

// Eq. (recons-8th-val) with the constant part removed (coefficients of Q_i
// vanish in the derivatives; in the value 185 Q_i combines with the others to 420 Q_i).
CGKS_HD __forceinline__ void p7_shifted(double a, double c, double d, double A, double B,
                                           double C, double D, double& v, double& vn, double& vnn) {
  v = (25.0 * a + 185.0 * c + 25.0 * d + 6.0 * A + 102.0 * B - 102.0 * C - 6.0 * D) * (1.0 / 420.0);
  vn = (-14.0 * a + 270.0 * c + 14.0 * d - 3.0 * A - 99.0 * B - 99.0 * C - 3.0 * D) * (1.0 / 108.0);
  vnn = (-4.0 * a + 4.0 * c - 4.0 * d - A - 9.0 * B + 9.0 * C + D) * 0.25;
}

// Left WENO-Z value at x_{i+1/2}, eqs. (right-left), (sub-stencil), (WENO-Z-w),
// (smooth-indicator), (tau).  The indicators are written as sums of squares of
// the candidate polynomials' derivative coefficients on I_i = [-1/2, 1/2]:
//   quadratic   beta = k1^2 + 13/3 k2^2
//   cubic       beta = (k1 + k3/4)^2 + 13/3 k2^2 + 781/20 k3^2
//   quartic     beta = (k1 + k3/4)^2 + 13/3 (k2 + 63/130 k4)^2 + 781/20 k3^2 + 1421461/2275 k4^2
// (exact integrals of sum_r (q^(r))^2; beta_1 from the cubic on Q_{i-1}, Q_i,
// Q_{i+1}, Q'_{i-1}).
// SLOPE: also *slope = h times the derivative at x_{i+1/2} of the WENO
// combination of the candidate polynomials (their slopes with the same
// nonlinear weights; an evaluated variant of the non-equilibrium side
// slopes).  The candidates' interface slopes, from their stencil conditions
// (csrc/candidate_slopes.py): s0 = -3a - 2A, s1 = s3 = s4 = c,
// s2 = c/2 + 3d/8 - D/4, s5 = 3a/2 + c/2 + A/2 + 3B/2, s6 = 2c - 3d/2 + 3C/2 + D/2.
template <bool SLOPE>
CGKS_HD __forceinline__ double weno_left_s(double a, double c, double d, double A, double B,
                                           double C, double D, double eps, double* slope) {
  constexpr double S2 = 13.0 / 3.0, S3 = 781.0 / 20.0, S4 = 1421461.0 / 2275.0, L42 = 63.0 / 130.0;
  // candidate values q_k(x_{i+1/2}) with Q_i removed
  const double q0 = (-7.0 * a - 4.0 * A) * (1.0 / 6.0);
  const double q1 = (-a + 2.0 * c) * (1.0 / 6.0);       // q1 == q3
  const double q2 = (32.0 * c - 13.0 * d + 6.0 * D) * (1.0 / 24.0);
  const double q4 = (5.0 * c - d) * (1.0 / 6.0);
  const double q5 = (10.0 * a + c + 3.0 * A + 21.0 * B) * (1.0 / 30.0);
  const double q6 = (19.0 * c + 10.0 * d - 21.0 * C - 3.0 * D) * (1.0 / 30.0);
  double k1, k2, k3, k4, t;
  // beta_0: S0 = {Q_{i-1}, Q_i, Q'_{i-1}}
  k1 = -A - 2.0 * a; k2 = -A - a;
  const double b0 = k1 * k1 + S2 * k2 * k2;
  // beta_1: cubic on {Q_{i-1}, Q_i, Q_{i+1}, Q'_{i-1}}
  k1 = -0.625 * A - 1.4375 * a + 0.1875 * c; k2 = 0.5 * (a + c); k3 = 0.5 * A + 0.75 * a + 0.25 * c;
  t = k1 + 0.25 * k3;
  const double b1 = t * t + S2 * k2 * k2 + S3 * k3 * k3;
  // beta_2: cubic on {Q_i, Q_{i+1}, Q_{i+2}, Q'_{i+2}}
  k1 = 0.875 * D + 3.75 * c - 1.8125 * d; k2 = -1.5 * D - 4.0 * c + 2.75 * d; k3 = 0.5 * D + c - 0.75 * d;
  t = k1 + 0.25 * k3;
  const double b2 = t * t + S2 * k2 * k2 + S3 * k3 * k3;
  // beta_3: quadratic on {Q_{i-1}, Q_i, Q_{i+1}}
  k1 = 0.5 * (c - a); k2 = 0.5 * (a + c);
  const double b3 = k1 * k1 + S2 * k2 * k2;
  // beta_4: quadratic on {Q_i, Q_{i+1}, Q_{i+2}}
  k1 = 2.0 * c - 0.5 * d; k2 = -c + 0.5 * d;
  const double b4 = k1 * k1 + S2 * k2 * k2;
  // beta_5: quartic on {Q_{i-1}, Q_i, Q_{i+1}, Q'_{i-1}, Q'_i}
  k1 = 1.25 * B + 0.125 * (a - c); k2 = 0.75 * A + 1.5 * B + 2.375 * a + 0.125 * c;
  k3 = -B + 0.5 * (c - a); k4 = -0.5 * A - B - 1.25 * a + 0.25 * c;
  t = k1 + 0.25 * k3;
  double u = k2 + L42 * k4;
  const double b5 = t * t + S2 * u * u + S3 * k3 * k3 + S4 * k4 * k4;
  // beta_6: quartic on {Q_i, Q_{i+1}, Q_{i+2}, Q'_{i+1}, Q'_{i+2}}
  k1 = -2.75 * C - 0.5 * D + c + 1.625 * d; k2 = 7.5 * C + 2.25 * D + 3.5 * c - 6.625 * d;
  k3 = -5.0 * C - 2.0 * D - 4.0 * c + 5.5 * d; k4 = C + 0.5 * D + c - 1.25 * d;
  t = k1 + 0.25 * k3;
  u = k2 + L42 * k4;
  const double b6 = t * t + S2 * u * u + S3 * k3 * k3 + S4 * k4 * k4;
  // WENO-Z weights with the reference value of eq. (tau):
  //   alpha_k = d_k (1 + z / x_k),  x_k = beta_k + eps,  value = sum alpha_k q_k / sum alpha_k.
  // Numerator and denominator are both multiplied by P = prod_j x_j, so that
  // alpha_k becomes d_k (P + z P_k) with P_k = prod_{j != k} x_j (prefix times
  // suffix products) and one reciprocal remains.  (x_k >= eps keeps P far from
  // underflow; it overflows only for indicators beyond 1e40.)
  const double z = fabs(3.0 * (b0 - b4) + (b4 - b3));
  const double x0 = b0 + eps, x1 = b1 + eps, x2 = b2 + eps, x3 = b3 + eps, x4 = b4 + eps, x5 = b5 + eps,
               x6 = b6 + eps;
  const double l1 = x0, l2 = l1 * x1, l3 = l2 * x2, l4 = l3 * x3, l5 = l4 * x4, l6 = l5 * x5;
  const double r5 = x6, r4 = r5 * x5, r3 = r4 * x4, r2 = r3 * x3, r1 = r2 * x2, r0 = r1 * x1;
  const double P = l6 * x6;
  const double a0 = (3.0 / 98.0) * (P + z * r0);
  const double a1 = (5.0 / 98.0) * (P + z * (l1 * r1));
  const double a2 = (4.0 / 49.0) * (P + z * (l2 * r2));
  const double a3 = (7.0 / 98.0) * (P + z * (l3 * r3));
  const double a4 = (7.0 / 98.0) * (P + z * (l4 * r4));
  const double a5 = (17.0 / 49.0) * (P + z * (l5 * r5));
  const double a6 = (17.0 / 49.0) * (P + z * l6);
  const double num = a0 * q0 + (a1 + a3) * q1 + a2 * q2 + a4 * q4 + a5 * q5 + a6 * q6;
  const double den = a0 + a1 + a2 + a3 + a4 + a5 + a6;
  const double iden = recip(den);
  if constexpr (SLOPE) {
    const double s0 = -3.0 * a - 2.0 * A;
    const double s2 = 0.5 * c + 0.375 * d - 0.25 * D;
    const double s5 = 1.5 * a + 0.5 * c + 0.5 * A + 1.5 * B;
    const double s6 = 2.0 * c - 1.5 * d + 1.5 * C + 0.5 * D;
    *slope = (a0 * s0 + (a1 + a3 + a4) * c + a2 * s2 + a5 * s5 + a6 * s6) * iden;
  }
  return num * iden;
}

CGKS_HD __forceinline__ double weno_left(double a, double c, double d, double A, double B,
                                         double C, double D, double eps) {
  return weno_left_s<false>(a, c, d, A, B, C, D, eps, nullptr);
}

// Full normal reconstruction of one component on one line.  Q[0..3] are the
// averages of cells i-1..i+2 minus Q_i, D[0..3] = h Q'.  The right value is the
// left procedure on the stencil mirrored about the interface (cell i+1 becomes
// the reference there, hence the "+ c").
CGKS_HD __forceinline__ Line5 normal_line(double a, double c, double d, double A, double B,
                                             double C, double D, double eps) {
  Line5 r;
  p7_shifted(a, c, d, A, B, C, D, r.v, r.vn, r.vnn);
  r.wl = weno_left(a, c, d, A, B, C, D, eps);
  r.wr = weno_left(d - c, -c, a - c, -D, -C, -B, -A, eps) + c;
  return r;
}

// ----------------------------------------------------------------------------
// Characteristic variables (Sec. 3.2: the reconstruction may act on the
// conservative or on the characteristic variables).  Per line and face, the
// WENO-Z states are reconstructed in the coordinates of the right
// eigenvectors of the Jacobian of the Euler flux normal to the face at the
// mean of the two cells beside it; P7 is linear and needs no change.
// At a state W (normal momentum first) with velocity (u, v), sound speed c,
// total enthalpy H, q2 = u^2 + v^2 and b = (gamma - 1)/c^2 the waves
// u - c, u (2D: twice), u + c have the right eigenvectors (columns of R)
//   (1, u - c, v, H - u c), (1, u, v, q2/2), (0, 0, 1, v), (1, u + c, v, H + u c)
// and L = R^-1 has the rows
//   (b q2/4 + u/(2c), -b u/2 - 1/(2c), -b v/2, b/2),  (1 - b q2/2, b u, b v, -b),
//   (-v, 0, 1, 0),  (b q2/4 - u/(2c), -b u/2 + 1/(2c), -b v/2, b/2)
// (NC = 3: without v and the shear wave).  The scaling of the eigenvectors
// matters (the WENO-Z weights are not scale invariant): first entry 1, and
// the shear wave's v entry 1.  Returns false when W is not admissible; the
// line then keeps the conservative variables.
// ----------------------------------------------------------------------------
template <int NC>
CGKS_HD __forceinline__ bool char_basis(const double* W, double gamma, double (&L)[NC][NC], double (&R)[NC][NC]) {
  if (!(W[0] > 0.0)) return false;
  const double rho = W[0];
  const double u = W[1] / rho;
  const double v = NC == 4 ? W[2] / rho : 0.0;
  const double q2 = u * u + v * v;
  const double p = (gamma - 1.0) * (W[NC - 1] - 0.5 * rho * q2);
  if (!(p > 0.0) || !(p < INFINITY) || !(rho < INFINITY)) return false;
  const double c = sqrt(gamma * p / rho);
  const double H = (W[NC - 1] + p) / rho;
  const double b = (gamma - 1.0) / (c * c);
  const double hc = 0.5 / c;
  constexpr int E = NC - 1;   // energy component, and the u + c wave
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) { L[i][j] = 0.0; R[i][j] = 0.0; }
  R[0][0] = 1.0; R[1][0] = u - c; R[E][0] = H - u * c;
  R[0][1] = 1.0; R[1][1] = u;     R[E][1] = 0.5 * q2;
  R[0][E] = 1.0; R[1][E] = u + c; R[E][E] = H + u * c;
  L[0][0] = 0.25 * b * q2 + u * hc; L[0][1] = -0.5 * b * u - hc; L[0][E] = 0.5 * b;
  L[1][0] = 1.0 - 0.5 * b * q2;     L[1][1] = b * u;             L[1][E] = -b;
  L[E][0] = 0.25 * b * q2 - u * hc; L[E][1] = -0.5 * b * u + hc; L[E][E] = 0.5 * b;
  if constexpr (NC == 4) {
    R[2][0] = v; R[2][1] = v; R[2][E] = v; R[2][2] = 1.0; R[E][2] = v;
    L[0][2] = -0.5 * b * v; L[1][2] = b * v; L[E][2] = -0.5 * b * v;
    L[2][0] = -v; L[2][2] = 1.0;
  }
  return true;
}

// The WENO-Z left and right states of one line in characteristic variables:
// a, c, d (cells i-1, i+1, i+2 minus cell i) and A..D (h Q' of cells i-1..i+2)
// per component are projected with L, reconstructed per characteristic
// component (the right state mirrored as in normal_line) and projected back
// with R; wl, wr are deviations from cell i.
template <int NC>
CGKS_HD __forceinline__ void weno_char(const double (&L)[NC][NC], const double (&R)[NC][NC], const double* a,
                                       const double* c, const double* d, const double* A, const double* B,
                                       const double* C, const double* D, double eps, double* wl, double* wr) {
  double cl[NC], cr[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    double x[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      x[0] += L[j][k] * a[k];
      x[1] += L[j][k] * c[k];
      x[2] += L[j][k] * d[k];
      x[3] += L[j][k] * A[k];
      x[4] += L[j][k] * B[k];
      x[5] += L[j][k] * C[k];
      x[6] += L[j][k] * D[k];
    }
    cl[j] = weno_left(x[0], x[1], x[2], x[3], x[4], x[5], x[6], eps);
    cr[j] = weno_left(x[2] - x[1], -x[1], x[0] - x[1], -x[6], -x[5], -x[4], -x[3], eps) + x[1];
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double sl = 0.0, sr = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      sl += R[k][j] * cl[j];
      sr += R[k][j] * cr[j];
    }
    wl[k] = sl;
    wr[k] = sr;
  }
}

// The cells' tangential gradient g of the 4 stencil cells carried across the
// face by the cubic through their averages: ht T (value at the face) and
// ht TN (its normal derivative at unit normal width), times the tangential
// width ht (the data of the tangential fits are width x derivative).
CGKS_HD __forceinline__ void cross_face(double g0, double g1, double g2, double g3, double ht, double& hT,
                                        double& hTN) {
  hT = ht * ((7.0 * (g1 + g2) - (g0 + g3)) * (1.0 / 12.0));
  hTN = ht * ((15.0 * (g2 - g1) + (g0 - g3)) * (1.0 / 12.0));
}

// ----------------------------------------------------------------------------
// Tangential fits (2D).  A face segment sees the stencil lines of the
// neighbouring segments and, for each line, the cells' own tangential
// gradient carried across the face (the cubic through the 4 cells of the
// normal stencil: its value T and normal derivative TN at the face).
// Two Gauss points: every quantity at a point comes from the three nearest
// segments (offsets -1..1): the quintic that matches the segment averages s_l
// and the segment averages of the tangential derivative (data d_l = width
// times average derivative), or for W_nn the quadratic through the averages.
// Weights at the nodes eta = -+1/(2 sqrt 3) (unit width; the kernels use the
// first and reach the second by mirroring):
//   p(eta) = sum v_l s_l + vd_l d_l, p' = sum d1_l s_l + d1d_l d_l,
//   p'' = sum d2_l s_l + d2d_l d_l, quadratic(eta) = sum q_l s_l.
// The mirrored node reads the segments in reverse order; its derivative data
// then change sign.  Four Gauss points: the same quintics at the 4-point
// nodes give W_nt and W_tt (the sextic below gives the rest).  Weights from
// the exact inverse of the 6x6 (3x3) condition matrix evaluated at the nodes
// (csrc/tangential_weights.py).
// ----------------------------------------------------------------------------
struct HermWT { double v[3], vd[3], d1[3], d1d[3], d2[3], d2d[3], q[3]; };

#define CGKS_HERM2_WEIGHTS { \
  {{-0.07540507117498404449950279, 0.9944444444444444444444444, 0.08096062673053960005505834}, \
   {-0.01665330702328691625202201, -0.4089564406759849165273137, -0.01943108480106469402979979}, \
   {-0.6944086473878967252606736, 1.347150628109126783854680, -0.6527419807212300585940069}, \
   {-0.1993945341743196992808274, 0.9722222222222222222222222, 0.1855056452854308103919385}, \
   {4.886751345948128822545744, -4.0, -0.8867513459481288225457439}, \
   {1.173575314054563391927340, 4.426352063787130861236807, 0.1735753140545633919273402}, \
   {0.1443375672974064411272872, 1.0, -0.1443375672974064411272872}}, \
  {{0.08096062673053960005505834, 0.9944444444444444444444444, -0.07540507117498404449950279}, \
   {0.01943108480106469402979979, 0.4089564406759849165273137, 0.01665330702328691625202201}, \
   {0.6527419807212300585940069, -1.347150628109126783854680, 0.6944086473878967252606736}, \
   {0.1855056452854308103919385, 0.9722222222222222222222222, -0.1993945341743196992808274}, \
   {-0.8867513459481288225457439, -4.0, 4.886751345948128822545744}, \
   {-0.1735753140545633919273402, -4.426352063787130861236807, -1.173575314054563391927340}, \
   {-0.1443375672974064411272872, 1.0, 0.1443375672974064411272872}} \
}
// inner (-a) and outer (-b) nodes of the 4-point rule
#define CGKS_HERM4_WEIGHTS { \
  {{-0.1248240833561131699440749, 1.124426413335020227523364, 0.0003976700210929424207106109}, \
   {-0.03210351457762360623395334, -0.2660001747648614712891579, 0.002891414172850832756992869}, \
   {-0.1526899822820735562383774, 0.8303038958212636973409479, -0.6776139135391901411025705}, \
   {-0.06231166909995143542794097, 1.404385843338815739450934, 0.1828497570182522808412001}, \
   {4.165330030890955969267389, -4.653238670008856194497662, 0.4879086391179002252302731}, \
   {1.106222711005295206895935, 2.791595304766893427494077, -0.2203966239991328903528958}, \
   {0.05777698297917839142993050, 1.054436555834071349541472, -0.1122135388132497409714024}}, \
  {{0.07355769190377441281049170, 0.7667300492500137860820779, 0.1597122588462118011074304}, \
   {0.02308107005580096648563723, -0.4972776892026319862157708, -0.04252610359263265617877837}, \
   {-1.408829046621189383642094, 1.833550488515874427317954, -0.4247214418946850436758601}, \
   {-0.3560936766249800353899954, 0.2418726600625448047667532, 0.1301134118359308906570084}, \
   {5.034219542738118133817983, -2.775332758562572376930909, -2.258886784175545756887074}, \
   {0.9787827549958941217382635, 5.723207196203161835693985, 0.5911163757146079332728091}, \
   {0.2663118796250726281005321, 0.8979443965468810314109091, -0.1642562761719536595114412}} \
}
__constant__ static const HermWT kHerm2[2] = CGKS_HERM2_WEIGHTS;
__constant__ static const HermWT kHerm4[2] = CGKS_HERM4_WEIGHTS;

template <int NL>
struct TangWT { double v[NL], d1[NL], d2[NL]; };

// The sextic through 7 segment averages (offsets -3..3) at the 4-point
// Gauss-Legendre nodes eta = -a (inner) and -b (outer), a = 0.16999052179...,
// b = 0.43056815579...; the nodes +a, +b read the lines in reverse order
// (first-derivative weights with opposite sign).  Weights from the exact
// rational inverse of the 7x7 segment-average matrix evaluated at the nodes;
// Gauss weights (18 + sqrt 30)/72 (inner) and (18 - sqrt 30)/72 (outer) for
// an average over the segment.
#define CGKS_TANG7_WEIGHTS { \
  {{0.00327670662777140150320, -0.0266359260617751224288, 0.0928282644451935365246, 1.08046056237311464266, -0.183384586025290289167, 0.0375843394851378397702, -0.00412936084415200886592}, \
   {-0.0234994586764076403944, 0.217583386144768507063, -1.09415803665141890662, 0.524691359684989440382, 0.497541637759546521474, -0.139445386633782430552, 0.0172864983723045086499}, \
   {-0.00808539123755721195341, -0.0258058754040666686056, 1.39474441702196471283, -2.98922056750361979378, 1.97853482298309596974, -0.390843887097514794698, 0.0406764812376977864692}}, \
  {{0.00860109764472105523262, -0.0796691475531970354643, 0.415576982717297023337, 0.849155569794037932652, -0.245805403605616208498, 0.0591434746546156592307, -0.00700257365185842648992}, \
   {-0.0153298262005816740398, 0.170954211803748928533, -1.34141626702514246895, 1.21722202742076867842, -0.0133313609372416838971, -0.0221303941025073900877, 0.00403160904095561002241}, \
   {-0.0547477785057617936884, 0.399186600655063098459, 0.438830376399876995413, -2.22166378623787680486, 1.86135977135016436283, -0.480496021826951022910, 0.0575308381654851647508}}, \
}
__constant__ static const TangWT<7> kTang7[2] = CGKS_TANG7_WEIGHTS;
constexpr double kGauss4Inner = 0.326072577431273071313, kGauss4Outer = 0.173927422568726928687;

// ----------------------------------------------------------------------------
// erfc and exp near zero.  The half-space moments take erfc(-s sqrt(lambda) U)
// and exp(-lambda U^2); at low Mach numbers both arguments are small, where the
// Maclaurin series converge fast:
//   erf(x) = 2/sqrt(pi) sum_n (-1)^n x^(2n+1) / (n! (2n+1)),   |x| <= 1/2, n <= 11
//            (first omitted term < 3e-18, relative to erfc >= 0.47: < 6e-18)
//   exp(y) = sum_n y^n / n!,                                     |y| <= 1/4, n <= 13
//            (first omitted term < 5e-20)
// Larger arguments use the library functions.  The operation counter keeps the
// library calls (one transcendental each).
// ----------------------------------------------------------------------------
#ifndef CGKS_OPCOUNT
CGKS_HD __forceinline__ double erfc_moment(double x) {
  if (!(fabs(x) <= 0.5)) return erfc(x);
  // coefficients (-1)^n / (n! (2n+1)), Horner in x^2, times 2/sqrt(pi)
  constexpr double c[12] = {1.0,
                            -1.0 / 3.0,
                            1.0 / 10.0,
                            -1.0 / 42.0,
                            1.0 / 216.0,
                            -1.0 / 1320.0,
                            1.0 / 9360.0,
                            -1.0 / 75600.0,
                            1.0 / 685440.0,
                            -1.0 / 6894720.0,
                            1.0 / 76204800.0,
                            -1.0 / 918086400.0};
  const double x2 = x * x;
  double sum = c[11];
#pragma unroll
  for (int n = 10; n >= 0; --n) sum = sum * x2 + c[n];
  return 1.0 - 1.1283791670955125739 * x * sum;
}

CGKS_HD __forceinline__ double exp_moment(double y) {
  if (!(fabs(y) <= 0.25)) return exp(y);
  constexpr double c[14] = {1.0,           1.0,           1.0 / 2.0,         1.0 / 6.0,          1.0 / 24.0,
                            1.0 / 120.0,   1.0 / 720.0,   1.0 / 5040.0,      1.0 / 40320.0,      1.0 / 362880.0,
                            1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0};
  double sum = c[13];
#pragma unroll
  for (int n = 12; n >= 0; --n) sum = sum * y + c[n];
  return sum;
}
#else
CGKS_HD __forceinline__ double erfc_moment(double x) { return erfc(x); }
CGKS_HD __forceinline__ double exp_moment(double y) { return exp(y); }
#endif

// ----------------------------------------------------------------------------
// gas-kinetic evolution at one interface point (normal = first velocity
// component).  NC = 3 (1D: rho, rhoU, rhoE) or 4 (2D: rho, rhoU, rhoV, rhoE).
// ----------------------------------------------------------------------------

template <int NC> struct Vec { double c[NC]; };

struct Gas {
  double gamma, K;     // K: internal degrees of freedom (K + dim = 2/(gamma-1))
  double tau_eps, tau_C;
  double mu;           // dynamic viscosity; 0 for the Euler equations
  double inv_g1;       // 1/(gamma - 1)
  double inv_KD;       // 1/(K + dim)
};

// Gas constants of a problem of dimension dim.
CGKS_HD inline Gas make_gas(double gamma, int dim, double tau_eps, double tau_C, double mu) {
  Gas g;
  g.gamma = gamma;
  g.K = 2.0 / (gamma - 1.0) - dim;
  g.tau_eps = tau_eps;
  g.tau_C = tau_C;
  g.mu = mu;
  g.inv_g1 = 1.0 / (gamma - 1.0);
  g.inv_KD = 1.0 / (g.K + dim);
  return g;
}

// Moments of a (half-)Maxwellian normalised by rho: mu[n] = <u^n> n<=6,
// mv[m] = <v^m> m<=5 (2D), x1 = <xi^2>, x2 = <xi^4>.
template <int NC>
struct Mom {
  double rho, U, V, lam;
  double ir, h;         // 1/rho, 1/(2 lambda) = p/rho
  double mu[7];
  double mv[6];
  double x1, x2;
};

template <int NC>
CGKS_HD __forceinline__ double pressure(const double* W, double gamma) {
  const double ir = recip(W[0]);
  double ke = W[1] * W[1];
  if constexpr (NC == 4) ke += W[2] * W[2];
  return (gamma - 1.0) * (W[NC - 1] - 0.5 * ke * ir);
}

template <int NC>
CGKS_HD __forceinline__ bool admissible(const double* W, double gamma) {
  if (!(W[0] > 0.0)) return false;
  const double p = pressure<NC>(W, gamma);
  return p > 0.0 && p < INFINITY && W[0] < INFINITY;
}

// half: 0 full space, +1 u > 0, -1 u < 0
template <int NC>
CGKS_HD __forceinline__ void moments(const double* W, const Gas& g, int half, Mom<NC>& m) {
  m.rho = W[0];
  const double ir = recip(W[0]);
  m.ir = ir;
  m.U = W[1] * ir;
  m.V = (NC == 4) ? W[2] * ir : 0.0;
  const double p = pressure<NC>(W, g.gamma);
  m.lam = 0.5 * m.rho * recip(p);
  const double h = p * ir;        // 1/(2 lambda)
  m.h = h;
  if (half == 0) {
    m.mu[0] = 1.0;
    m.mu[1] = m.U;
  } else {
    const double s = (double)half;
    const double sl = sqrt(m.lam);
    m.mu[0] = 0.5 * erfc_moment(-s * sl * m.U);
    // 1/sqrt(lambda) = 2 h sqrt(lambda)
    m.mu[1] = m.U * m.mu[0] + s * exp_moment(-m.lam * m.U * m.U) * (0.56418958354775628695 * h * sl);
  }
#pragma unroll
  for (int n = 1; n < 6; ++n) m.mu[n + 1] = m.U * m.mu[n] + (double)n * h * m.mu[n - 1];
  if constexpr (NC == 4) {
    m.mv[0] = 1.0;
    m.mv[1] = m.V;
#pragma unroll
    for (int n = 1; n < 5; ++n) m.mv[n + 1] = m.V * m.mv[n] + (double)n * h * m.mv[n - 1];
  }
  m.x1 = g.K * h;
  m.x2 = (g.K * g.K + 2.0 * g.K) * h * h;
}

// Solve <psi a> = b for the expansion a = a0 + a1 u [+ a2 v] + a_e (u^2 [+ v^2] + xi^2)/2
// of a Maxwellian (closed-form inverse of the moment matrix).
template <int NC>
CGKS_HD __forceinline__ void slope(const Mom<NC>& m, const Gas& g, const double* b, double* a) {
  const double KD = g.K + (NC == 4 ? 2.0 : 1.0);   // = 2/(gamma-1)
  const double U = m.U, V = m.V, lam = m.lam;
  double q = U * U + KD * m.h;
  if constexpr (NC == 4) q += V * V;
  const double Re = 2.0 * b[NC - 1] - q * b[0];
  const double Ru = b[1] - U * b[0];
  if constexpr (NC == 4) {
    const double Rv = b[2] - V * b[0];
    a[3] = 4.0 * lam * lam * (Re - 2.0 * U * Ru - 2.0 * V * Rv) * g.inv_KD;
    a[2] = 2.0 * lam * Rv - V * a[3];
    a[1] = 2.0 * lam * Ru - U * a[3];
    a[0] = b[0] - U * a[1] - V * a[2] - 0.5 * a[3] * q;
  } else {
    a[2] = 4.0 * lam * lam * (Re - 2.0 * U * Ru) * g.inv_KD;
    a[1] = 2.0 * lam * Ru - U * a[2];
    a[0] = b[0] - U * a[1] - 0.5 * a[2] * q;
  }
}

// <u^n v^m psi a> for a Maxwellian (rho factor not included).
template <int NC>
CGKS_HD __forceinline__ void mom_psi_a(const Mom<NC>& M, int n, int m, const double* a, double* out) {
  auto E = [&](int p, int q) -> double {
    if constexpr (NC == 4) return M.mu[p] * M.mv[q]; else return q == 0 ? M.mu[p] : 0.0;
  };
  // <u^p v^q psi_e>, psi_e = (u^2 [+ v^2] + xi^2)/2
  auto H = [&](int p, int q) -> double {
    double s = E(p + 2, q) + E(p, q) * M.x1;
    if constexpr (NC == 4) s += E(p, q + 2);
    return 0.5 * s;
  };
  // <u^p v^q psi_e^2>
  auto Q = [&](int p, int q) -> double {
    double s = E(p + 4, q) + E(p, q) * M.x2 + 2.0 * E(p + 2, q) * M.x1;
    if constexpr (NC == 4) s += E(p, q + 4) + 2.0 * E(p + 2, q + 2) + 2.0 * E(p, q + 2) * M.x1;
    return 0.25 * s;
  };
  if constexpr (NC == 4) {
    out[0] = a[0] * E(n, m) + a[1] * E(n + 1, m) + a[2] * E(n, m + 1) + a[3] * H(n, m);
    out[1] = a[0] * E(n + 1, m) + a[1] * E(n + 2, m) + a[2] * E(n + 1, m + 1) + a[3] * H(n + 1, m);
    out[2] = a[0] * E(n, m + 1) + a[1] * E(n + 1, m + 1) + a[2] * E(n, m + 2) + a[3] * H(n, m + 1);
    out[3] = a[0] * H(n, m) + a[1] * H(n + 1, m) + a[2] * H(n, m + 1) + a[3] * Q(n, m);
  } else {
    out[0] = a[0] * E(n, 0) + a[1] * E(n + 1, 0) + a[2] * H(n, 0);
    out[1] = a[0] * E(n + 1, 0) + a[1] * E(n + 2, 0) + a[2] * H(n + 1, 0);
    out[2] = a[0] * H(n, 0) + a[1] * H(n + 1, 0) + a[2] * Q(n, 0);
  }
}

// <u^n v^m psi>
template <int NC>
CGKS_HD __forceinline__ void mom_psi(const Mom<NC>& M, int n, int m, double* out) {
  double one[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) one[k] = (k == 0) ? 1.0 : 0.0;
  mom_psi_a<NC>(M, n, m, one, out);
}

// Moments of the slope terms of one Maxwellian.  With the expansions
// a_n . psi and a_t . psi of the normal and tangential slopes, the slope
// polynomial P = u (a_n . psi) + v (a_t . psi) collects into
//   P = c_u u + c_uu u^2 + c_uv u v + c_v v + c_vv v^2 + A u e + B v e,
//   e = u^2 + v^2 + xi^2,  c_u = a_n0, c_uu = a_n1, c_uv = a_n2 + a_t1,
//   c_v = a_t0, c_vv = a_t2, A = a_n3 / 2, B = a_t3 / 2
// (1D: P = c_u u + c_uu u^2 + A u e, e = u^2 + xi^2).  Su = <u psi P>
// (always) and, with PSI, Sp = <psi P>, from the products
// E(a, b) = <u^a><v^b> of the moment table, each formed once, and the
// moments of e and e^2 (<xi^2> = x1, <xi^4> = x2; E(0, 0) = <u^0> is the mass
// fraction of a half space):
//   <u^a v^b e>   = E(a+2,b) + E(a,b+2) + x1 E(a,b),
//   <u^a v^b e^2> = E(a+4,b) + 2 E(a+2,b+2) + E(a,b+4) + 2 x1 (E(a+2,b) + E(a,b+2)) + x2 E(a,b).
// The same sums as mom_psi_a over the two slopes, with every product of the
// moment table formed once.
template <int NC, bool PSI>
CGKS_HD __forceinline__ void slope_moments(const Mom<NC>& M, const double* an, const double* at, double* Sp,
                                           double* Su) {
  const double* mu = M.mu;
  const double x1 = M.x1, x2 = M.x2;
  if constexpr (NC == 4) {
    const double* mv = M.mv;
    // the moment table (a >= 1, b >= 1)
    const double E11 = mu[1] * mv[1], E12 = mu[1] * mv[2], E13 = mu[1] * mv[3], E14 = mu[1] * mv[4];
    const double E21 = mu[2] * mv[1], E22 = mu[2] * mv[2], E23 = mu[2] * mv[3];
    const double E31 = mu[3] * mv[1], E32 = mu[3] * mv[2];
    const double E41 = mu[4] * mv[1];
    // <u^a v^b e>
    const double eM11 = fma(x1, E11, E31 + E13), eM20 = fma(x1, mu[2], mu[4] + E22);
    const double eM30 = fma(x1, mu[3], mu[5] + E32), eM21 = fma(x1, E21, E41 + E23);
    const double eM12 = fma(x1, E12, E32 + E14);
    const double eM10 = fma(x1, mu[1], mu[3] + E12);
    const double cu = an[0], cuu = an[1], cuv = an[2] + at[1], cv = at[0], cvv = at[2];
    const double A = 0.5 * an[3], B = 0.5 * at[3];
    // <u^a v^b P> = cu E(a+1,b) + cuu E(a+2,b) + cuv E(a+1,b+1) + cv E(a,b+1) + cvv E(a,b+2)
    //               + A <u^(a+1) v^b e> + B <u^a v^(b+1) e>
    const double S1 = cu * mu[2] + cuu * mu[3] + cuv * E21 + cv * E11 + cvv * E12 + A * eM20 + B * eM11;
    const double E15 = mu[1] * mv[5], E24 = mu[2] * mv[4], E33 = mu[3] * mv[3], E42 = mu[4] * mv[2];
    const double E51 = mu[5] * mv[1];
    const double T1 = cu * mu[3] + cuu * mu[4] + cuv * E31 + cv * E21 + cvv * E22 + A * eM30 + B * eM21;
    const double T2 = cu * E21 + cuu * E31 + cuv * E22 + cv * E12 + cvv * E13 + A * eM21 + B * eM12;
    // <u e P>: <u^a v^b e^2> for (a, b) = (2, 0), (1, 1)
    const double e2M20 = mu[6] + 2.0 * E42 + E24 + 2.0 * x1 * (mu[4] + E22) + x2 * mu[2];
    const double e2M11 = E51 + 2.0 * E33 + E15 + 2.0 * x1 * (E31 + E13) + x2 * E11;
    const double T3 = cu * eM20 + cuu * eM30 + cuv * eM21 + cv * eM11 + cvv * eM12 + A * e2M20 + B * e2M11;
    Su[0] = S1;
    Su[1] = T1;
    Su[2] = T2;
    Su[3] = 0.5 * T3;
    if constexpr (PSI) {
      // E(0, b) = <u^0> <v^b>: <u^0> is the mass fraction of a half space
      const double E01 = mu[0] * mv[1], E02 = mu[0] * mv[2], E03 = mu[0] * mv[3], E04 = mu[0] * mv[4],
                   E05 = mu[0] * mv[5];
      const double eM01 = fma(x1, E01, E21 + E03), eM02 = fma(x1, E02, E22 + E04);
      const double S0 = cu * mu[1] + cuu * mu[2] + cuv * E11 + cv * E01 + cvv * E02 + A * eM10 + B * eM01;
      const double S2 = cu * E11 + cuu * E21 + cuv * E12 + cv * E02 + cvv * E03 + A * eM11 + B * eM02;
      const double e2M10 = mu[5] + 2.0 * E32 + E14 + 2.0 * x1 * (mu[3] + E12) + x2 * mu[1];
      const double e2M01 = E41 + 2.0 * E23 + E05 + 2.0 * x1 * (E21 + E03) + x2 * E01;
      const double S3 = cu * eM10 + cuu * eM20 + cuv * eM11 + cv * eM01 + cvv * eM02 + A * e2M10 + B * e2M01;
      Sp[0] = S0;
      Sp[1] = S1;
      Sp[2] = S2;
      Sp[3] = 0.5 * S3;
    }
  } else {
    (void)at;
    const double cu = an[0], cuu = an[1], A = 0.5 * an[2];
    const double eM1 = fma(x1, mu[1], mu[3]), eM2 = fma(x1, mu[2], mu[4]), eM3 = fma(x1, mu[3], mu[5]);
    const double S1 = cu * mu[2] + cuu * mu[3] + A * eM2;
    const double T1 = cu * mu[3] + cuu * mu[4] + A * eM3;
    const double e2M2 = mu[6] + 2.0 * x1 * mu[4] + x2 * mu[2];
    const double T3 = cu * eM2 + cuu * eM3 + A * e2M2;
    Su[0] = S1;
    Su[1] = T1;
    Su[2] = 0.5 * T3;
    if constexpr (PSI) {
      const double S0 = cu * mu[1] + cuu * mu[2] + A * eM1;
      const double e2M1 = mu[5] + 2.0 * x1 * mu[3] + x2 * mu[1];
      const double S3 = cu * eM1 + cuu * eM2 + A * e2M1;
      Sp[0] = S0;
      Sp[1] = S1;
      Sp[2] = 0.5 * S3;
    }
  }
}

// Exact Euler first and second time derivatives at a point (Cauchy-Kowalewski
// in primitive variables) and the flux time derivative dF/dt along the
// solution.  2D form; the 1D case has no y dependence and V = 0.
struct CK {
  double Wt[4], Wtt[4], Ft[4];
};

CGKS_HD __forceinline__ void euler_ck(const Gas& gas, const double* W, const double* Wx, const double* Wy,
                                         const double* Wxx, const double* Wxy, const double* Wyy, CK& o) {
  const double gamma = gas.gamma;
  const double g1 = gamma - 1.0;
  const double r = W[0], ir = recip(r);
  const double U = W[1] * ir, V = W[2] * ir;
  const double q2 = U * U + V * V;
  const double p = g1 * (W[3] - 0.5 * r * q2);
  // first derivatives of primitives (a = x, y)
  const double rx = Wx[0], ry = Wy[0];
  const double Ux = (Wx[1] - U * rx) * ir, Uy = (Wy[1] - U * ry) * ir;
  const double Vx = (Wx[2] - V * rx) * ir, Vy = (Wy[2] - V * ry) * ir;
  const double px = g1 * (Wx[3] - 0.5 * rx * q2 - r * (U * Ux + V * Vx));
  const double py = g1 * (Wy[3] - 0.5 * ry * q2 - r * (U * Uy + V * Vy));
  // second derivatives
  const double rxx = Wxx[0], rxy = Wxy[0], ryy = Wyy[0];
  const double Uxx = (Wxx[1] - rxx * U - 2.0 * rx * Ux) * ir;
  const double Uxy = (Wxy[1] - rxy * U - rx * Uy - ry * Ux) * ir;
  const double Uyy = (Wyy[1] - ryy * U - 2.0 * ry * Uy) * ir;
  const double Vxx = (Wxx[2] - rxx * V - 2.0 * rx * Vx) * ir;
  const double Vxy = (Wxy[2] - rxy * V - rx * Vy - ry * Vx) * ir;
  const double Vyy = (Wyy[2] - ryy * V - 2.0 * ry * Vy) * ir;
  const double pxx = g1 * (Wxx[3] - 0.5 * rxx * q2 - 2.0 * rx * (U * Ux + V * Vx) - r * (Ux * Ux + Vx * Vx) - r * (U * Uxx + V * Vxx));
  const double pxy = g1 * (Wxy[3] - 0.5 * rxy * q2 - rx * (U * Uy + V * Vy) - ry * (U * Ux + V * Vx) - r * (Ux * Uy + Vx * Vy) - r * (U * Uxy + V * Vxy));
  const double pyy = g1 * (Wyy[3] - 0.5 * ryy * q2 - 2.0 * ry * (U * Uy + V * Vy) - r * (Uy * Uy + Vy * Vy) - r * (U * Uyy + V * Vyy));
  // first time derivatives
  const double dv = Ux + Vy;
  const double rt = -(U * rx + V * ry + r * dv);
  const double Ut = -(U * Ux + V * Uy + px * ir);
  const double Vt = -(U * Vx + V * Vy + py * ir);
  const double pt = -(U * px + V * py + gamma * p * dv);
  // mixed derivatives q_tx, q_ty
  const double dvx = Uxx + Vxy, dvy = Uxy + Vyy;
  const double ir2 = ir * ir;
  const double rtx = -(Ux * rx + U * rxx + Vx * ry + V * rxy + rx * dv + r * dvx);
  const double rty = -(Uy * rx + U * rxy + Vy * ry + V * ryy + ry * dv + r * dvy);
  const double Utx = -(Ux * Ux + U * Uxx + Vx * Uy + V * Uxy + pxx * ir - px * rx * ir2);
  const double Uty = -(Uy * Ux + U * Uxy + Vy * Uy + V * Uyy + pxy * ir - px * ry * ir2);
  const double Vtx = -(Ux * Vx + U * Vxx + Vx * Vy + V * Vxy + pxy * ir - py * rx * ir2);
  const double Vty = -(Uy * Vx + U * Vxy + Vy * Vy + V * Vyy + pyy * ir - py * ry * ir2);
  const double ptx = -(Ux * px + U * pxx + Vx * py + V * pxy + gamma * px * dv + gamma * p * dvx);
  const double pty = -(Uy * px + U * pxy + Vy * py + V * pyy + gamma * py * dv + gamma * p * dvy);
  // second time derivatives
  const double dvt = Utx + Vty;
  const double rtt = -(Ut * rx + U * rtx + Vt * ry + V * rty + rt * dv + r * dvt);
  const double Utt = -(Ut * Ux + U * Utx + Vt * Uy + V * Uty + ptx * ir - px * rt * ir2);
  const double Vtt = -(Ut * Vx + U * Vtx + Vt * Vy + V * Vty + pty * ir - py * rt * ir2);
  const double ptt = -(Ut * px + U * ptx + Vt * py + V * pty + gamma * pt * dv + gamma * p * dvt);
  const double E = W[3];
  const double Et = pt * gas.inv_g1 + 0.5 * rt * q2 + r * (U * Ut + V * Vt);
  o.Wt[0] = rt;
  o.Wt[1] = rt * U + r * Ut;
  o.Wt[2] = rt * V + r * Vt;
  o.Wt[3] = Et;
  o.Wtt[0] = rtt;
  o.Wtt[1] = rtt * U + 2.0 * rt * Ut + r * Utt;
  o.Wtt[2] = rtt * V + 2.0 * rt * Vt + r * Vtt;
  o.Wtt[3] = ptt * gas.inv_g1 + 0.5 * rtt * q2 + 2.0 * rt * (U * Ut + V * Vt) + r * (Ut * Ut + Vt * Vt) + r * (U * Utt + V * Vtt);
  // d/dt of the x flux (rhoU, rhoU^2 + p, rhoUV, U(E + p)) along the solution
  o.Ft[0] = o.Wt[1];
  o.Ft[1] = rt * U * U + 2.0 * r * U * Ut + pt;
  o.Ft[2] = rt * U * V + r * Ut * V + r * U * Vt;
  o.Ft[3] = Ut * (E + p) + U * (Et + pt);
}

// Inputs / outputs of one interface point.
template <int NC>
struct PointIn {
  double W0[NC], Wn[NC], Wt[NC], Wnn[NC], Wnt[NC], Wtt[NC], Wl[NC], Wr[NC];
};

template <int NC>
struct PointOut {
  double F[NC], Ft[NC], Wt[NC], Wtt[NC], Nh[NC], Nf[NC], W0[NC];
  int guard;
};

// Kinetic sums of the two non-equilibrium sides: M4 = sum rho <u psi>_side,
// D35 accumulates -rho <u psi (a_n u + a_t v)>_side (and later + the
// equilibrium's slope term), Slr = sum rho <psi>_side,
// Salr = sum rho <psi (a_n u + a_t v)>_side.
template <int NC>
struct SideSums {
  double M4[NC], D35[NC], Slr[NC], Salr[NC];
  CGKS_HD __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < NC; ++k) { M4[k] = 0.0; D35[k] = 0.0; Slr[k] = 0.0; Salr[k] = 0.0; }
  }
  template <bool FULL>
  CGKS_HD __forceinline__ void pin() {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      CGKS_PIN(M4[k]);
      CGKS_PIN(D35[k]);
      if constexpr (FULL) { CGKS_PIN(Slr[k]); CGKS_PIN(Salr[k]); }
    }
  }
};

// Collision times of Sec. 4, p_l, p_r of the nonlinear (WENO) states and p0
// of the equilibrium state W0.  tau_ce is the collision time of the
// Chapman-Enskog term, tau the one in exp(-t/tau):
//   Euler (mu = 0):  tau_ce = C |p_l - p_r|/(p_l + p_r) dt,  tau = eps dt + tau_ce
//   Navier-Stokes:   tau_ce = mu/p0 + C |p_l - p_r|/(p_l + p_r) dt = tau
template <int NC>
CGKS_HD __forceinline__ double collision_time(const double* Wl, const double* Wr, const double* W0, const Gas& g,
                                              double dt, double& tau_ce) {
  const double pl = pressure<NC>(Wl, g.gamma), pr = pressure<NC>(Wr, g.gamma);
  const double jump = g.tau_C * fabs((pl - pr) * recip(pl + pr)) * dt;
  if (g.mu > 0.0) {
    tau_ce = g.mu * recip(pressure<NC>(W0, g.gamma)) + jump;
    return tau_ce;
  }
  tau_ce = jump;
  return g.tau_eps * dt + jump;
}

// tau from tau_ce (the same operations as collision_time).
CGKS_HD __forceinline__ double tau_of(const Gas& g, double dt, double tau_ce) {
  return g.mu > 0.0 ? tau_ce : g.tau_eps * dt + tau_ce;
}

// One non-equilibrium side (half space u > 0 for side = +1, u < 0 for -1):
// the slopes of the linear reconstruction (Wn, Wt) expressed in this side's
// Maxwellian (they use only its U, V, lambda), and its kinetic sums.
template <int NC, bool FULL>
CGKS_HD __forceinline__ void side_terms(const double* Ws, int side, const double* Wn, const double* Wt,
                                        const Gas& g, SideSums<NC>& acc) {
  Mom<NC> m;
  moments<NC>(Ws, g, side, m);
  double bn[NC], an[NC], at[NC] = {}, t1[NC], t2[NC];
  const double ir = m.ir;
#pragma unroll
  for (int k = 0; k < NC; ++k) bn[k] = Wn[k] * ir;
  slope<NC>(m, g, bn, an);
  if constexpr (NC == 4) {
#pragma unroll
    for (int k = 0; k < NC; ++k) bn[k] = Wt[k] * ir;
    slope<NC>(m, g, bn, at);
  }
  // <u psi> and, with FULL, <psi>
  if constexpr (NC == 4) {
    t1[0] = m.mu[1];
    t1[1] = m.mu[2];
    t1[2] = m.mu[1] * m.mv[1];
    t1[3] = 0.5 * fma(m.x1, m.mu[1], m.mu[3] + m.mu[1] * m.mv[2]);
  } else {
    t1[0] = m.mu[1];
    t1[1] = m.mu[2];
    t1[2] = 0.5 * fma(m.x1, m.mu[1], m.mu[3]);
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) acc.M4[k] += m.rho * t1[k];
  // the slope terms: <u psi P> and <psi P>, P = u (a_n . psi) + v (a_t . psi)
  slope_moments<NC, FULL>(m, an, at, t2, t1);
#pragma unroll
  for (int k = 0; k < NC; ++k) acc.D35[k] -= m.rho * t1[k];
  if constexpr (FULL) {
#pragma unroll
    for (int k = 0; k < NC; ++k) acc.Salr[k] += m.rho * t2[k];
    double t0[NC];
    t0[0] = m.mu[0];
    t0[1] = m.mu[1];
    if constexpr (NC == 4) {
      t0[2] = m.mu[0] * m.mv[1];
      t0[3] = 0.5 * fma(m.mu[0], m.mv[2] + m.x1, m.mu[2]);
    } else {
      t0[2] = 0.5 * fma(m.mu[0], m.x1, m.mu[2]);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) acc.Slr[k] += m.rho * t0[k];
  }
}

// Kinetic collision state of the two sides, rho_l <psi>_{l,u>0} + rho_r <psi>_{r,u<0}
// (used in place of an inadmissible linear equilibrium state).
template <int NC>
CGKS_HD __forceinline__ void collision_state(const double* Wl, const double* Wr, const Gas& g, double* S) {
  Mom<NC> m;
  double t1[NC];
  moments<NC>(Wl, g, +1, m);
  mom_psi<NC>(m, 0, 0, t1);
#pragma unroll
  for (int k = 0; k < NC; ++k) S[k] = m.rho * t1[k];
  moments<NC>(Wr, g, -1, m);
  mom_psi<NC>(m, 0, 0, t1);
#pragma unroll
  for (int k = 0; k < NC; ++k) S[k] += m.rho * t1[k];
}

// Slope part of the equilibrium M3 = rho0 <u psi (a_n u + a_t v)>_0: D35 += M3;
// with FULL also the Chapman-Enskog flux Fce = -tau_ce (M2 + M3), M2 the
// flux time derivative rho0 <u psi A>_0.
template <int NC, bool FULL>
CGKS_HD __forceinline__ void equilibrium_terms(const double* W0, const double* Wn, const double* Wt, const Gas& g,
                                               double tau_ce, const double* M2, double* D35, double* Fce) {
  Mom<NC> m;
  moments<NC>(W0, g, 0, m);
  double bn[NC], an[NC], at[NC] = {}, t1[NC];
  const double ir = m.ir;
#pragma unroll
  for (int k = 0; k < NC; ++k) bn[k] = Wn[k] * ir;
  slope<NC>(m, g, bn, an);
  if constexpr (NC == 4) {
#pragma unroll
    for (int k = 0; k < NC; ++k) bn[k] = Wt[k] * ir;
    slope<NC>(m, g, bn, at);
  }
  slope_moments<NC, false>(m, an, at, nullptr, t1);     // <u psi (a_n u + a_t v)>
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double m3 = m.rho * t1[k];
    D35[k] += m3;
    if constexpr (FULL) Fce[k] = -tau_ce * (M2[k] + m3);
  }
}

// Exact Euler derivatives of the equilibrium at the point, in the NC layout:
// W_t, W_tt and the flux time derivative M2 = dF/dt.
template <int NC>
CGKS_HD __forceinline__ void ck_terms(const Gas& gas, const double* W0, const double* Wn, const double* Wt,
                                      const double* Wnn, const double* Wnt, const double* Wtt,
                                      double* Wt_o, double* Wtt_o, double* M2) {
  CK ck;
  if constexpr (NC == 4) {
    euler_ck(gas, W0, Wn, Wt, Wnn, Wnt, Wtt, ck);
#pragma unroll
    for (int k = 0; k < 4; ++k) { Wt_o[k] = ck.Wt[k]; Wtt_o[k] = ck.Wtt[k]; M2[k] = ck.Ft[k]; }
  } else {   // 1D embedded as V = 0 without y dependence
    const double W4[4] = {W0[0], W0[1], 0.0, W0[2]};
    const double x4[4] = {Wn[0], Wn[1], 0.0, Wn[2]};
    const double xx4[4] = {Wnn[0], Wnn[1], 0.0, Wnn[2]};
    const double z4[4] = {0.0, 0.0, 0.0, 0.0};
    euler_ck(gas, W4, x4, z4, xx4, z4, z4, ck);
    Wt_o[0] = ck.Wt[0]; Wt_o[1] = ck.Wt[1]; Wt_o[2] = ck.Wt[3];
    Wtt_o[0] = ck.Wtt[0]; Wtt_o[1] = ck.Wtt[1]; Wtt_o[2] = ck.Wtt[3];
    M2[0] = ck.Ft[0]; M2[1] = ck.Ft[1]; M2[2] = ck.Ft[3];
  }
}

// Combination of the moment vectors with the time coefficients of the flux
// extraction (Eh = e^{-dt/(2 tau)}, E = Eh^2):
//   F  = M1 + e4 (M4 - M1) + e3 (M3 - M5) + Fce
//   Ft = M2 + e1' (M1 - M4) + e3' (M3 - M5)
// and (FULL) the non-equilibrium remainders e^{-t/tau}[-W0 - t W_t + S_lr - t S_alr]
// at t = dt/2 (Nh) and t = dt (Nf).  M1 = F(W0), the Euler flux; Fce the
// Chapman-Enskog flux (constant in time, so only in F; Fce may be out.F).
template <int NC, bool FULL>
CGKS_HD __forceinline__ void combine(const double* W0, const double* M2, const SideSums<NC>& sd, double tau,
                                     double dt, const Gas& g, const double* Fce, PointOut<NC>& out) {
  double M1[NC];
  {
    const double ir = recip(W0[0]);
    const double U = W0[1] * ir;
    const double p = pressure<NC>(W0, g.gamma);
    M1[0] = W0[1];
    M1[1] = W0[1] * U + p;
    if constexpr (NC == 4) M1[2] = W0[2] * U;
    M1[NC - 1] = (W0[NC - 1] + p) * U;
  }
  // Eh = e^{a}, a = -dt/(2 tau).  Every term Eh contributes is at most
  // (4/3)|a| e^{a} relative to the term it is added to, below 3.2e-17 for
  // a < -42: there Eh is taken as 0 and the exponential skipped (the usual
  // case in smooth flow, where a is about -50).
  const double ah = -0.5 * dt * recip(tau);
  const double Eh = ah < -42.0 ? 0.0 : exp(ah);
  const double omh = 1.0 - Eh;
  const double idt = recip(dt);
  const double e1p = 4.0 * tau * omh * omh * idt * idt;
  const double e3p = 4.0 * tau * omh * (dt * Eh - tau * omh) * idt * idt;
#pragma unroll
  for (int k = 0; k < NC; ++k) out.Ft[k] = M2[k] + e1p * (M1[k] - sd.M4[k]) + e3p * sd.D35[k];
  if constexpr (FULL) {
    const double e4 = tau * omh * (3.0 - Eh) * idt;
    const double e3 = (tau * tau * omh * (3.0 - Eh) - tau * dt * Eh * (2.0 - Eh)) * idt;
    const double E = Eh * Eh;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      out.F[k] = M1[k] + e4 * (sd.M4[k] - M1[k]) + e3 * sd.D35[k] + Fce[k];
      const double base = sd.Slr[k] - W0[k];
      const double slp = out.Wt[k] + sd.Salr[k];
      out.Nh[k] = Eh * (base - 0.5 * dt * slp);
      out.Nf[k] = E * (base - dt * slp);
      out.W0[k] = W0[k];
    }
  }
}

// The interface evolution at one point (eq. 3rd-simplify-flux, second-order
// part for the flux): the collision time tau in exp(-t/tau), its pressure-jump
// part in the Chapman-Enskog term.  The phases above in order; FULL = false
// computes only what the second stage needs (Ft, Wtt).
// Wln, Wrn: the normal slopes of the two non-equilibrium sides (the linear
// reconstruction's in.Wn as the scheme reads it, or the WENO-weighted slopes
// of the evaluated variant).
template <int NC, bool FULL>
CGKS_HD __forceinline__ void gks_point(const PointIn<NC>& in, const double* Wln, const double* Wrn, const Gas& g,
                                       double dt, PointOut<NC>& out) {
  // equilibrium from the linear reconstruction; the kinetic collision state
  // of the two sides if it is not admissible
  double W0[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) W0[k] = in.W0[k];
  out.guard = 0;
  if (!admissible<NC>(W0, g.gamma)) {
    collision_state<NC>(in.Wl, in.Wr, g, W0);
    out.guard = 1;
  }
  double M2[NC];
  ck_terms<NC>(g, W0, in.Wn, in.Wt, in.Wnn, in.Wnt, in.Wtt, out.Wt, out.Wtt, M2);
  double tau_ce;
  const double tau = collision_time<NC>(in.Wl, in.Wr, W0, g, dt, tau_ce);
  SideSums<NC> sd;
  sd.zero();
  side_terms<NC, FULL>(in.Wl, +1, Wln, in.Wt, g, sd);
  side_terms<NC, FULL>(in.Wr, -1, Wrn, in.Wt, g, sd);
  equilibrium_terms<NC, FULL>(W0, in.Wn, in.Wt, g, tau_ce, M2, sd.D35, out.F);   // D35 = M3 - M5
  combine<NC, FULL>(W0, M2, sd, tau, dt, g, out.F, out);
}

template <int NC, bool FULL>
CGKS_HD __forceinline__ void gks_point(const PointIn<NC>& in, const Gas& g, double dt, PointOut<NC>& out) {
  gks_point<NC, FULL>(in, in.Wn, in.Wn, g, dt, out);
}

// ----------------------------------------------------------------------------
// Tangential reconstruction of one face point from the NL stencil lines of its
// face segment (offsets -NL/2..NL/2; NL = 3 with two Gauss points, 7 with
// four).  get(q, l) returns quantity q of line l: q = 4*j + k for
// j = (P7, hn P7_n, hn^2 P7_nn, WENO left, WENO right) and component k (each
// shifted by the line's own reference cell), q = 20 + k the reference cell
// average, q = 24 + k the line's tangential gradient at the face times ht
// (ht T) and q = 28 + k its normal derivative times hn ht (hn ht TN).
// Value-type quantities are moved to the face segment's reference (the
// middle line) before the fit; hn, ht are the normal and tangential cell
// widths.  dsg = -1 when get presents the lines in reverse order (the
// mirrored Gauss point: the derivative data change sign).
// ----------------------------------------------------------------------------
// Offsets that move the value-type quantities of line l to the middle line's
// reference: off[l] = ref(l) - ref(NL/2); returns ref(NL/2).
template <int NL, class Get>
CGKS_HD __forceinline__ double tang_offsets(Get get, int k, double* off) {
  const double rj = get(20 + k, NL / 2);
#pragma unroll
  for (int l = 0; l < NL; ++l) off[l] = get(20 + k, l) - rj;
  return rj;
}

// sum_l c[l] (get(q, l) + off[l]) (value-type quantity, off from tang_offsets)
template <int NL, class Get>
CGKS_HD __forceinline__ double tang_value(Get get, const double* c, int q, const double* off) {
  double s = 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) s += c[l] * (get(q, l) + off[l]);
  return s;
}

// sum_l c[l] get(q, l) (derivative-type quantity, no reference shift)
template <int NL, class Get>
CGKS_HD __forceinline__ double tang_deriv(Get get, const double* c, int q) {
  double s = 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) s += c[l] * get(q, l);
  return s;
}

// The three-segment quintic over the middle lines of an NL-line stencil:
// value-type quantity q (averages, with the offsets) and its tangential
// derivative data qd; ws/wd: weights of the averages and of the data.
template <int NL, class Get>
CGKS_HD __forceinline__ double herm_value(Get get, const double* ws, const double* wd, int q, int qd,
                                          const double* off, double dsg) {
  constexpr int L0 = NL / 2 - 1;
  double s = 0, d = 0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    s += ws[l] * (get(q, L0 + l) + off[L0 + l]);
    d += wd[l] * get(qd, L0 + l);
  }
  return s + dsg * d;
}

// the same for a derivative-type quantity (no reference shift)
template <int NL, class Get>
CGKS_HD __forceinline__ double herm_deriv(Get get, const double* ws, const double* wd, int q, int qd, double dsg) {
  constexpr int L0 = NL / 2 - 1;
  double s = 0, d = 0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    s += ws[l] * get(q, L0 + l);
    d += wd[l] * get(qd, L0 + l);
  }
  return s + dsg * d;
}

// The tangential-WENO variant (two Gauss points): the value at the first node
// eta = -1/(2 sqrt 3) (unit segment width; the mirrored node reads the
// segments in reverse order) from the averages s[0..4] of the five nearest
// segments: the three quadratics with the averages of segments (-2..0),
// (-1..1), (0..2), evaluated at the node, combined with WENO-Z weights of
// the normal reconstruction's form (tau = |beta_0 - beta_2|, Jiang-Shu
// indicators of the three averages) whose linear part gives the quartic
// through the five averages at the node.
CGKS_HD __forceinline__ double tang_weno5(const double* s, double eps) {
  constexpr double r3 = 1.7320508075688772935;   // sqrt(3)
  // the quadratics at the node: centre segment value plus sqrt(3)/12 times
  // a difference of the averages
  const double q0 = s[2] + (r3 / 12.0) * (4.0 * s[1] - s[0] - 3.0 * s[2]);
  const double q1 = s[2] + (r3 / 12.0) * (s[1] - s[3]);
  const double q2 = s[2] + (r3 / 12.0) * (3.0 * s[2] - 4.0 * s[3] + s[4]);
  const double a0 = s[0] - 2.0 * s[1] + s[2], c0 = s[0] - 4.0 * s[1] + 3.0 * s[2];
  const double a1 = s[1] - 2.0 * s[2] + s[3], c1 = s[1] - s[3];
  const double a2 = s[2] - 2.0 * s[3] + s[4], c2 = 3.0 * s[2] - 4.0 * s[3] + s[4];
  const double b0 = (13.0 / 12.0) * a0 * a0 + 0.25 * c0 * c0;
  const double b1 = (13.0 / 12.0) * a1 * a1 + 0.25 * c1 * c1;
  const double b2 = (13.0 / 12.0) * a2 * a2 + 0.25 * c2 * c2;
  const double tau = fabs(b0 - b2);
  const double w0 = (7.0 / 36.0 + r3 / 1080.0) * (1.0 + tau * recip(b0 + eps));
  const double w1 = (11.0 / 18.0) * (1.0 + tau * recip(b1 + eps));
  const double w2 = (7.0 / 36.0 - r3 / 1080.0) * (1.0 + tau * recip(b2 + eps));
  return (w0 * q0 + w1 * q1 + w2 * q2) * recip(w0 + w1 + w2);
}

// The same at a node eta of the four-point rule: the quadratics evaluated at
// eta (y = eta - c for the segment centres c = -1, 0, 1) and the linear
// weights of that node (from csrc/tang_weno_weights.py: the quartic through
// the five averages at eta).
struct TwNode { double eta, d0, d1, d2; };
// first node of each mirror pair: inner -a, outer -b
constexpr TwNode kTwInner = {-0.169990521792428132401, 0.128164158435505840028, 0.521969149850356295584,
                             0.349866691714137864388};
constexpr TwNode kTwOuter = {-0.430568155797026287612, 0.265842097477831923315, 0.611250490032248606455,
                             0.122907412489919470230};
CGKS_HD __forceinline__ double tang_weno5_at(const double* s, double eps, const TwNode& n) {
  double q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double y = n.eta - (k - 1.0), w2 = 0.5 * y * y - 1.0 / 24.0;
    q[k] = (w2 - 0.5 * y) * s[k] + (1.0 - 2.0 * w2) * s[k + 1] + (w2 + 0.5 * y) * s[k + 2];
  }
  const double a0 = s[0] - 2.0 * s[1] + s[2], c0 = s[0] - 4.0 * s[1] + 3.0 * s[2];
  const double a1 = s[1] - 2.0 * s[2] + s[3], c1 = s[1] - s[3];
  const double a2 = s[2] - 2.0 * s[3] + s[4], c2 = 3.0 * s[2] - 4.0 * s[3] + s[4];
  const double b0 = (13.0 / 12.0) * a0 * a0 + 0.25 * c0 * c0;
  const double b1 = (13.0 / 12.0) * a1 * a1 + 0.25 * c1 * c1;
  const double b2 = (13.0 / 12.0) * a2 * a2 + 0.25 * c2 * c2;
  const double tau = fabs(b0 - b2);
  const double w0 = n.d0 * (1.0 + tau * recip(b0 + eps));
  const double w1 = n.d1 * (1.0 + tau * recip(b1 + eps));
  const double wq = n.d2 * (1.0 + tau * recip(b2 + eps));
  return (w0 * q[0] + w1 * q[1] + wq * q[2]) * recip(w0 + w1 + wq);
}

// The point quantities of component k (h: quintic weights at this node; w7:
// sextic weights, used when NL = 7).  Value-type results are deviations from
// the middle line's reference.
template <int NL>
struct TangEval {
  const TangWT<7>& w7;
  const HermWT& h;
  double dsg;
  template <class Get> CGKS_HD __forceinline__ double W0(Get get, int k, const double* off) const {
    if constexpr (NL == 3) return herm_value<3>(get, h.v, h.vd, k, 24 + k, off, dsg);
    else return tang_value<NL>(get, w7.v, k, off);
  }
  template <class Get> CGKS_HD __forceinline__ double side(Get get, int q, int k, const double* off) const {
    if constexpr (NL == 3) return herm_value<3>(get, h.v, h.vd, q, 24 + k, off, dsg);
    else return tang_value<NL>(get, w7.v, q, off);
  }
  template <class Get> CGKS_HD __forceinline__ double Wt(Get get, int k, const double* off) const {
    if constexpr (NL == 3) return herm_value<3>(get, h.d1, h.d1d, k, 24 + k, off, dsg);
    else return tang_value<NL>(get, w7.d1, k, off);
  }
  template <class Get> CGKS_HD __forceinline__ double Wtt(Get get, int k, const double* off) const {
    return herm_value<NL>(get, h.d2, h.d2d, k, 24 + k, off, dsg);
  }
  template <class Get> CGKS_HD __forceinline__ double Wn(Get get, int k) const { return Wn_of(get, 4 + k, k); }
  // a normal derivative at the point from the line quantity q of component k
  // (the linear reconstruction's, or a side slope of the evaluated variant)
  template <class Get> CGKS_HD __forceinline__ double Wn_of(Get get, int q, int k) const {
    if constexpr (NL == 3) return herm_deriv<3>(get, h.v, h.vd, q, 28 + k, dsg);
    else return tang_deriv<NL>(get, w7.v, q);
  }
  template <class Get> CGKS_HD __forceinline__ double Wnt(Get get, int k) const {
    return herm_deriv<NL>(get, h.d1, h.d1d, 4 + k, 28 + k, dsg);
  }
  template <class Get> CGKS_HD __forceinline__ double Wnn(Get get, int k) const {
    if constexpr (NL == 3) return tang_deriv<3>(get, h.q, 8 + k);
    else return tang_deriv<NL>(get, w7.v, 8 + k);
  }
};

// All inputs of the point evaluation at once (host checks and operation count).
template <int NL, class Get>
CGKS_HD __forceinline__ void tangential_point(Get get, const TangWT<7>& w7, const HermWT& h, double dsg, double hn,
                                              double ht, PointIn<4>& in, double* dev, double* ref) {
  const double inv_ht = 1.0 / ht, inv_hn = 1.0 / hn;
  const TangEval<NL> te{w7, h, dsg};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double off[NL];
    const double rj = tang_offsets<NL>(get, k, off);
    const double v = te.W0(get, k, off);
    ref[k] = rj;
    dev[k] = v;
    in.W0[k] = rj + v;
    in.Wn[k] = te.Wn(get, k) * inv_hn;
    in.Wnn[k] = te.Wnn(get, k) * inv_hn * inv_hn;
    in.Wt[k] = te.Wt(get, k, off) * inv_ht;
    in.Wnt[k] = te.Wnt(get, k) * inv_hn * inv_ht;
    in.Wtt[k] = te.Wtt(get, k, off) * inv_ht * inv_ht;
    in.Wl[k] = rj + te.side(get, 12 + k, k, off);
    in.Wr[k] = rj + te.side(get, 16 + k, k, off);
  }
}

// Gauss average (weight wg of this point: 1/2 for two points) of the per-point face results.  Stage 1 keeps
// F, F_t and the interface states at t + dt/2 (A) and the stage-n part of the
// state at t + dt (B), both as deviations from the face reference (Sec. 2.2);
// stage 2 keeps F_t and W_tt.
template <int NC, bool FULL>
CGKS_HD __forceinline__ void face_accumulate(double* acc, const PointOut<NC>& o, const double* dev,
                                             const double* ref, double dt, double wg = 0.5) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if constexpr (FULL) {
      const double d0 = o.guard ? o.W0[k] - ref[k] : dev[k];
      acc[k] += wg * o.F[k];
      acc[NC + k] += wg * o.Ft[k];
      acc[2 * NC + k] += wg * (d0 + 0.5 * dt * o.Wt[k] + dt * dt / 8.0 * o.Wtt[k] + o.Nh[k]);
      acc[3 * NC + k] += wg * (d0 + dt * o.Wt[k] + dt * dt / 6.0 * o.Wtt[k] + o.Nf[k]);
    } else {
      acc[k] += wg * o.Ft[k];
      acc[NC + k] += wg * o.Wtt[k];
    }
  }
}

// One Gauss point of a 2D face segment, evaluated phase by phase so that few
// values are live at a time: every tangential quantity is evaluated from the
// line data right before the phase that first needs it (the reference/deviation
// pair of the final state is re-read at the end).  get(q, l), w7, h and dsg
// as for tangential_point; inv_hn, inv_ht: inverse normal and tangential cell
// widths, inv_ht negated (and dsg = -1) when get presents the lines in
// reverse order (the other Gauss point: the same fits mirrored).
// right(k): average of the cell right of the face (fallback of an inadmissible
// right WENO state; the left one falls back to the reference cell).
// DIR 1 (y faces) rotates the momenta so that the normal one comes first.
// acc receives this point's share wg of the Gauss average (face_accumulate
// from zero); guard / nbad count the equilibrium and WENO fallbacks.
// TW (the tangential-WENO variant): the two nonlinear states come in tws
// (Wl, Wr, unrotated) instead of from the quintic of the three segments.
template <int DIR, bool FULL, int NL, bool SS = false, bool TW = false, class Get, class Right>
CGKS_HD __forceinline__ void face_point(Get get, Right right, const TangWT<7>& w7, const HermWT& h, double dsg,
                                        double inv_hn, double inv_ht, const Gas& gas, double dt, double* acc,
                                        int& guard, int& nbad, double wg = 0.5, const double* tws = nullptr) {
  const TangEval<NL> te{w7, h, dsg};
  auto rot = [](double* v) {
    if (DIR == 1) { const double t = v[1]; v[1] = v[2]; v[2] = t; }
  };

  // nonlinear states (inadmissible ones fall back to the adjacent cell
  // averages) and the linear equilibrium state (the kinetic collision state
  // of the two sides if it is inadmissible)
  double Wl[4], Wr[4], W0[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double off[NL];
    const double rj = tang_offsets<NL>(get, k, off);
    if constexpr (TW) {
      Wl[k] = tws[k];
      Wr[k] = tws[4 + k];
    } else {
      Wl[k] = rj + te.side(get, 12 + k, k, off);
      Wr[k] = rj + te.side(get, 16 + k, k, off);
    }
    W0[k] = rj + te.W0(get, k, off);
    CGKS_PIN(Wl[k]);
    CGKS_PIN(Wr[k]);
    CGKS_PIN(W0[k]);
    CGKS_BREAK();
  }
  nbad = 0;
  bool bad_l = false, bad_r = false;
  if (!admissible<4>(Wl, gas.gamma)) {
#pragma unroll
    for (int k = 0; k < 4; ++k) Wl[k] = get(20 + k, NL / 2);
    ++nbad;
    bad_l = true;
  }
  if (!admissible<4>(Wr, gas.gamma)) {
#pragma unroll
    for (int k = 0; k < 4; ++k) Wr[k] = right(k);
    ++nbad;
    bad_r = true;
  }
  rot(Wl);
  rot(Wr);
  rot(W0);
  guard = 0;
  if (!admissible<4>(W0, gas.gamma)) {
    collision_state<4>(Wl, Wr, gas, W0);
    guard = 1;
  }
  // only tau_ce is kept across the phases: tau is formed again from it (the
  // same operations) where the combination needs it
  double tau_ce;
  collision_time<4>(Wl, Wr, W0, gas, dt, tau_ce);
  CGKS_PIN(tau_ce);
#pragma unroll
  for (int k = 0; k < 4; ++k) CGKS_PIN(W0[k]);
  CGKS_BREAK();

  // normal and tangential first derivatives
  double Wn[4], Wt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double off[NL];
    tang_offsets<NL>(get, k, off);
    Wn[k] = te.Wn(get, k) * inv_hn;
    Wt[k] = te.Wt(get, k, off) * inv_ht;
    CGKS_PIN(Wn[k]);
    CGKS_PIN(Wt[k]);
    CGKS_BREAK();
  }
  rot(Wn);
  rot(Wt);

  // normal slopes of the two non-equilibrium sides: the linear
  // reconstruction's Wn, or (SS, the evaluated variant) each line's
  // WENO-weighted side slopes (LDS rows 32-35 left, 36-39 right, h-scaled)
  // taken to the point like Wn, one side at a time; a side that fell back
  // to its cell average takes Wn
  double Wsn[4];
  auto side_slope = [&](int row0, bool bad) {
#pragma unroll
    for (int k = 0; k < 4; ++k) Wsn[k] = te.Wn_of(get, row0 + k, k) * inv_hn;
    rot(Wsn);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (bad) Wsn[k] = Wn[k];
  };

  // the two non-equilibrium sides (each phase's results are pinned before its
  // barrier so that its arithmetic stays in the phase)
  SideSums<4> sd;
  sd.zero();
  if constexpr (SS) side_slope(32, bad_l);
  side_terms<4, FULL>(Wl, +1, SS ? Wsn : Wn, Wt, gas, sd);
  sd.pin<FULL>();
  CGKS_BREAK();
  if constexpr (SS) side_slope(36, bad_r);
  side_terms<4, FULL>(Wr, -1, SS ? Wsn : Wn, Wt, gas, sd);
  sd.pin<FULL>();
  CGKS_BREAK();

  // Euler derivatives of the equilibrium
  double Wt_o[4], Wtt_o[4], M2[4];
  {
    double Wnn[4], Wnt[4], Wtt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double off[NL];
      tang_offsets<NL>(get, k, off);
      Wnn[k] = te.Wnn(get, k) * inv_hn * inv_hn;
      Wnt[k] = te.Wnt(get, k) * inv_hn * inv_ht;
      Wtt[k] = te.Wtt(get, k, off) * inv_ht * inv_ht;
      CGKS_PIN(Wnn[k]);
      CGKS_PIN(Wnt[k]);
      CGKS_PIN(Wtt[k]);
      CGKS_BREAK();
    }
    rot(Wnn);
    rot(Wnt);
    rot(Wtt);
    ck_terms<4>(gas, W0, Wn, Wt, Wnn, Wnt, Wtt, Wt_o, Wtt_o, M2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      CGKS_PIN(Wt_o[k]);
      CGKS_PIN(Wtt_o[k]);
      CGKS_PIN(M2[k]);
    }
  }
  CGKS_BREAK();

  // slope part of the equilibrium, the Chapman-Enskog flux and the combination
  PointOut<4> o;
  equilibrium_terms<4, FULL>(W0, Wn, Wt, gas, tau_ce, M2, sd.D35, o.F);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    CGKS_PIN(sd.D35[k]);
    if constexpr (FULL) CGKS_PIN(o.F[k]);
  }
  CGKS_BREAK();
#pragma unroll
  for (int k = 0; k < 4; ++k) { o.Wt[k] = Wt_o[k]; o.Wtt[k] = Wtt_o[k]; }
  combine<4, FULL>(W0, M2, sd, tau_of(gas, dt, tau_ce), dt, gas, o.F, o);
  o.guard = guard;
  rot(o.F); rot(o.Ft); rot(o.Wt); rot(o.Wtt); rot(o.Nh); rot(o.Nf); rot(o.W0);
  CGKS_BREAK();

  // dev, ref in the grid frame, like the outputs rotated back above
  double dev[4], ref[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double off[NL];
    ref[k] = tang_offsets<NL>(get, k, off);
    dev[k] = te.W0(get, k, off);
    CGKS_PIN(ref[k]);
    CGKS_PIN(dev[k]);
    CGKS_BREAK();
  }
  constexpr int NO = FULL ? 16 : 8;
#pragma unroll
  for (int q = 0; q < NO; ++q) acc[q] = 0.0;
  face_accumulate<4, FULL>(acc, o, dev, ref, dt, wg);
}

}  // namespace cgks
