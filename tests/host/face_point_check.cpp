// Host check of the phase-by-phase face-point evaluation (face_point) against
// the direct composition tangential_point -> gks_point -> face_accumulate, on
// seeded random line data; both Gauss points (the second one by mirrored line
// order in face_point, by its own weights in the composition), both face
// directions, both stages, Euler and Navier-Stokes collision times, with and
// without the WENO / equilibrium fallbacks.  First, the tangential weight
// tables are checked against polynomials: the three-segment quintic and
// quadratic at the 2- and 4-point nodes.
//
// Prints "weights <max error>", then one line per case:
// "<dir> <stage> <gp> <case> <max relative difference> ...".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "cgks_device.h"

using namespace cgks;

static const HermWT kH2[2] = CGKS_HERM2_WEIGHTS;
static const HermWT kH4[2] = CGKS_HERM4_WEIGHTS;
static const TangWT<7> kT7[2] = CGKS_TANG7_WEIGHTS;

// max error of the weights of one node against a random quintic / quadratic
static double check_weights(const HermWT& w, double eta, std::mt19937_64& rng) {
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double c[6];
  for (double& x : c) x = U(rng);
  auto P = [&](double x) { double r = 0; for (int p = 5; p >= 0; --p) r = r * x + c[p]; return r; };
  auto P1 = [&](double x) { double r = 0; for (int p = 5; p >= 1; --p) r = r * x + p * c[p]; return r; };
  auto P2 = [&](double x) { double r = 0; for (int p = 5; p >= 2; --p) r = r * x + p * (p - 1) * c[p]; return r; };
  auto I = [&](double x) { double r = 0; for (int p = 5; p >= 0; --p) r = r * x + c[p] / (p + 1); return r * x; };
  double sv[3], dv[3];
  for (int l = 0; l < 3; ++l) {
    const double a = l - 1.5, b = l - 0.5;
    sv[l] = I(b) - I(a);
    dv[l] = P(b) - P(a);
  }
  double v = 0, d1 = 0, d2 = 0;
  for (int l = 0; l < 3; ++l) {
    v += w.v[l] * sv[l] + w.vd[l] * dv[l];
    d1 += w.d1[l] * sv[l] + w.d1d[l] * dv[l];
    d2 += w.d2[l] * sv[l] + w.d2d[l] * dv[l];
  }
  double e = std::fmax(std::fabs(v - P(eta)), std::fmax(std::fabs(d1 - P1(eta)), std::fabs(d2 - P2(eta))));
  // the quadratic: averages of c0 + c1 x + c2 x^2
  const double q0 = c[0], q1 = c[1], q2 = c[2];
  double sq[3];
  for (int l = 0; l < 3; ++l) {
    const double a = l - 1.5, b = l - 0.5;
    sq[l] = q0 + q1 * 0.5 * (a + b) + q2 * (a * a + a * b + b * b) / 3.0;
  }
  double qv = 0;
  for (int l = 0; l < 3; ++l) qv += w.q[l] * sq[l];
  return std::fmax(e, std::fabs(qv - (q0 + q1 * eta + q2 * eta * eta)));
}

template <int DIR, bool FULL>
static double run(const double (&lines)[32][3], const double* right, int gp, const Gas& gas, double dt, double hn,
                  double ht, int& guard_ref, int& guard_new, int& bad_ref, int& bad_new) {
  auto get = [&](int q, int l) { return lines[q][l]; };
  // direct composition with the node's own weights
  PointIn<4> in;
  double dev[4], ref[4];
  tangential_point<3>(get, kT7[0], kH2[gp], 1.0, hn, ht, in, dev, ref);
  bad_ref = 0;
  if (!admissible<4>(in.Wl, gas.gamma)) { for (int k = 0; k < 4; ++k) in.Wl[k] = ref[k]; ++bad_ref; }
  if (!admissible<4>(in.Wr, gas.gamma)) { for (int k = 0; k < 4; ++k) in.Wr[k] = right[k]; ++bad_ref; }
  auto sw = [](double* v) { const double t = v[1]; v[1] = v[2]; v[2] = t; };
  if (DIR == 1) { sw(in.W0); sw(in.Wn); sw(in.Wt); sw(in.Wnn); sw(in.Wnt); sw(in.Wtt); sw(in.Wl); sw(in.Wr); }
  PointOut<4> o;
  gks_point<4, FULL>(in, gas, dt, o);
  if (DIR == 1) { sw(o.F); sw(o.Ft); sw(o.Wt); sw(o.Wtt); sw(o.Nh); sw(o.Nf); sw(o.W0); }
  guard_ref = o.guard;
  constexpr int NO = FULL ? 16 : 8;
  double a_ref[16] = {0};
  face_accumulate<4, FULL>(a_ref, o, dev, ref, dt);
  // phase-by-phase evaluation; the second point reads the lines mirrored
  auto getm = [&](int q, int l) { return lines[q][gp ? 2 - l : l]; };
  auto rightf = [&](int k) { return right[k]; };
  double a_new[16];
  face_point<DIR, FULL, 3>(getm, rightf, kT7[0], kH2[0], gp ? -1.0 : 1.0, 1.0 / hn, gp ? -1.0 / ht : 1.0 / ht, gas, dt,
                           a_new, guard_new, bad_new);
  double err = 0.0;
  for (int q = 0; q < NO; ++q) {
    const double s = std::fmax(std::fabs(a_ref[q]), 1e-300);
    err = std::fmax(err, std::fabs(a_new[q] - a_ref[q]) / s);
  }
  return err;
}

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  const double hn = 1.0 / 300, ht = 1.0 / 200, dt = 1.5e-3;
  const double base[4] = {1.0, 0.35, -0.27, 2.6};
  int fails = 0;
  {
    const double g2 = 0.5 / std::sqrt(3.0);
    const double a4 = 0.5 * std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    const double b4 = 0.5 * std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    double e = 0.0;
    for (int r = 0; r < 20; ++r) {
      e = std::fmax(e, check_weights(kH2[0], -g2, rng));
      e = std::fmax(e, check_weights(kH2[1], g2, rng));
      e = std::fmax(e, check_weights(kH4[0], -a4, rng));
      e = std::fmax(e, check_weights(kH4[1], -b4, rng));
    }
    std::printf("weights %.3e\n", e);
    if (!(e < 1e-13)) ++fails;
  }
  for (int vis = 0; vis < 2; ++vis)   // Euler, then Navier-Stokes (mu > 0)
  for (int c = 0; c < 40; ++c) {
    const Gas gas = make_gas(1.4, 2, 0.01, 1.0, vis ? 2e-3 : 0.0);
    // case 0..29 smooth; 30..34 inadmissible right WENO state; 35..39 inadmissible linear state
    double lines[32][3], right[4];
    for (int l = 0; l < 3; ++l)
      for (int k = 0; k < 4; ++k) {
        const double refv = base[k] * (1.0 + 0.05 * U(rng));
        lines[20 + k][l] = refv;
        lines[k][l] = 0.02 * U(rng) * std::fabs(base[k]);          // P7 value (deviation)
        lines[4 + k][l] = 0.05 * U(rng) * std::fabs(base[k]);      // h * normal derivative
        lines[8 + k][l] = 0.01 * U(rng) * std::fabs(base[k]);      // h^2 * second derivative
        lines[12 + k][l] = 0.02 * U(rng) * std::fabs(base[k]);     // left WENO state (deviation)
        lines[16 + k][l] = 0.02 * U(rng) * std::fabs(base[k]);     // right WENO state (deviation)
        lines[24 + k][l] = 0.02 * U(rng) * std::fabs(base[k]);     // ht * tangential gradient at the face
        lines[28 + k][l] = 0.05 * U(rng) * std::fabs(base[k]);     // its normal derivative (hn ht)
      }
    for (int k = 0; k < 4; ++k) right[k] = base[k] * (1.0 + 0.03 * U(rng));
    if (c >= 30 && c < 35)
      for (int l = 0; l < 3; ++l) lines[16][l] = -1.5;              // negative right density
    if (c >= 35)
      for (int l = 0; l < 3; ++l) { lines[3][l] = -2.55; lines[15][l] = 0.0; lines[19][l] = 0.0; }  // p < 0 in W0 only
    for (int dir = 0; dir < 2; ++dir)
      for (int st = 1; st <= 2; ++st)
        for (int gp = 0; gp < 2; ++gp) {
          int gr, gn, br, bn;
          double e;
          if (dir == 0) e = st == 1 ? run<0, true>(lines, right, gp, gas, dt, hn, ht, gr, gn, br, bn)
                                    : run<0, false>(lines, right, gp, gas, dt, hn, ht, gr, gn, br, bn);
          else e = st == 1 ? run<1, true>(lines, right, gp, gas, dt, hn, ht, gr, gn, br, bn)
                           : run<1, false>(lines, right, gp, gas, dt, hn, ht, gr, gn, br, bn);
          const bool ok = e < 1e-11 && gr == gn && br == bn;
          if (!ok) ++fails;
          std::printf("%d %d %d %d %.3e %d %d %d %d%s\n", dir, st, gp, c, e, gr, gn, br, bn, ok ? "" : " FAIL");
        }
  }
  std::printf("fails %d\n", fails);
  return fails ? 1 : 0;
}
