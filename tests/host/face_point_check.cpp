// Host check of the phase-by-phase face-point evaluation (face_point) against
// the direct composition tangential_point -> gks_point -> face_accumulate, on
// seeded random line data; both Gauss points, both face directions, both
// stages, Euler and Navier-Stokes collision times, with and without the WENO /
// equilibrium fallbacks.
//
// Prints one line per case: "<dir> <stage> <gp> <case> <max relative difference>".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "cgks_device.h"

using namespace cgks;

static const TangW kW[2] = CGKS_TANG_WEIGHTS;

template <int DIR, bool FULL>
static double run(const double (&lines)[24][5], const double* right, int gp, const Gas& gas, double dt, double hn,
                  double ht, int& guard_ref, int& guard_new, int& bad_ref, int& bad_new) {
  auto get = [&](int q, int l) { return lines[q][l]; };
  // direct composition
  PointIn<4> in;
  double dev[4], ref[4];
  tangential_point(get, kW[gp], hn, ht, in, dev, ref);
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
  auto getm = [&](int q, int l) { return lines[q][gp ? 4 - l : l]; };
  auto rightf = [&](int k) { return right[k]; };
  double a_new[16];
  face_point<DIR, FULL>(getm, rightf, kW[0], 1.0 / hn, gp ? -1.0 / ht : 1.0 / ht, gas, dt, a_new, guard_new, bad_new);
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
  for (int vis = 0; vis < 2; ++vis)   // Euler, then Navier-Stokes (mu > 0)
  for (int c = 0; c < 40; ++c) {
    const Gas gas = make_gas(1.4, 2, 0.01, 1.0, vis ? 2e-3 : 0.0);
    // case 0..29 smooth; 30..34 inadmissible right WENO state; 35..39 inadmissible linear state
    double lines[24][5], right[4];
    for (int l = 0; l < 5; ++l)
      for (int k = 0; k < 4; ++k) {
        const double refv = base[k] * (1.0 + 0.05 * U(rng));
        lines[20 + k][l] = refv;
        lines[k][l] = 0.02 * U(rng) * std::fabs(base[k]);          // P7 value (deviation)
        lines[4 + k][l] = 0.05 * U(rng) * std::fabs(base[k]);      // h * normal derivative
        lines[8 + k][l] = 0.01 * U(rng) * std::fabs(base[k]);      // h^2 * second derivative
        lines[12 + k][l] = 0.02 * U(rng) * std::fabs(base[k]);     // left WENO state (deviation)
        lines[16 + k][l] = 0.02 * U(rng) * std::fabs(base[k]);     // right WENO state (deviation)
      }
    for (int k = 0; k < 4; ++k) right[k] = base[k] * (1.0 + 0.03 * U(rng));
    if (c >= 30 && c < 35)
      for (int l = 0; l < 5; ++l) lines[16][l] = -1.5;              // negative right density
    if (c >= 35)
      for (int l = 0; l < 5; ++l) { lines[3][l] = -2.55; lines[15][l] = 0.0; lines[19][l] = 0.0; }  // p < 0 in W0 only
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
