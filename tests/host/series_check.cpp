// The near-zero series for erfc and exp used by the half-space moments,
// against the C library on a dense set of arguments inside their ranges and a
// few outside (where the library is used).  Prints the largest relative
// errors in units of 2^-52.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "cgks_device.h"

int main() {
  double e_erfc = 0.0, e_exp = 0.0;
  for (int i = -200000; i <= 200000; ++i) {
    const double x = 0.6 * i / 200000.0;      // [-0.6, 0.6], beyond the series range at both ends
    const double r = std::erfc(x);
    e_erfc = std::fmax(e_erfc, std::fabs(cgks::erfc_moment(x) - r) / r);
    const double y = 0.3 * i / 200000.0;      // [-0.3, 0.3]
    const double q = std::exp(y);
    e_exp = std::fmax(e_exp, std::fabs(cgks::exp_moment(y) - q) / q);
  }
  const double ulp = std::ldexp(1.0, -52);
  std::printf("erfc %.3f exp %.3f\n", e_erfc / ulp, e_exp / ulp);
  return (e_erfc <= 4 * ulp && e_exp <= 4 * ulp) ? 0 : 1;
}
