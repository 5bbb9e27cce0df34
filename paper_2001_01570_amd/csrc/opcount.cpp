// Operation count of the device arithmetic (algorithmic work per unit).
//
// The device functions of cgks_device.h are compiled for the host with every
// double replaced by a counting scalar: additions/subtractions, multiplications
// and divisions are counted (a fused multiply-add is a multiplication plus an
// addition, i.e. 2 flops), square roots, exponentials and complementary error
// functions separately.  Counting runs the device building blocks the kernels
// run (reconstruction, tangential fits, point evolution, Gauss average),
// each tangential quantity once per point, on a smooth representative state
// (no guard fires, both WENO sides evaluated).
//
// Units:  x- or y-face segment of one stage (4 normal reconstructions of its
// own line with the cells' tangential gradients carried across the face, 2
// Gauss points: tangential fits, gas-kinetic evolution, Gauss average) and
// one cell update.  The kernels' halo recomputation of stencil
// lines and the face kernels' second read of each point's reference state are
// not algorithmic work and are not counted.
//
// Output: JSON on stdout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <tuple>
#include <utility>

struct OpCounts {
  long add = 0, mul = 0, div = 0, sqrt_ = 0, exp_ = 0, erfc_ = 0;
};
static OpCounts g_ops;

// Value numbering: every value carries an id; an operation on operands that
// have been combined the same way before within the unit being counted (the
// same operation on the same ids; + and * commutative) yields the earlier
// value and is not counted again, as common-subexpression elimination would
// keep it.  So a product written twice in the source is one operation.
// Literal constants are numbered by value, inputs each get their own id.
// An operation with an exact 0 operand (additions, multiplications) or an
// exact +-1 factor is structural (a unit vector, an initial accumulator) and
// is folded by the compiler: it is not counted.  The representative state has
// no zero data, so only structural constants are skipped.  Negation and
// fabs are operand modifiers and not counted.
enum { OP_ADD = 1, OP_SUB, OP_MUL, OP_DIV, OP_NEG, OP_ABS, OP_SQRT, OP_EXP, OP_ERFC };
static std::map<std::tuple<int, long, long>, long> g_vn;
static std::map<double, long> g_lit;
static long g_next_id = 1;
inline long lit_id(double x) {
  auto it = g_lit.find(x);
  if (it != g_lit.end()) return it->second;
  return g_lit[x] = g_next_id++;
}
struct CD {
  double v;
  long id;
  constexpr CD(double x = 0.0) : v(x), id(0) {}   // a literal: numbered by its value where used
  constexpr CD(double x, long i) : v(x), id(i) {}
  static CD input(double x) { return CD(x, g_next_id++); }
  CD& operator+=(const CD& o);
  CD& operator-=(const CD& o);
  CD& operator*=(const CD& o);
  CD& operator/=(const CD& o);
};
// the result of op on (a, b); counter incremented only for a new value
inline CD vn(int op, const CD& a, const CD& b, double r, long* counter) {
  long ia = a.id ? a.id : lit_id(a.v), ib = b.id ? b.id : lit_id(b.v);
  if ((op == OP_ADD || op == OP_MUL) && ia > ib) std::swap(ia, ib);
  auto key = std::make_tuple(op, ia, ib);
  auto it = g_vn.find(key);
  if (it != g_vn.end()) return CD(r, it->second);
  if (counter) ++*counter;
  const long id = g_next_id++;
  g_vn[key] = id;
  return CD(r, id);
}
inline CD operator+(const CD& a, const CD& b) {
  if (a.v == 0.0) return b;
  if (b.v == 0.0) return a;
  return vn(OP_ADD, a, b, a.v + b.v, &g_ops.add);
}
inline CD operator-(const CD& a, const CD& b) {
  if (b.v == 0.0) return a;
  return vn(OP_SUB, a, b, a.v - b.v, a.v == 0.0 ? nullptr : &g_ops.add);
}
inline CD operator*(const CD& a, const CD& b) {
  if (a.v == 0.0 || b.v == 0.0) return CD(0.0);
  if (a.v == 1.0) return b;
  if (b.v == 1.0) return a;
  if (a.v == -1.0 || b.v == -1.0) return vn(OP_MUL, a, b, a.v * b.v, nullptr);
  return vn(OP_MUL, a, b, a.v * b.v, &g_ops.mul);
}
inline CD operator/(const CD& a, const CD& b) { return vn(OP_DIV, a, b, a.v / b.v, &g_ops.div); }
inline CD operator-(const CD& a) { return vn(OP_NEG, a, a, -a.v, nullptr); }
inline CD& CD::operator+=(const CD& o) { return *this = *this + o; }
inline CD& CD::operator-=(const CD& o) { return *this = *this - o; }
inline CD& CD::operator*=(const CD& o) { return *this = *this * o; }
inline CD& CD::operator/=(const CD& o) { return *this = *this / o; }
inline bool operator<(const CD& a, const CD& b) { return a.v < b.v; }
inline bool operator>(const CD& a, const CD& b) { return a.v > b.v; }
inline bool operator<=(const CD& a, const CD& b) { return a.v <= b.v; }
inline bool operator>=(const CD& a, const CD& b) { return a.v >= b.v; }
inline bool operator==(const CD& a, const CD& b) { return a.v == b.v; }
inline bool operator!=(const CD& a, const CD& b) { return a.v != b.v; }
inline bool operator!(const CD& a) { return !a.v; }
inline CD fma(const CD& a, const CD& b, const CD& c) { return a * b + c; }
inline CD fabs(const CD& a) { return vn(OP_ABS, a, a, std::fabs(a.v), nullptr); }
inline CD sqrt(const CD& a) { return vn(OP_SQRT, a, a, std::sqrt(a.v), &g_ops.sqrt_); }
inline CD exp(const CD& a) { return vn(OP_EXP, a, a, std::exp(a.v), &g_ops.exp_); }
inline CD erfc(const CD& a) { return vn(OP_ERFC, a, a, std::erfc(a.v), &g_ops.erfc_); }

#define CGKS_OPCOUNT
#define double CD
#include "cgks_device.h"
#undef double

using namespace cgks;

static OpCounts snap() {   // start of a unit: values of earlier units are not reused
  g_vn.clear();
  return g_ops;
}
static OpCounts diff(const OpCounts& a, const OpCounts& b) {
  OpCounts d;
  d.add = b.add - a.add; d.mul = b.mul - a.mul; d.div = b.div - a.div;
  d.sqrt_ = b.sqrt_ - a.sqrt_; d.exp_ = b.exp_ - a.exp_; d.erfc_ = b.erfc_ - a.erfc_;
  return d;
}
static long flops(const OpCounts& c) { return c.add + c.mul + c.div; }

static void emit(const char* name, const OpCounts& c, bool comma) {
  std::printf("    \"%s\": {\"add\": %ld, \"mul\": %ld, \"div\": %ld, \"sqrt\": %ld, \"exp\": %ld, \"erfc\": %ld, \"flops\": %ld}%s\n",
              name, c.add, c.mul, c.div, c.sqrt_, c.exp_, c.erfc_, flops(c), comma ? "," : "");
}

int main() {
  static const TangWT<7> host_tang7[2] = CGKS_TANG7_WEIGHTS;
  static const HermWT host_herm2[2] = CGKS_HERM2_WEIGHTS;
  static const HermWT host_herm4[2] = CGKS_HERM4_WEIGHTS;
  const double gamma = 1.4;
  const Gas gas = make_gas(gamma, 2, 0.01, 1.0, 0.0);
  const double dt = 6e-4, hn = 1.0 / 512, ht = 1.0 / 512;

  // one normal reconstruction (one line, one component)
  OpCounts a = snap();
  Line5 L = normal_line(CD::input(1.1e-4), CD::input(-0.9e-4), CD::input(2.1e-4), CD::input(0.5e-4), CD::input(-0.7e-4),
                        CD::input(1.3e-4), CD::input(0.2e-4), CD::input(1e-6));
  (void)L;
  CD hT, hTN;
  cross_face(CD::input(0.3), CD::input(-0.2), CD::input(0.25), CD::input(0.1), CD::input(ht), hT, hTN);
  const OpCounts recon = diff(a, snap());

  // tangential fits to one Gauss point (4 components): three segments
  CD lines[32][3];
  for (int q = 0; q < 32; ++q)
    for (int l = 0; l < 3; ++l) lines[q][l] = CD::input(1e-5 * (q + 1) * (l + 1));
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 4; ++k) lines[20 + k][l] = CD::input((k == 3 ? 1.8 : 1.0) + 1e-4 * l);
  auto get = [&](int q, int l) { return lines[q][l]; };
  PointIn<4> in;
  CD dev[4], ref[4];
  a = snap();
  tangential_point<3>(get, host_tang7[0], host_herm2[0], CD(1.0), CD::input(hn), CD::input(ht), in, dev, ref);
  const OpCounts tang = diff(a, snap());
  // the sextic through 7 segment averages (four Gauss points per segment)
  CD lines7[32][7];
  for (int q = 0; q < 32; ++q)
    for (int l = 0; l < 7; ++l) lines7[q][l] = CD::input(1e-5 * (q + 1) * (l + 1));
  for (int l = 0; l < 7; ++l)
    for (int k = 0; k < 4; ++k) lines7[20 + k][l] = CD::input((k == 3 ? 1.8 : 1.0) + 1e-4 * l);
  auto get7 = [&](int q, int l) { return lines7[q][l]; };
  {
    PointIn<4> in7;
    a = snap();
    tangential_point<7>(get7, host_tang7[0], host_herm4[0], CD(1.0), CD::input(hn), CD::input(ht), in7, dev, ref);
  }
  const OpCounts tang7 = diff(a, snap());
  a = snap();
  tangential_point<3>(get, host_tang7[0], host_herm2[0], CD(1.0), CD::input(hn), CD::input(ht), in, dev, ref);   // the input of the point counts below
  (void)diff(a, snap());
  for (int k = 0; k < 4; ++k) { in.Wl[k] = CD::input(in.W0[k].v + 1e-9); in.Wr[k] = CD::input(in.W0[k].v - 1e-9); }

  PointOut<4> o;
  a = snap();
  gks_point<4, true>(in, gas, CD::input(dt), o);
  const OpCounts gks1 = diff(a, snap());
  a = snap();
  gks_point<4, false>(in, gas, CD::input(dt), o);
  const OpCounts gks2 = diff(a, snap());

  CD acc[16];
  for (int q = 0; q < 16; ++q) acc[q] = CD(0.0);
  a = snap();
  face_accumulate<4, true>(acc, o, dev, ref, CD::input(dt));
  const OpCounts acc1 = diff(a, snap());
  a = snap();
  face_accumulate<4, false>(acc, o, dev, ref, CD::input(dt));
  const OpCounts acc2 = diff(a, snap());

  // per face segment of a stage: 4 component reconstructions of its own line
  // (with the tangential gradients carried across the face), M Gauss points
  // (tangential fits + evolution + accumulation)
  auto seg = [&](const OpCounts& g, const OpCounts& ac, const OpCounts& tg, long m) {
    OpCounts s;
    s.add = 4 * recon.add + m * (tg.add + g.add + ac.add);
    s.mul = 4 * recon.mul + m * (tg.mul + g.mul + ac.mul);
    s.div = 4 * recon.div + m * (tg.div + g.div + ac.div);
    s.sqrt_ = 4 * recon.sqrt_ + m * (tg.sqrt_ + g.sqrt_ + ac.sqrt_);
    s.exp_ = 4 * recon.exp_ + m * (tg.exp_ + g.exp_ + ac.exp_);
    s.erfc_ = 4 * recon.erfc_ + m * (tg.erfc_ + g.erfc_ + ac.erfc_);
    return s;
  };
  const OpCounts seg1 = seg(gks1, acc1, tang, 2), seg2 = seg(gks2, acc2, tang, 2);
  // four Gauss points per segment with the 7-line stencil (gauss_points = 4)
  const OpCounts seg1g4 = seg(gks1, acc1, tang7, 4), seg2g4 = seg(gks2, acc2, tang7, 4);
  // cell updates per component (see k_update2): stage 1: L, Lt (2 faces x 2 directions,
  // 4 sub, 2 div, 2 add each) 12 + 2 jump sub + W*, P (3 mul 2 add each ~ 10) +
  // 4 gradients (1 sub 1 add 1 div) 12 -> 36; stage 2: Lt 6 + W (2) + 2 gradients (1 sub 1 mul 1 div 1 add) 8 -> 16
  OpCounts up1, up2;
  up1.add = 4 * 20; up1.mul = 4 * 8; up1.div = 4 * 8;
  up2.add = 4 * 8; up2.mul = 4 * 4; up2.div = 4 * 4;
  std::printf("{\n  \"units\": {\n");
  emit("recon_line_component", recon, true);   // normal reconstruction + cross_face
  emit("tangential_point", tang, true);
  emit("gks_point_stage1", gks1, true);
  emit("gks_point_stage2", gks2, true);
  emit("face_segment_stage1", seg1, true);
  emit("face_segment_stage2", seg2, true);
  emit("cell_update_stage1", up1, true);
  emit("cell_update_stage2", up2, true);
  emit("tangential_point_7", tang7, true);
  emit("face_segment_stage1_4pt", seg1g4, true);
  emit("face_segment_stage2_4pt", seg2g4, false);
  std::printf("  },\n");
  const long cell_step = 2 * flops(seg1) + 2 * flops(seg2) + flops(up1) + flops(up2);
  std::printf("  \"flops_per_cell_step\": %ld,\n", cell_step);
  std::printf("  \"transcendentals_per_cell_step\": {\"sqrt\": %ld, \"exp\": %ld, \"erfc\": %ld},\n",
              2 * (seg1.sqrt_ + seg2.sqrt_), 2 * (seg1.exp_ + seg2.exp_), 2 * (seg1.erfc_ + seg2.erfc_));
  std::printf("  \"per_launch_units\": {\n");
  std::printf("    \"xfaces1\": {\"units\": \"ny*(nx+1)\", \"flops_per_unit\": %ld},\n", flops(seg1));
  std::printf("    \"yfaces1\": {\"units\": \"(ny+1)*nx\", \"flops_per_unit\": %ld},\n", flops(seg1));
  std::printf("    \"xfaces2\": {\"units\": \"ny*(nx+1)\", \"flops_per_unit\": %ld},\n", flops(seg2));
  std::printf("    \"yfaces2\": {\"units\": \"(ny+1)*nx\", \"flops_per_unit\": %ld},\n", flops(seg2));
  std::printf("    \"update1\": {\"units\": \"nx*ny\", \"flops_per_unit\": %ld},\n", flops(up1));
  std::printf("    \"update2\": {\"units\": \"nx*ny\", \"flops_per_unit\": %ld}\n", flops(up2));
  std::printf("  },\n");
  std::printf("  \"per_launch_units_4pt\": {\n");
  std::printf("    \"xfaces1\": {\"units\": \"ny*(nx+1)\", \"flops_per_unit\": %ld},\n", flops(seg1g4));
  std::printf("    \"yfaces1\": {\"units\": \"(ny+1)*nx\", \"flops_per_unit\": %ld},\n", flops(seg1g4));
  std::printf("    \"xfaces2\": {\"units\": \"ny*(nx+1)\", \"flops_per_unit\": %ld},\n", flops(seg2g4));
  std::printf("    \"yfaces2\": {\"units\": \"(ny+1)*nx\", \"flops_per_unit\": %ld},\n", flops(seg2g4));
  std::printf("    \"update1\": {\"units\": \"nx*ny\", \"flops_per_unit\": %ld},\n", flops(up1));
  std::printf("    \"update2\": {\"units\": \"nx*ny\", \"flops_per_unit\": %ld}\n", flops(up2));
  std::printf("  }\n}\n");
  return 0;
}
