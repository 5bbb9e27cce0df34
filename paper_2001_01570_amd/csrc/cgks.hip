// Kernels and C ABI of the compact 8th-order gas-kinetic scheme on gfx950.
//
// One time step (two-stage fourth-order method, eq. step-hyper-1) is eight
// launches on the context's stream:
//   begin   (1 thread)   step size from the CFL maximum of the previous step
//   xfaces1, yfaces1     normal reconstruction of line segments into LDS, tangential
//                        fits to the Gauss points, gas-kinetic evolution per point
//   update1              W*, P (partial sums of the final update), gradients of W*
//   xfaces2, yfaces2     same on W*, only F_t and W_tt
//   update2              W^{n+1}, its gradients, CFL maximum and admissibility
//   end     (1 thread)   commit (or keep the old state after a non-physical one)
// The step size, time and status live in device memory so that consecutive
// steps need no host round trip.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <new>
#include <vector>

#include "cgks.h"
#include "cgks_device.h"
#include "tuning_table.h"

namespace cgks {

// Face tile: F faces along the normal x T face segments along the tangential,
// 256 threads (one per Gauss point).  Shapes differ in halo overhead ((T+2 HALO)/T
// reconstructed line segments per face segment) and in the width of the rows
// they read and write; the shape is chosen per direction at run time (tuned).
// M Gauss points per segment (one thread each); the tangential stencil has
// 2 HALO + 1 lines (1: the three nearest segments with two points, 2: five,
// for the tangential-WENO variant, 3: the
// sextic through 7 with four).
template <int F_, int T_, int M_ = 2, int HALO_ = 1>
struct Tile {
  static constexpr int F = F_, T = T_, M = M_, HALO = HALO_;
  static constexpr int H = T_ + 2 * HALO_;  // tangential extent including the halo
  static constexpr int NSEG = F_ * H;       // reconstructed line segments per tile
  static_assert(M_ * F_ * T_ == 256 && (64 / M_) % F_ == 0, "one 256-thread block per tile");
};
using Tile8x16 = Tile<8, 16>;
using Tile4x32 = Tile<4, 32>;
using Tile2x64 = Tile<2, 64>;
constexpr int kTileShapes = 3;
// two points with the 5-segment halo of the tangential-WENO variant
using Tile4x32W = Tile<4, 32, 2, 2>;
using Tile2x64W = Tile<2, 64, 2, 2>;
// four Gauss points per segment with the 7-line stencil (x faces, y faces)
using Tile4x16G4 = Tile<4, 16, 4, 3>;
using Tile2x32G4 = Tile<2, 32, 4, 3>;
constexpr int NQ = 32;          // per segment: 5 quantities x 4 components, 4 reference values, 2 x 4 tangential-gradient data
constexpr int FACE_THREADS = 256;   // one thread per Gauss point of the tile's face segments
// waves per SIMD the face kernels are compiled for (register budget 512 / waves:
// 168 at 3; the latency of the point evaluation needs the occupancy more than
// stage 1 needs its last few registers)
#ifndef FACE_WAVES
#define FACE_WAVES(stage) 3
#endif

// Compiler-level memory barrier between the phases of the point evaluation:
// LDS values are re-read in each phase instead of being held in registers.

struct Geom {
  int dim, nx, ny;
  double dx, dy, eps;
  double inv_dx, inv_dy;
  int bc[4];
  double inflow[4][4];   // conservative inflow state per side
  Gas gas;
  int charv;             // WENO-Z states in characteristic variables
  int sides;             // WENO-weighted slopes of the non-equilibrium sides
  int tw;                // tangential WENO-Z of the WENO-Z states (two points)
};

struct Params {          // written by the host before a batch of steps
  double t_end;          // +inf: no end time
  double dt_override;    // > 0: use this step size
  long long max_step;    // no step begins once the step count reaches this
};

struct Scalars {
  Params prm;
  double t, dt, cfl, fixed_dt, last_dt;
  unsigned long long bad_cell;
  unsigned long long guard_w0, guard_weno;
  long long step;
  int status, active, last, cur;
};

struct Bufs {
  double* lam_part;   // per-block CFL maxima of the last update
  double* S[2];    // state double buffer
  double* Ws;      // intermediate state W*
  double* P;       // W + dt L + dt^2/6 L_t and the gradient counterpart
  double* FX;      // x-face results
  double* FY;      // y-face results
  Scalars* sc;
};

// ---------------------------------------------------------------- boundaries
// Ghost cells are never stored: a cell index outside the grid is mapped to its
// source cell and the boundary rule is applied on load (x rule, then y rule,
// i.e. x ghosts first and y ghosts over all columns).

__device__ __forceinline__ int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int src_index(int i, int n, int bclo, int bchi, int& kind, int& side) {
  if (i >= 0 && i < n) { kind = -1; return i; }
  if (i < 0) {
    kind = bclo; side = 0;
    if (bclo == CGKS_PERIODIC) return wrap(i, n);
    if (bclo == CGKS_WALL || bclo == CGKS_NOSLIP) return -i - 1;
    return 0;
  }
  kind = bchi; side = 1;
  if (bchi == CGKS_PERIODIC) return wrap(i, n);
  if (bchi == CGKS_WALL || bchi == CGKS_NOSLIP) return 2 * n - 1 - i;
  return n - 1;
}

// rule of one side on (W, gradient along dir): free -> zero gradients,
// inflow -> fixed state and zero gradients, walls -> mirror
// Parity of component k under the mirror about a wall normal to axis: the
// normal momentum is odd (slip wall), every momentum for a no-slip wall.
template <int NC>
__device__ __forceinline__ double wall_parity(int kind, int axis, int k) {
  return (k == 1 + axis || (kind == CGKS_NOSLIP && k >= 1 && k <= NC - 2)) ? -1.0 : 1.0;
}

template <int NC>
__device__ __forceinline__ void apply_rule(const Geom& G, int kind, int side, int axis, int dir,
                                           double* W, double* Gd) {
  if (kind < 0 || kind == CGKS_PERIODIC) return;
  if (kind == CGKS_FREE) {
#pragma unroll
    for (int k = 0; k < NC; ++k) Gd[k] = 0.0;
  } else if (kind == CGKS_INFLOW) {
#pragma unroll
    for (int k = 0; k < NC; ++k) { W[k] = G.inflow[side][k]; Gd[k] = 0.0; }
  } else {  // walls: W with its parity, normal gradient opposite parity, tangential same
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double par = wall_parity<NC>(kind, axis, k);
      W[k] *= par;
      Gd[k] *= dir == axis ? -par : par;
    }
  }
}

// Gradient planes of a state buffer (NC averages, then 2 x NC gradient planes
// in 2D, NC in 1D, each N values).  GT = double: FP64 storage; GT = float:
// the gradient planes are stored as FP32 in the same buffer (averages FP64).
template <class GT>
__device__ __forceinline__ const GT* grad_planes(const double* S, size_t N, int nc) {
  return reinterpret_cast<const GT*>(S + nc * N);
}
template <class GT>
__device__ __forceinline__ GT* grad_planes(double* S, size_t N, int nc) {
  return reinterpret_cast<GT*>(S + nc * N);
}

// W and its gradient along dir (0: x, 1: y) of cell (i, j), ghosts included
template <int NC, class GT = double>
__device__ __forceinline__ void load_cell(const double* S, const Geom& G, int i, int j, int dir,
                                          double* W, double* Gd) {
  int kx, sx = 0, ky = -1, sy = 0;
  const int si = src_index(i, G.nx, G.bc[0], G.bc[1], kx, sx);
  int sj = 0;
  if constexpr (NC == 4) sj = src_index(j, G.ny, G.bc[2], G.bc[3], ky, sy);
  const size_t N = (size_t)G.nx * (NC == 4 ? G.ny : 1);
  const size_t id = (size_t)sj * G.nx + si;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    W[k] = S[k * N + id];
    Gd[k] = grad_planes<GT>(S, N, NC)[(NC * dir + k) * N + id];
  }
  apply_rule<NC>(G, kx, sx, 0, dir, W, Gd);
  if constexpr (NC == 4) apply_rule<NC>(G, ky, 2 + sy, 1, dir, W, Gd);
}

// the boundary rules of one component k, x rule then y rule (kinds and sides
// from src_index), on its value w and its gradients along dir (gn) and, with
// TANG, along the other axis (gt)
template <bool TANG>
__device__ __forceinline__ void comp_rule(const Geom& G, int kx, int sx, int ky, int sy, int dir, int k,
                                          double& w, double& gn, double& gt) {
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int kind = a == 0 ? kx : ky;
    if (kind < 0 || kind == CGKS_PERIODIC) continue;
    const int side = a == 0 ? sx : 2 + sy;
    if (kind == CGKS_FREE) {
      gn = 0.0;
      if (TANG) gt = 0.0;
    } else if (kind == CGKS_INFLOW) {
      w = G.inflow[side][k];
      gn = 0.0;
      if (TANG) gt = 0.0;
    } else {  // walls about axis a: the gradient along a has the opposite parity
      const double par = wall_parity<4>(kind, a, k);
      w *= par;
      gn *= dir == a ? -par : par;
      if (TANG) gt *= dir == a ? par : -par;
    }
  }
}

// one component k of W and of its gradients along dir (gn) and along the other
// axis (gt) at cell (i, j), ghosts included (2D)
template <class GT>
__device__ __forceinline__ void load_comp(const double* S, const Geom& G, int i, int j, int dir, int k,
                                          double& w, double& gn, double& gt) {
  int kx, sx = 0, ky, sy = 0;
  const int si = src_index(i, G.nx, G.bc[0], G.bc[1], kx, sx);
  const int sj = src_index(j, G.ny, G.bc[2], G.bc[3], ky, sy);
  const size_t N = (size_t)G.nx * G.ny;
  const size_t id = (size_t)sj * G.nx + si;
  w = S[k * N + id];
  gn = grad_planes<GT>(S, N, 4)[(4 * dir + k) * N + id];
  gt = grad_planes<GT>(S, N, 4)[(4 * (1 - dir) + k) * N + id];
  comp_rule<true>(G, kx, sx, ky, sy, dir, k, w, gn, gt);
}

// the averages only (any storage of the gradients)
template <int NC>
__device__ __forceinline__ void load_avg(const double* S, const Geom& G, int i, int j, double* W) {
  int kx, sx = 0, ky = -1, sy = 0;
  const int si = src_index(i, G.nx, G.bc[0], G.bc[1], kx, sx);
  int sj = 0;
  if constexpr (NC == 4) sj = src_index(j, G.ny, G.bc[2], G.bc[3], ky, sy);
  const size_t N = (size_t)G.nx * (NC == 4 ? G.ny : 1);
  const size_t id = (size_t)sj * G.nx + si;
  double Gd[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) { W[k] = S[k * N + id]; Gd[k] = 0.0; }
  apply_rule<NC>(G, kx, sx, 0, 0, W, Gd);
  if constexpr (NC == 4) apply_rule<NC>(G, ky, 2 + sy, 1, 0, W, Gd);
}

// ---------------------------------------------------------------- step control

// Step size: the CFL maximum of the current state is the max of the per-block
// partial maxima written by the last update (or by the scan after set_state).
__device__ __forceinline__ void begin_body(Scalars* sc, const double* lam_part, int nparts) {
  __shared__ double red[4];
  double lam = 0.0;
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) lam = fmax(lam, lam_part[k]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lam = fmax(lam, __shfl_xor(lam, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lam;
  __syncthreads();
  if (threadIdx.x != 0) return;
  lam = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  sc->active = 0;
  if (sc->status != 0 || sc->step >= sc->prm.max_step) return;
  const double rem = sc->prm.t_end - sc->t;
  if (!(rem > 0.0)) { sc->dt = 0.0; return; }
  double dt = sc->prm.dt_override;
  if (!(dt > 0.0)) dt = sc->fixed_dt > 0.0 ? sc->fixed_dt : sc->cfl / lam;
  int last = 0;
  if (dt * (1.0 + 1e-9) >= rem) { dt = rem; last = 1; }
  if (!(dt > 0.0) || !(dt < INFINITY)) { sc->status = CGKS_ENONPHYS; return; }
  sc->dt = dt;
  sc->last = last;
  sc->active = 1;
}

__global__ __launch_bounds__(256) void k_begin(Scalars* sc, const double* lam_part, int nparts) {
  begin_body(sc, lam_part, nparts);
}

__device__ __forceinline__ void end_body(Scalars* sc) {
  if (threadIdx.x != 0 || !sc->active) return;
  if (sc->status == 0) {
    sc->t = sc->last ? sc->prm.t_end : sc->t + sc->dt;
    sc->step += 1;
    sc->cur ^= 1;
    sc->last_dt = sc->dt;
  }
  sc->active = 0;
}

__global__ void k_end(Scalars* sc) { end_body(sc); }

// block maximum of the per-cell CFL rates, one partial per block (256 threads)
__device__ __forceinline__ void reduce_lambda(double* lam_part, int part, double lam) {
  __shared__ double red[4];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lam = fmax(lam, __shfl_xor(lam, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lam;
  __syncthreads();
  if (threadIdx.x == 0) lam_part[part] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

template <int NC>
__device__ __forceinline__ double cell_lambda(const double* W, const Geom& G) {
  const double ir = 1.0 / W[0];
  const double p = pressure<NC>(W, G.gas.gamma);
  const double c = sqrt(G.gas.gamma * p * ir);
  double l = (fabs(W[1] * ir) + c) / G.dx;
  if constexpr (NC == 4) l = fmax(l, (fabs(W[2] * ir) + c) / G.dy);
  return l;
}

__device__ __forceinline__ void flag_bad(Scalars* sc, unsigned long long cell) {
  atomicMin(&sc->bad_cell, cell);
  atomicMin(&sc->status, CGKS_ENONPHYS);
}

// admissibility and CFL maximum of the current state (after set_state); same
// grid as the final update so that it leaves the same partials
template <int NC>
__global__ __launch_bounds__(256) void k_scan(Geom G, Bufs B) {
  Scalars* sc = B.sc;
  const double* S = B.S[sc->cur];
  int i, j;
  if (NC == 4) { i = blockIdx.x * 64 + (threadIdx.x & 63); j = blockIdx.y * 4 + (threadIdx.x >> 6); }
  else { i = blockIdx.x * 256 + threadIdx.x; j = 0; }
  const size_t N = (size_t)G.nx * (NC == 4 ? G.ny : 1);
  double lam = 0.0;
  if (i < G.nx && j < (NC == 4 ? G.ny : 1)) {
    const size_t id = (size_t)j * G.nx + i;
    double W[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) W[k] = S[k * N + id];
    if (!admissible<NC>(W, G.gas.gamma)) flag_bad(sc, id);
    else lam = cell_lambda<NC>(W, G);
  }
  reduce_lambda(B.lam_part, blockIdx.y * gridDim.x + blockIdx.x, lam);
}

// ---------------------------------------------------------------- 2D faces

// Face kernel of one direction.  DIR 0: x faces (normal x, tangential y);
// DIR 1: y faces (normal y, tangential x, momenta swapped for the evolution).
// Tile: TF faces x TT segments, 256 threads, small enough in LDS and registers
// for two blocks per CU (one block's reconstruction overlaps the other's point
// evaluation).  Phase 1 reconstructs TF x (TT + 2 HALO) line segments (each
// shifted by its own reference cell), with the cells' tangential gradients
// carried across the face, into LDS (CH: the WENO-Z states in characteristic
// variables, from a second pass over the segments); phase 2 runs one Gauss
// point per thread: tangential fits, gas-kinetic evolution, Gauss average
// over the lanes of the segment.
// Tile of this block when consecutive blocks go round-robin to the XCDs: each
// XCD (its own L2) gets a contiguous run of tiles in row-major order, so the
// stencil halos shared by neighbouring tiles are fetched into one L2.
constexpr int NXCD = 8;
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int n = gridDim.x * gridDim.y;
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  const int q = n / NXCD, r = n % NXCD;
  const int x = b % NXCD, local = b / NXCD;
  const int logical = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + local;
  bx = logical % gridDim.x;
  by = logical / gridDim.x;
}

// Tile (bx, by) of the face grid of one direction: DIR 0 tiles (faces, rows),
// DIR 1 tiles (columns, faces).
// lds: the kernel's LDS tile, NQ rows of NSEG line segments.
template <int DIR, int STAGE, class GT = double, class TL = Tile8x16, bool CH = false, bool SS = false,
          bool TW = false>
__device__ __forceinline__ void faces2_body(const Geom& G, const Bufs& B, int bx, int by,
                                            double (*lds)[TL::NSEG]) {
  constexpr int TF = TL::F, TT = TL::T, TH = TL::H, NSEG = TL::NSEG, HALO = TL::HALO;
  Scalars* sc = B.sc;
  if (!sc->active || sc->status != 0) return;
  const double dt = sc->dt;
  const double* S = STAGE == 1 ? B.S[sc->cur] : B.Ws;

  const int nn = DIR == 0 ? G.nx : G.ny;     // cells along the normal
  const int nt = DIR == 0 ? G.ny : G.nx;     // cells along the tangential
  const double hn = DIR == 0 ? G.dx : G.dy;
  const double ht = DIR == 0 ? G.dy : G.dx;
  const int f0 = (DIR == 0 ? bx : by) * TF;
  const int t0 = (DIR == 0 ? by : bx) * TT;

  // phase 1: line segments (face f, tangential index tt), one (component,
  // segment) pair per item, component-major so that consecutive threads read
  // consecutive cells along x.  The 4 stencil cells f-2..f+1 of a line come
  // straight from memory (each cell serves 4 lines: cache hits); tiles away
  // from the boundary skip the boundary rules, which map every index in
  // [-2, n + 1] into the grid.
  {
    const int i0 = DIR == 0 ? f0 - 2 : t0 - HALO, j0 = DIR == 0 ? t0 - HALO : f0 - 2;
    const bool interior = i0 >= 0 && j0 >= 0 && i0 + TH <= G.nx && j0 + TH <= G.ny;
    constexpr bool charv = CH;
    const size_t N = (size_t)G.nx * G.ny;
#pragma unroll 1
    for (int item = threadIdx.x; item < NSEG * 4; item += FACE_THREADS) {
      const int k = item / NSEG, s = item % NSEG;
      int fl, tl, pos;
      if (DIR == 0) { tl = s / TF; fl = s % TF; pos = tl * TF + fl; }
      else { fl = s / TH; tl = s % TH; pos = fl * TH + tl; }
      const int f = f0 + fl, ta = t0 - HALO + tl;
      if (f > nn || ta > nt + HALO - 1) continue;
      double w[4], gd[4], gt[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int i = DIR == 0 ? f - 2 + m : ta, j = DIR == 0 ? ta : f - 2 + m;
        if (interior) {
          const size_t id = (size_t)j * G.nx + i;
          w[m] = S[k * N + id];
          gd[m] = grad_planes<GT>(S, N, 4)[(4 * DIR + k) * N + id];
          gt[m] = grad_planes<GT>(S, N, 4)[(4 * (1 - DIR) + k) * N + id];
        } else {
          load_comp<GT>(S, G, i, j, DIR, k, w[m], gd[m], gt[m]);
        }
      }
      const double ref = w[1];
      const double a = w[0] - ref, c = w[2] - ref, d = w[3] - ref;
      const double A = hn * gd[0], Bq = hn * gd[1], C = hn * gd[2], D = hn * gd[3];
      double v, vn, vnn;
      p7_shifted(a, c, d, A, Bq, C, D, v, vn, vnn);
      lds[0 * 4 + k][pos] = v;
      lds[1 * 4 + k][pos] = vn;
      lds[2 * 4 + k][pos] = vnn;
      if constexpr (!charv) {
        lds[3 * 4 + k][pos] = weno_left(a, c, d, A, Bq, C, D, G.eps);
        lds[4 * 4 + k][pos] = weno_left(d - c, -c, a - c, -D, -C, -Bq, -A, G.eps) + c;
      }
      if constexpr (SS) {   // the side slopes of the evaluated variant (h-scaled)
        double sl, sr;
        weno_left_s<true>(a, c, d, A, Bq, C, D, G.eps, &sl);
        weno_left_s<true>(d - c, -c, a - c, -D, -C, -Bq, -A, G.eps, &sr);
        lds[NQ + k][pos] = sl;
        lds[NQ + 4 + k][pos] = -sr;
      }
      lds[20 + k][pos] = ref;
      // the cells' tangential gradient carried across the face by the cubic
      // through the 4 stencil cells: value and (unit-width) normal derivative
      double hT, hTN;
      cross_face(gt[0], gt[1], gt[2], gt[3], ht, hT, hTN);
      lds[24 + k][pos] = hT;
      lds[28 + k][pos] = hTN;
    }
    // characteristic variables: the WENO-Z states of each line segment from
    // all four components (normal momentum first on y faces)
    if constexpr (charv) {
#pragma unroll 1
      for (int s = threadIdx.x; s < NSEG; s += FACE_THREADS) {
        int fl, tl, pos;
        if (DIR == 0) { tl = s / TF; fl = s % TF; pos = tl * TF + fl; }
        else { fl = s / TH; tl = s % TH; pos = fl * TH + tl; }
        const int f = f0 + fl, ta = t0 - HALO + tl;
        if (f > nn || ta > nt + HALO - 1) continue;
        // the 4 cells: source indices, loads, then the per-component rules of
        // the loop above (the array form, load_cell, compiled in this kernel
        // gave wrong ghost values at no-slip walls normal to the face
        // direction)
        double Wc[4][4], Dc[4][4];
        int kx[4], sx[4], ky[4], sy[4];
        size_t id[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int i = DIR == 0 ? f - 2 + m : ta, j = DIR == 0 ? ta : f - 2 + m;
          sx[m] = 0;
          sy[m] = 0;
          const int si = src_index(i, G.nx, G.bc[0], G.bc[1], kx[m], sx[m]);
          const int sj = src_index(j, G.ny, G.bc[2], G.bc[3], ky[m], sy[m]);
          id[m] = (size_t)sj * G.nx + si;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            Wc[m][k] = S[k * N + id[m]];
            Dc[m][k] = grad_planes<GT>(S, N, 4)[(4 * DIR + k) * N + id[m]];
          }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (!interior) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              double unused = 0.0;
              comp_rule<false>(G, kx[m], sx[m], ky[m], sy[m], DIR, k, Wc[m][k], Dc[m][k], unused);
            }
          }
          if (DIR == 1) {
            double t = Wc[m][1]; Wc[m][1] = Wc[m][2]; Wc[m][2] = t;
            t = Dc[m][1]; Dc[m][1] = Dc[m][2]; Dc[m][2] = t;
          }
        }
        double Wm[4], L[4][4], R[4][4], a[4], c[4], d[4], A[4], Bq[4], C[4], D[4], wl[4], wr[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double ref = Wc[1][k];
          Wm[k] = 0.5 * (Wc[1][k] + Wc[2][k]);
          a[k] = Wc[0][k] - ref; c[k] = Wc[2][k] - ref; d[k] = Wc[3][k] - ref;
          A[k] = hn * Dc[0][k]; Bq[k] = hn * Dc[1][k]; C[k] = hn * Dc[2][k]; D[k] = hn * Dc[3][k];
        }
        if (!char_basis<4>(Wm, G.gas.gamma, L, R)) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) L[i][j] = R[i][j] = i == j ? 1.0 : 0.0;
        }
        weno_char<4>(L, R, a, c, d, A, Bq, C, D, G.eps, wl, wr);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int ks = DIR == 1 && (k == 1 || k == 2) ? 3 - k : k;
          lds[3 * 4 + ks][pos] = wl[k];
          lds[4 * 4 + ks][pos] = wr[k];
        }
      }
    }
  }
  __syncthreads();

  // phase 2: one Gauss point per thread (face_point); the mirrored point reads
  // the stencil lines in reverse order.  Two points: waves 0-1 evaluate the
  // first point of the 128 segments and waves 2-3 the mirrored one, so that
  // the mirror sign and the line order are the same for a whole wave;
  // consecutive lanes take consecutive segments (along the face within a
  // row of TF faces for x faces, along the face for y faces), so their LDS
  // reads are consecutive.  Four points: waves 0-1 take the inner pair of
  // nodes and waves 2-3 the outer pair (pr, the same for a whole wave, so
  // that the node weights are scalar loads), each wave 32 segments with the
  // mirror pair in its two half-waves (x faces) or adjacent lanes (y faces);
  // point gp = 2 pr + mirror.
  constexpr int M = TL::M, NL = 2 * HALO + 1;
  int mirror, fl, tl, seg = 0, pr = 0;
  if constexpr (M == 2) {
    mirror = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
    seg = threadIdx.x & 127;
    if (DIR == 0) { fl = seg % TF; tl = seg / TF; }
    else { tl = seg % TT; fl = seg / TT; }
  } else {
    const int lane = threadIdx.x & 63;
    pr = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
    mirror = DIR == 0 ? lane >> 5 : lane & 1;
    seg = 32 * ((threadIdx.x >> 6) & 1) + (DIR == 0 ? (lane & 31) : (lane >> 1));
    if (DIR == 0) { fl = seg % TF; tl = seg / TF; }
    else { tl = seg % TT; fl = seg / TT; }
  }
  constexpr int PAIR = DIR == 0 ? 32 : 1;   // four points: lane distance of the mirror pair
  const int f = f0 + fl, tt = t0 + tl;
  const bool live = f <= nn && tt < nt;
  const int lstride = DIR == 0 ? TF : 1;    // next stencil line in LDS
  const int lfirst = (DIR == 0 ? tl * TF + fl : fl * TH + tl) + (mirror ? (NL - 1) * lstride : 0);
  const int lstep = mirror ? -lstride : lstride;
  auto get = [&](int q, int l) { return lds[q][lfirst + lstep * l]; };
  auto right_cell = [&](int k) {            // the cell right of the face, boundary rule applied
    double W[4];
    if (DIR == 0) load_avg<4>(S, G, f, tt, W); else load_avg<4>(S, G, tt, f, W);
    return W[k];
  };
  constexpr int NO = STAGE == 1 ? 16 : 8;
  double acc[NO] = {};
  int guard = 0, nbad = 0;
  const double inv_hn = DIR == 0 ? G.inv_dx : G.inv_dy, inv_ht = DIR == 0 ? G.inv_dy : G.inv_dx;
  const double dsg = mirror ? -1.0 : 1.0;
  if constexpr (M == 2 && TW) {
    // the tangential-WENO variant: the nonlinear states from the 5 segments,
    // the rest from the middle three as with the 3-segment halo
    static_assert(HALO == 2, "the two-point tangential WENO needs the 5-segment tiles");
    if (live) {
      double tws[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double rj = get(20 + k, 2);
        double sl[5], sr[5];
#pragma unroll
        for (int l = 0; l < 5; ++l) {
          const double off = get(20 + k, l) - rj;
          sl[l] = off + get(12 + k, l);
          sr[l] = off + get(16 + k, l);
        }
        tws[k] = rj + tang_weno5(sl, G.eps);
        tws[4 + k] = rj + tang_weno5(sr, G.eps);
      }
      auto get3 = [&](int q, int l) { return get(q, l + 1); };
      face_point<DIR, STAGE == 1, 3, false, true>(get3, right_cell, kTang7[0], kHerm2[0], dsg, inv_hn,
                                                  mirror ? -inv_ht : inv_ht, G.gas, dt, acc, guard, nbad, 0.5, tws);
    }
  } else if constexpr (M == 2) {
    if (live)
      face_point<DIR, STAGE == 1, NL, SS>(get, right_cell, kTang7[0], kHerm2[0], dsg, inv_hn,
                                          mirror ? -inv_ht : inv_ht, G.gas, dt, acc, guard, nbad);
  } else if constexpr (TW) {
    // four points with the tangential WENO: the middle five of the seven
    // segments at this wave's node
    if (live) {
      const TwNode node = pr ? kTwOuter : kTwInner;
      double tws[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double rj = get(20 + k, 3);
        double sl[5], sr[5];
#pragma unroll
        for (int l = 0; l < 5; ++l) {
          const double off = get(20 + k, l + 1) - rj;
          sl[l] = off + get(12 + k, l + 1);
          sr[l] = off + get(16 + k, l + 1);
        }
        tws[k] = rj + tang_weno5_at(sl, G.eps, node);
        tws[4 + k] = rj + tang_weno5_at(sr, G.eps, node);
      }
      face_point<DIR, STAGE == 1, NL, false, true>(get, right_cell, kTang7[pr], kHerm4[pr], dsg, inv_hn,
                                                   mirror ? -inv_ht : inv_ht, G.gas, dt, acc, guard, nbad,
                                                   pr ? kGauss4Outer : kGauss4Inner, tws);
    }
  } else {
    if (live)
      face_point<DIR, STAGE == 1, NL, SS>(get, right_cell, kTang7[pr], kHerm4[pr], dsg, inv_hn,
                                          mirror ? -inv_ht : inv_ht, G.gas, dt, acc, guard, nbad,
                                          pr ? kGauss4Outer : kGauss4Inner);
  }
  if (guard) atomicAdd(&sc->guard_w0, 1ull);
  if (nbad) atomicAdd(&sc->guard_weno, (unsigned long long)nbad);

  // Gauss average over the points of the segment (each point weighted in
  // face_point), once every wave has finished reading the reconstruction:
  // two points, the mirrored point's waves hand their results to the first
  // point's through LDS; four points, the mirror pairs are summed by a lane
  // exchange and the outer pair's waves hand their sums to the inner pair's
  // through LDS.  The first point's lane writes.
  if constexpr (M == 2) {
    __syncthreads();
    if (mirror == 1 && live) {
#pragma unroll
      for (int q = 0; q < NO; ++q) lds[q][seg] = acc[q];
    }
    __syncthreads();
    if (mirror == 1 || !live) return;
#pragma unroll
    for (int q = 0; q < NO; ++q) acc[q] += lds[q][seg];
  } else {
#pragma unroll
    for (int q = 0; q < NO; ++q) acc[q] += __shfl_xor(acc[q], PAIR, 64);
  }
  if constexpr (M == 4) {
    __syncthreads();
    if (pr == 1 && mirror == 0 && live) {
#pragma unroll
      for (int q = 0; q < NO; ++q) lds[q][seg] = acc[q];
    }
    __syncthreads();
    if (pr == 1 || !live) return;
#pragma unroll
    for (int q = 0; q < NO; ++q) acc[q] += lds[q][seg];
  }
  if (mirror) return;
  double* F = DIR == 0 ? B.FX : B.FY;
  // x faces: [q][row][face] (nx+1 per row); y faces: [q][face][column] (nx per row)
  const size_t plane = DIR == 0 ? (size_t)G.ny * (G.nx + 1) : (size_t)(G.ny + 1) * G.nx;
  const size_t idx = DIR == 0 ? (size_t)tt * (G.nx + 1) + f : (size_t)f * G.nx + tt;
#pragma unroll
  for (int q = 0; q < NO; ++q) F[q * plane + idx] = acc[q];
}

template <int DIR, int STAGE, class GT, class TL, bool CH, bool SS = false, bool TW = false>
__global__ __launch_bounds__(FACE_THREADS, FACE_WAVES(STAGE)) void k_faces2(Geom G, Bufs B) {
  __shared__ double lds[SS ? NQ + 8 : NQ][TL::NSEG];   // SS: 8 rows of side slopes
  int bx, by;
  xcd_tile(bx, by);
  faces2_body<DIR, STAGE, GT, TL, CH, SS, TW>(G, B, bx, by, lds);
}

// ---------------------------------------------------------------- 2D update

// Cell block (bx, by) of 64 x 4 cells; part: its index among the CFL partials.
template <int STAGE, class GT = double>
__device__ __forceinline__ void update2_body(const Geom& G, const Bufs& B, int bx, int by, int part) {
  Scalars* sc = B.sc;
  if (!sc->active || sc->status != 0) return;
  const double dt = sc->dt;
  const int i = bx * 64 + (threadIdx.x & 63);
  const int j = by * 4 + (threadIdx.x >> 6);
  const bool in = i < G.nx && j < G.ny;
  const size_t N = (size_t)G.nx * G.ny;
  const size_t id = (size_t)j * G.nx + i;
  const size_t px = (size_t)G.ny * (G.nx + 1), py = (size_t)(G.ny + 1) * G.nx;
  const size_t xl = (size_t)j * (G.nx + 1) + i, xr = xl + 1;
  const size_t yl = (size_t)j * G.nx + i, yr = yl + G.nx;
  double lam = 0.0;
  if (in) {
    if (STAGE == 1) {
      const double* S = B.S[sc->cur];
      double W[4], Wm[4], Wb[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) W[k] = S[k * N + id];
      load_avg<4>(S, G, i - 1, j, Wm);
      load_avg<4>(S, G, i, j - 1, Wb);
      double Wst[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double* FX = B.FX;
        const double* FY = B.FY;
        double L = -(FX[k * px + xr] - FX[k * px + xl]) / G.dx;
        double Lt = -(FX[(4 + k) * px + xr] - FX[(4 + k) * px + xl]) / G.dx;
        L += -(FY[k * py + yr] - FY[k * py + yl]) / G.dy;
        Lt += -(FY[(4 + k) * py + yr] - FY[(4 + k) * py + yl]) / G.dy;
        const double jx = W[k] - Wm[k], jy = W[k] - Wb[k];
        Wst[k] = W[k] + 0.5 * dt * L + dt * dt / 8.0 * Lt;
        B.Ws[k * N + id] = Wst[k];
        B.P[k * N + id] = W[k] + dt * L + dt * dt / 6.0 * Lt;
        GT* gws = grad_planes<GT>(B.Ws, N, 4);
        GT* gp = grad_planes<GT>(B.P, N, 4);
        gws[k * N + id] = (GT)(((FX[(8 + k) * px + xr] - FX[(8 + k) * px + xl]) + jx) / G.dx);
        gp[k * N + id] = (GT)(((FX[(12 + k) * px + xr] - FX[(12 + k) * px + xl]) + jx) / G.dx);
        gws[(4 + k) * N + id] = (GT)(((FY[(8 + k) * py + yr] - FY[(8 + k) * py + yl]) + jy) / G.dy);
        gp[(4 + k) * N + id] = (GT)(((FY[(12 + k) * py + yr] - FY[(12 + k) * py + yl]) + jy) / G.dy);
      }
      if (!admissible<4>(Wst, G.gas.gamma)) flag_bad(sc, id);
    } else {
      double* So = B.S[sc->cur ^ 1];
      const double c3 = dt * dt / 3.0;
      double Wn[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double* FX = B.FX;
        const double* FY = B.FY;
        double Lt = -(FX[k * px + xr] - FX[k * px + xl]) / G.dx;
        Lt += -(FY[k * py + yr] - FY[k * py + yl]) / G.dy;
        Wn[k] = B.P[k * N + id] + c3 * Lt;
        So[k * N + id] = Wn[k];
        GT* go = grad_planes<GT>(So, N, 4);
        const GT* gp = grad_planes<GT>(B.P, N, 4);
        go[k * N + id] = (GT)((double)gp[k * N + id] + c3 * (FX[(4 + k) * px + xr] - FX[(4 + k) * px + xl]) / G.dx);
        go[(4 + k) * N + id] =
            (GT)((double)gp[(4 + k) * N + id] + c3 * (FY[(4 + k) * py + yr] - FY[(4 + k) * py + yl]) / G.dy);
      }
      if (!admissible<4>(Wn, G.gas.gamma)) flag_bad(sc, id);
      else lam = cell_lambda<4>(Wn, G);
    }
  }
  if (STAGE == 2) reduce_lambda(B.lam_part, part, lam);
}

template <int STAGE, class GT>
__global__ __launch_bounds__(256) void k_update2(Geom G, Bufs B) {
  update2_body<STAGE, GT>(G, B, blockIdx.x, blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x);
}

// State layout conversion for FP32 storage (2D): the averages are copied, the
// 8 gradient planes converted (to storage: rounded to nearest FP32).
__global__ __launch_bounds__(256) void k_to_storage32(const double* src, double* dst, size_t N) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) dst[k * N + id] = src[k * N + id];
  float* g = grad_planes<float>(dst, N, 4);
#pragma unroll
  for (int q = 0; q < 8; ++q) g[q * N + id] = (float)src[(4 + q) * N + id];
}

__global__ __launch_bounds__(256) void k_from_storage32(const double* src, double* dst, size_t N) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) dst[k * N + id] = src[k * N + id];
  const float* g = grad_planes<float>(src, N, 4);
#pragma unroll
  for (int q = 0; q < 8; ++q) dst[(4 + q) * N + id] = (double)g[q * N + id];
}

// ---------------------------------------------------------------- 1D

// face f (0..nx) of one stage
template <int STAGE>
__device__ __forceinline__ void faces1_body(const Geom& G, const Bufs& B, int f) {
  Scalars* sc = B.sc;
  if (!sc->active || sc->status != 0) return;
  const double dt = sc->dt;
  const double* S = STAGE == 1 ? B.S[sc->cur] : B.Ws;
  if (f > G.nx) return;
  const double h = G.dx;
  double Wc[4][3], Dc[4][3];
#pragma unroll
  for (int m = 0; m < 4; ++m) load_cell<3>(S, G, f - 2 + m, 0, 0, Wc[m], Dc[m]);
  PointIn<3> in;
  double dev[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ref = Wc[1][k];
    const Line5 L = normal_line(Wc[0][k] - ref, Wc[2][k] - ref, Wc[3][k] - ref, h * Dc[0][k], h * Dc[1][k],
                                h * Dc[2][k], h * Dc[3][k], G.eps);
    dev[k] = L.v;
    in.W0[k] = ref + L.v;
    in.Wn[k] = L.vn / h;
    in.Wnn[k] = L.vnn / (h * h);
    in.Wt[k] = 0.0; in.Wnt[k] = 0.0; in.Wtt[k] = 0.0;
    in.Wl[k] = ref + L.wl;
    in.Wr[k] = ref + L.wr;
  }
  if (G.charv) {   // the WENO-Z states in the characteristic variables of the mean of cells i, i+1
    double Wm[3], L[3][3], R[3][3], a[3], c[3], d[3], A[3], Bv[3], C[3], D[3], wl[3], wr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double ref = Wc[1][k];
      Wm[k] = 0.5 * (Wc[1][k] + Wc[2][k]);
      a[k] = Wc[0][k] - ref; c[k] = Wc[2][k] - ref; d[k] = Wc[3][k] - ref;
      A[k] = h * Dc[0][k]; Bv[k] = h * Dc[1][k]; C[k] = h * Dc[2][k]; D[k] = h * Dc[3][k];
    }
    if (!char_basis<3>(Wm, G.gas.gamma, L, R)) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) L[i][j] = R[i][j] = i == j ? 1.0 : 0.0;
    }
    weno_char<3>(L, R, a, c, d, A, Bv, C, D, G.eps, wl, wr);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      in.Wl[k] = Wc[1][k] + wl[k];
      in.Wr[k] = Wc[1][k] + wr[k];
    }
  }
  // normal slopes of the two non-equilibrium sides: the linear
  // reconstruction's, or (the evaluated variant) the WENO-weighted slopes of
  // the candidates; a side that falls back to its cell average takes the
  // linear slope
  double Wln[3], Wrn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) Wln[k] = Wrn[k] = in.Wn[k];
  if (G.sides) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double ref = Wc[1][k];
      const double a = Wc[0][k] - ref, c = Wc[2][k] - ref, d = Wc[3][k] - ref;
      const double A = h * Dc[0][k], Bq = h * Dc[1][k], C = h * Dc[2][k], D = h * Dc[3][k];
      double sl, sr;
      weno_left_s<true>(a, c, d, A, Bq, C, D, G.eps, &sl);
      weno_left_s<true>(d - c, -c, a - c, -D, -C, -Bq, -A, G.eps, &sr);
      Wln[k] = sl / h;
      Wrn[k] = -sr / h;
    }
  }
  int gweno = 0;
  if (!admissible<3>(in.Wl, G.gas.gamma)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { in.Wl[k] = Wc[1][k]; Wln[k] = in.Wn[k]; }
    ++gweno;
  }
  if (!admissible<3>(in.Wr, G.gas.gamma)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { in.Wr[k] = Wc[2][k]; Wrn[k] = in.Wn[k]; }
    ++gweno;
  }
  PointOut<3> o;
  gks_point<3, STAGE == 1>(in, Wln, Wrn, G.gas, dt, o);
  if (o.guard) atomicAdd(&sc->guard_w0, 1ull);
  if (gweno) atomicAdd(&sc->guard_weno, (unsigned long long)gweno);
  const size_t plane = (size_t)G.nx + 1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (STAGE == 1) {
      const double d0 = o.guard ? o.W0[k] - Wc[1][k] : dev[k];
      B.FX[k * plane + f] = o.F[k];
      B.FX[(3 + k) * plane + f] = o.Ft[k];
      B.FX[(6 + k) * plane + f] = d0 + 0.5 * dt * o.Wt[k] + dt * dt / 8.0 * o.Wtt[k] + o.Nh[k];
      B.FX[(9 + k) * plane + f] = d0 + dt * o.Wt[k] + dt * dt / 6.0 * o.Wtt[k] + o.Nf[k];
    } else {
      B.FX[k * plane + f] = o.Ft[k];
      B.FX[(3 + k) * plane + f] = o.Wtt[k];
    }
  }
}

template <int STAGE>
__global__ __launch_bounds__(256) void k_faces1(Geom G, Bufs B) {
  faces1_body<STAGE>(G, B, blockIdx.x * blockDim.x + threadIdx.x);
}

// cell i (0..nx-1) of one stage; returns the cell's CFL rate after stage 2 (else 0)
template <int STAGE>
__device__ __forceinline__ double update1_body(const Geom& G, const Bufs& B, int i) {
  Scalars* sc = B.sc;
  if (!sc->active || sc->status != 0) return 0.0;
  const double dt = sc->dt;
  const size_t N = (size_t)G.nx;
  const size_t plane = N + 1;
  double lam = 0.0;
  if (i < G.nx) {
    if (STAGE == 1) {
      const double* S = B.S[sc->cur];
      double W[3], Wm[3], Wst[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) W[k] = S[k * N + i];
      load_avg<3>(S, G, i - 1, 0, Wm);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double L = -(B.FX[k * plane + i + 1] - B.FX[k * plane + i]) / G.dx;
        const double Lt = -(B.FX[(3 + k) * plane + i + 1] - B.FX[(3 + k) * plane + i]) / G.dx;
        const double jx = W[k] - Wm[k];
        Wst[k] = W[k] + 0.5 * dt * L + dt * dt / 8.0 * Lt;
        B.Ws[k * N + i] = Wst[k];
        B.P[k * N + i] = W[k] + dt * L + dt * dt / 6.0 * Lt;
        B.Ws[(3 + k) * N + i] = ((B.FX[(6 + k) * plane + i + 1] - B.FX[(6 + k) * plane + i]) + jx) / G.dx;
        B.P[(3 + k) * N + i] = ((B.FX[(9 + k) * plane + i + 1] - B.FX[(9 + k) * plane + i]) + jx) / G.dx;
      }
      if (!admissible<3>(Wst, G.gas.gamma)) flag_bad(sc, i);
    } else {
      double* So = B.S[sc->cur ^ 1];
      const double c3 = dt * dt / 3.0;
      double Wn[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double Lt = -(B.FX[k * plane + i + 1] - B.FX[k * plane + i]) / G.dx;
        Wn[k] = B.P[k * N + i] + c3 * Lt;
        So[k * N + i] = Wn[k];
        So[(3 + k) * N + i] = B.P[(3 + k) * N + i] + c3 * (B.FX[(3 + k) * plane + i + 1] - B.FX[(3 + k) * plane + i]) / G.dx;
      }
      if (!admissible<3>(Wn, G.gas.gamma)) flag_bad(sc, i);
      else lam = cell_lambda<3>(Wn, G);
    }
  }
  return lam;
}

template <int STAGE>
__global__ __launch_bounds__(256) void k_update1(Geom G, Bufs B) {
  // a step that does not run leaves the CFL partials of the last one that did
  if (!B.sc->active || B.sc->status != 0) return;
  const double lam = update1_body<STAGE>(G, B, blockIdx.x * blockDim.x + threadIdx.x);
  if (STAGE == 2) reduce_lambda(B.lam_part, blockIdx.x, lam);
}

// Small 1D grids: nsteps whole steps in one launch of one block.  The phases
// of a step run in the order of the separate kernels (begin, faces 1,
// update 1, faces 2, update 2, end) with block barriers in place of the
// kernel boundaries, on the same device functions (the compiler may contract
// a few operations differently here, so the results agree with the separate
// launches to rounding, not always bitwise).  Every barrier is reached by every thread: the
// bodies return early on their own, never around a barrier.  The CFL partials
// are written per 256 cells, as by the update grid.
__global__ __launch_bounds__(256) void k_steps1(Geom G, Bufs B, int nsteps, int nparts) {
  __shared__ double red[4];
  Scalars* sc = B.sc;
  for (int s = 0; s < nsteps; ++s) {
    begin_body(sc, B.lam_part, nparts);
    __syncthreads();
    for (int f = threadIdx.x; f <= G.nx; f += 256) faces1_body<1>(G, B, f);
    __syncthreads();
    for (int i = threadIdx.x; i < G.nx; i += 256) update1_body<1>(G, B, i);
    __syncthreads();
    for (int f = threadIdx.x; f <= G.nx; f += 256) faces1_body<2>(G, B, f);
    __syncthreads();
    for (int b = 0; b < nparts; ++b) {
      double lam = update1_body<2>(G, B, b * 256 + (int)threadIdx.x);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) lam = fmax(lam, __shfl_xor(lam, o, 64));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lam;
      __syncthreads();
      if (threadIdx.x == 0 && sc->active && sc->status == 0)   // as k_update1: only a step that runs
        B.lam_part[b] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
      __syncthreads();
    }
    end_body(sc);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- batch

// Many independent 2D problems advanced by the same launches.  A batched
// launch covers a device-resident work list: the tiles (or cell blocks) of
// all running slots, one block each.  Its grid is a power-of-two bucket of
// the list's length (blocks past the end return at once), so the list may
// change between runs without a new graph until it outgrows its bucket.
// Within a run each slot keeps its own step size, time and status.  Slots
// of each kind (Gauss points x gradient storage) have face work lists of
// their own, launched with that kind's kernels; the updates have one list per
// storage.
constexpr int kMaxSlots = 1024;

struct SlotDev {
  Geom G;
  Bufs B;
  int gw[2];           // tiles along the first axis of the x-face and y-face grids
  int guw;             // blocks along x of the update grid
  int nparts;          // CFL partial maxima (update blocks)
};

// Slot kinds: the face kernels differ by Gauss points (bit 0: four),
// gradient storage (bit 1: FP32) and the variables of the WENO-Z states
// (bit 2: characteristic).
// bits 0-1: four points, FP32 storage; bits 2-3 (exclusive options):
// characteristic variables, the side-slope variant, the tangential-WENO
// variant (two points only)
enum { BK_G2 = 0, BK_G4 = 1, BK_G2_F32 = 2, BK_G4_F32 = 3, BK_CHAR = 4, BK_SIDE = 8, BK_TW = 12, BK_KINDS = 16 };
constexpr bool kind_g4(int kind) { return kind & 1; }
constexpr bool kind_f32(int kind) { return kind & 2; }
constexpr bool kind_char(int kind) { return (kind & 12) == BK_CHAR; }
constexpr bool kind_side(int kind) { return (kind & 12) == BK_SIDE; }
constexpr bool kind_tw(int kind) { return (kind & 12) == BK_TW; }

// Running slots of one kind: work item i of a face direction belongs to the
// k-th of them when pre[dir][k] <= i < pre[dir][k + 1] (face tiles).
struct FaceList {
  int n;
  int slot[kMaxSlots];
  int pre[2][kMaxSlots + 1];
};
// Running slots of one storage (0: FP64, 1: FP32 gradients): update blocks.
struct UpdateList {
  int n;
  int slot[kMaxSlots];
  int pre[kMaxSlots + 1];
};
struct BatchTable {
  int n;               // every running slot (step begin and end)
  int slot[kMaxSlots];
  FaceList face[BK_KINDS];
  UpdateList upd[2];
};

__device__ __forceinline__ int find_slot(const int* pre, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Work item of this block in a list of `total` items, or -1: consecutive
// blocks go round-robin to the XCDs, so each XCD takes a contiguous share of
// the list (neighbouring tiles of a slot share an L2).  The grid (a multiple
// of the XCD count) must hold at least NXCD * ceil(total / NXCD) blocks.
__device__ __forceinline__ int xcd_item(int total) {
  const int per = (total + NXCD - 1) / NXCD;
  const int x = blockIdx.x % NXCD, local = blockIdx.x / NXCD;
  const int item = x * per + local;
  return local < per && item < total ? item : -1;
}

__global__ __launch_bounds__(256) void kb_begin(const SlotDev* slots, const BatchTable* tab) {
  if ((int)blockIdx.x >= tab->n) return;
  const SlotDev& sd = slots[tab->slot[blockIdx.x]];
  begin_body(sd.B.sc, sd.B.lam_part, sd.nparts);
}

__global__ void kb_end(const SlotDev* slots, const BatchTable* tab) {
  if ((int)blockIdx.x >= tab->n) return;
  end_body(slots[tab->slot[blockIdx.x]].B.sc);
}

// Face tiles of the slots of one kind (tile shape TL, gradient storage GT,
// characteristic variables CH, side-slope variant SS).
template <int DIR, int STAGE, class GT, class TL, bool CH, bool SS = false, bool TW = false>
__global__ __launch_bounds__(FACE_THREADS, FACE_WAVES(STAGE)) void kb_faces(const SlotDev* slots,
                                                                            const BatchTable* tab, int kind) {
  __shared__ double lds[SS ? NQ + 8 : NQ][TL::NSEG];
  const FaceList& L = tab->face[kind];
  const int n = L.n;
  const int* pre = L.pre[DIR];
  const int item = xcd_item(pre[n]);
  if (item < 0) return;
  const int k = find_slot(pre, n, item);
  const SlotDev& sd = slots[L.slot[k]];
  const int local = item - pre[k];
  const int w = sd.gw[DIR];
  faces2_body<DIR, STAGE, GT, TL, CH, SS, TW>(sd.G, sd.B, local % w, local / w, lds);
}

template <int STAGE, class GT>
__global__ __launch_bounds__(256) void kb_update(const SlotDev* slots, const BatchTable* tab, int storage) {
  const UpdateList& L = tab->upd[storage];
  const int n = L.n;
  const int item = blockIdx.x;
  if (item >= L.pre[n]) return;
  const int k = find_slot(L.pre, n, item);
  const SlotDev& sd = slots[L.slot[k]];
  const int local = item - L.pre[k];
  update2_body<STAGE, GT>(sd.G, sd.B, local % sd.guw, local / sd.guw, local);
}

}  // namespace cgks

// ================================================================ host side

using namespace cgks;

constexpr int kKinds = 8;
constexpr size_t kEventPairs = 1024;

struct cgks_ctx {
  cgks_config cfg;
  hipStream_t stream;
  Geom G;
  Bufs B;
  Scalars* host_sc;     // pinned mirror
  size_t N, nf;
  int has_state;
  // profiling: event pairs around hot kernel launches
  int profiling;
  std::vector<hipEvent_t>* events;
  std::vector<int>* ev_kind;
  size_t ev_used;
  double ms[kKinds];
  long calls[kKinds];
  // run_steps replays GRAPH_STEPS steps as one HIP graph (captured on first use)
  hipGraphExec_t exec;
  int tile[2];          // face tile shape per direction (0: 8x16, 1: 4x32, 2: 2x64)
};

constexpr long GRAPH_STEPS = 25;

// resolve recorded event pairs into the per-kernel accumulators (synchronises)
static int resolve_events(cgks_ctx* c) {
  if (!c->events || c->ev_used == 0) return CGKS_OK;
  if (hipEventSynchronize((*c->events)[2 * c->ev_used - 1]) != hipSuccess) return CGKS_EDEVICE;
  for (size_t k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, (*c->events)[2 * k], (*c->events)[2 * k + 1]) != hipSuccess) return CGKS_EDEVICE;
    const int kind = (*c->ev_kind)[k];
    c->ms[kind] += ms;
    c->calls[kind] += 1;
  }
  c->ev_used = 0;
  return CGKS_OK;
}

// launch helper: records an event pair around the launch while profiling
template <class F>
static void timed(cgks_ctx* c, int kind, F&& launch) {
  if (!(c->profiling & (1 << kind))) { launch(); return; }
  if (c->ev_used == kEventPairs) resolve_events(c);
  (void)hipEventRecord((*c->events)[2 * c->ev_used], c->stream);
  launch();
  (void)hipEventRecord((*c->events)[2 * c->ev_used + 1], c->stream);
  (*c->ev_kind)[c->ev_used] = kind;
  c->ev_used += 1;
}

// grid of the update kernels (and of the scan): 64x4 cells per block in 2D, 256 in 1D
static dim3 update_grid(const Geom& G) {
  if (G.dim == 2) return dim3((unsigned)((G.nx + 63) / 64), (unsigned)((G.ny + 3) / 4));
  return dim3((unsigned)((G.nx + 255) / 256), 1);
}

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return CGKS_EDEVICE; \
  } while (0)

static int validate(const cgks_config* c) {
  if (!c) return CGKS_EINVAL;
  if (c->dim != 1 && c->dim != 2) return CGKS_EINVAL;
  if (c->nx < 1 || (c->dim == 2 && c->ny < 1)) return CGKS_EINVAL;
  if ((long long)c->nx * (c->dim == 2 ? c->ny : 1) > (1ll << 31) / 16) return CGKS_EINVAL;
  if (!(c->gamma > 1.0) || !(c->x1 > c->x0) || (c->dim == 2 && !(c->y1 > c->y0))) return CGKS_EINVAL;
  if (!(c->cfl > 0.0) && !(c->fixed_dt > 0.0)) return CGKS_EINVAL;
  if (!(c->weno_eps > 0.0) || !(c->tau_eps > 0.0) || c->tau_C < 0.0) return CGKS_EINVAL;
  if (!(c->mu >= 0.0) || !std::isfinite(c->mu)) return CGKS_EINVAL;
  if (c->storage != CGKS_FP64 && !(c->storage == CGKS_FP32_STORAGE && c->dim == 2)) return CGKS_EINVAL;
  const int gp = c->gauss_points ? c->gauss_points : 2;
  if (gp != 2 && !(gp == 4 && c->dim == 2)) return CGKS_EINVAL;
  if (c->recon_vars != CGKS_CONSERVATIVE && c->recon_vars != CGKS_CHARACTERISTIC) return CGKS_EINVAL;
  if (c->side_slopes != 0 && (c->side_slopes != 1 || c->recon_vars != CGKS_CONSERVATIVE)) return CGKS_EINVAL;
  if (c->tang_weno != 0 && (c->tang_weno != 1 || c->dim != 2 || c->recon_vars != CGKS_CONSERVATIVE ||
                            c->side_slopes != 0))
    return CGKS_EINVAL;
  for (int s = 0; s < 2 * c->dim; ++s) {
    if (c->bc[s] < 0 || c->bc[s] > 4) return CGKS_EINVAL;
    const int n = s < 2 ? c->nx : c->ny;
    if ((c->bc[s] == CGKS_WALL || c->bc[s] == CGKS_NOSLIP) && n < (gp == 4 ? 3 : 2)) return CGKS_EINVAL;
    if (c->bc[s] == CGKS_INFLOW) {
      const double* q = c->inflow_prim[s];
      if (!(q[0] > 0.0) || !(q[3] > 0.0)) return CGKS_EINVAL;
    }
  }
  if ((c->bc[0] == CGKS_PERIODIC) != (c->bc[1] == CGKS_PERIODIC)) return CGKS_EINVAL;
  if (c->dim == 2 && (c->bc[2] == CGKS_PERIODIC) != (c->bc[3] == CGKS_PERIODIC)) return CGKS_EINVAL;
  return CGKS_OK;
}

// Geometry, gas constants and conservative inflow states of a configuration.
static void make_geom(const cgks_config& cfg, Geom& G) {
  std::memset(&G, 0, sizeof G);
  G.dim = cfg.dim;
  G.nx = cfg.nx;
  G.ny = cfg.dim == 2 ? cfg.ny : 1;
  G.dx = (cfg.x1 - cfg.x0) / cfg.nx;
  G.dy = cfg.dim == 2 ? (cfg.y1 - cfg.y0) / cfg.ny : 1.0;
  G.inv_dx = 1.0 / G.dx;
  G.inv_dy = 1.0 / G.dy;
  G.eps = cfg.weno_eps;
  G.charv = cfg.recon_vars == CGKS_CHARACTERISTIC;
  G.sides = cfg.side_slopes == 1;
  G.tw = cfg.tang_weno == 1;
  G.gas = make_gas(cfg.gamma, cfg.dim, cfg.tau_eps, cfg.tau_C, cfg.mu);
  for (int s = 0; s < 4; ++s) {
    G.bc[s] = s < 2 * cfg.dim ? cfg.bc[s] : CGKS_PERIODIC;
    const double* q = cfg.inflow_prim[s];
    const double g1 = cfg.gamma - 1.0;
    if (cfg.dim == 2) {
      G.inflow[s][0] = q[0]; G.inflow[s][1] = q[0] * q[1]; G.inflow[s][2] = q[0] * q[2];
      G.inflow[s][3] = q[3] / g1 + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2]);
    } else {
      G.inflow[s][0] = q[0]; G.inflow[s][1] = q[0] * q[1];
      G.inflow[s][2] = q[3] / g1 + 0.5 * q[0] * q[1] * q[1]; G.inflow[s][3] = 0.0;
    }
  }
}

static void free_bufs(cgks_ctx* c) {
  (void)hipFree(c->B.S[0]); (void)hipFree(c->B.S[1]); (void)hipFree(c->B.Ws); (void)hipFree(c->B.P);
  (void)hipFree(c->B.FX); (void)hipFree(c->B.FY); (void)hipFree(c->B.sc); (void)hipFree(c->B.lam_part);
  if (c->host_sc) (void)hipHostFree(c->host_sc);
}

// Face tile shapes of a 2D grid: the tuned entry nearest in cell count (log scale).
static void tuned_tiles(int nx, int ny, int* tile) {
  const double lc = std::log((double)nx * (double)ny);
  double best = INFINITY;
  tile[0] = tile[1] = 0;
  for (const TuneEntry& e : kTuneTable) {
    const double d = std::fabs(std::log((double)e.nx * (double)e.ny) - lc);
    if (d < best) { best = d; tile[0] = e.x; tile[1] = e.y; }
  }
}

extern "C" int cgks_create(const cgks_config* cfg, void* hip_stream, cgks_ctx** out) {
  if (!out) return CGKS_EINVAL;
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  cgks_ctx* c = new (std::nothrow) cgks_ctx();
  if (!c) return CGKS_ENOMEM;
  std::memset(c, 0, sizeof *c);
  c->cfg = *cfg;
  if (cfg->dim == 1) c->cfg.ny = 1;
  if (c->cfg.gauss_points == 0) c->cfg.gauss_points = 2;
  c->stream = (hipStream_t)hip_stream;
  Geom& G = c->G;
  make_geom(c->cfg, G);
  c->N = (size_t)G.nx * G.ny;
  c->nf = cfg->dim == 2 ? 12 : 6;
  const size_t fbytes = c->nf * c->N * sizeof(double);
  size_t fx = 0, fy = 0;
  if (cfg->dim == 2) {
    fx = (size_t)16 * G.ny * (G.nx + 1) * sizeof(double);
    fy = (size_t)16 * (G.ny + 1) * G.nx * sizeof(double);
  } else {
    fx = (size_t)12 * (G.nx + 1) * sizeof(double);
    fy = sizeof(double);
  }
  bool ok = hipMalloc(&c->B.S[0], fbytes) == hipSuccess && hipMalloc(&c->B.S[1], fbytes) == hipSuccess &&
            hipMalloc(&c->B.Ws, fbytes) == hipSuccess && hipMalloc(&c->B.P, fbytes) == hipSuccess &&
            hipMalloc(&c->B.FX, fx) == hipSuccess && hipMalloc(&c->B.FY, fy) == hipSuccess &&
            hipMalloc(&c->B.sc, sizeof(Scalars)) == hipSuccess &&
            hipMalloc(&c->B.lam_part, sizeof(double) * (size_t)update_grid(G).x * update_grid(G).y) == hipSuccess &&
            hipHostMalloc(&c->host_sc, sizeof(Scalars), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_bufs(c);
    delete c;
    return CGKS_ENOMEM;
  }
  std::memset(c->host_sc, 0, sizeof(Scalars));
  if (cfg->dim == 2) tuned_tiles(G.nx, G.ny, c->tile);
  *out = c;
  return CGKS_OK;
}

extern "C" void cgks_destroy(cgks_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->events) {
    for (hipEvent_t e : *c->events) (void)hipEventDestroy(e);
    delete c->events;
    delete c->ev_kind;
  }
  free_bufs(c);
  delete c;
}

extern "C" int cgks_set_profiling(cgks_ctx* c, int on) {
  if (!c) return CGKS_EINVAL;
  if (on && !c->events) {
    auto* ev = new (std::nothrow) std::vector<hipEvent_t>(2 * kEventPairs, nullptr);
    auto* kind = new (std::nothrow) std::vector<int>(kEventPairs);
    bool ok = ev && kind;
    for (size_t k = 0; ok && k < ev->size(); ++k) ok = hipEventCreate(&(*ev)[k]) == hipSuccess;
    if (!ok) {                       // leave the context without profiling state
      if (ev)
        for (hipEvent_t e : *ev)
          if (e) (void)hipEventDestroy(e);
      delete ev;
      delete kind;
      return CGKS_ENOMEM;
    }
    c->events = ev;
    c->ev_kind = kind;
  }
  if (on) {
    HIPCHK(hipStreamSynchronize(c->stream));
    c->ev_used = 0;
    for (int k = 0; k < kKinds; ++k) { c->ms[k] = 0.0; c->calls[k] = 0; }
  } else {
    int rc = resolve_events(c);
    if (rc) return rc;
  }
  c->profiling = on;
  return CGKS_OK;
}

extern "C" int cgks_set_tiles(cgks_ctx* c, int x_shape, int y_shape) {
  if (!c || x_shape < 0 || x_shape >= kTileShapes || y_shape < 0 || y_shape >= kTileShapes) return CGKS_EINVAL;
  if (c->tile[0] != x_shape || c->tile[1] != y_shape) {
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->exec) (void)hipGraphExecDestroy(c->exec);   // the graph holds the old launches
    c->exec = nullptr;
  }
  c->tile[0] = x_shape;
  c->tile[1] = y_shape;
  return CGKS_OK;
}

extern "C" int cgks_kernel_times(cgks_ctx* c, double* ms, long* calls, int n) {
  if (!c || !ms || !calls) return CGKS_EINVAL;
  int rc = resolve_events(c);
  if (rc) return rc;
  const int kinds = c->G.dim == 2 ? 6 : 4;
  for (int k = 0; k < n && k < kinds; ++k) { ms[k] = c->ms[k]; calls[k] = c->calls[k]; }
  return kinds;
}

static int pull_scalars(cgks_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->host_sc, c->B.sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CGKS_OK;
}

static int push_params(cgks_ctx* c, double t_end, double dt_override) {
  // the pinned mirror holds the last pulled scalars; only the parameter block is sent
  c->host_sc->prm.t_end = t_end;
  c->host_sc->prm.dt_override = dt_override;
  c->host_sc->prm.max_step = LLONG_MAX;
  HIPCHK(hipMemcpyAsync(c->B.sc, c->host_sc, sizeof(Params), hipMemcpyHostToDevice, c->stream));
  return CGKS_OK;
}

extern "C" int cgks_set_state(cgks_ctx* c, const double* fields, int on_device, double t0) {
  if (!c || !fields) return CGKS_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  Scalars& h = *c->host_sc;
  std::memset(&h, 0, sizeof h);
  h.prm.t_end = INFINITY;
  h.t = t0;
  h.cfl = c->cfg.cfl;
  h.fixed_dt = c->cfg.fixed_dt;
  h.bad_cell = ULLONG_MAX;
  if (c->cfg.storage == CGKS_FP32_STORAGE) {
    // host fields are staged in W* (free between steps), then converted
    const double* src = fields;
    if (!on_device) {
      HIPCHK(hipMemcpyAsync(c->B.Ws, fields, c->nf * c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
      src = c->B.Ws;
    }
    k_to_storage32<<<(unsigned)((c->N + 255) / 256), 256, 0, c->stream>>>(src, c->B.S[0], c->N);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpyAsync(c->B.S[0], fields, c->nf * c->N * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipMemcpyAsync(c->B.sc, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
  if (c->cfg.dim == 2) k_scan<4><<<update_grid(c->G), 256, 0, c->stream>>>(c->G, c->B);
  else k_scan<3><<<update_grid(c->G), 256, 0, c->stream>>>(c->G, c->B);
  HIPCHK(hipGetLastError());
  int rc = pull_scalars(c);
  if (rc) return rc;
  c->has_state = 1;
  if (h.status != 0) {
    c->has_state = 0;
    return CGKS_ENONPHYS;
  }
  return CGKS_OK;
}

// The launches of one step on stream s for geometry G and buffers B.  run(kind,
// launch) issues each kernel launch (the context brackets them with events
// while profiling).  gp: Gauss points; tiles: face tile shape per direction.
template <class Run>
static void launch_step_on(const Geom& G, const Bufs& B, int gp, int storage, const int* tiles, hipStream_t s,
                           Run&& run) {
  const dim3 gu = update_grid(G);
  k_begin<<<1, 256, 0, s>>>(B.sc, B.lam_part, (int)(gu.x * gu.y));
  if (G.dim == 2) {
    // one direction's face kernel of one stage with the given tile shape
    auto faces = [&](auto dir, auto stage, auto gt, int kind) {
      constexpr int DIR = decltype(dir)::value, STAGE = decltype(stage)::value;
      using GT = decltype(gt);
      auto go = [&](auto tl, auto ch, auto ss, auto tw) {
        using TL = decltype(tl);
        constexpr bool CH = decltype(ch)::value, SS = decltype(ss)::value, TW = decltype(tw)::value;
        const dim3 g = DIR == 0 ? dim3((G.nx + 1 + TL::F - 1) / TL::F, (G.ny + TL::T - 1) / TL::T)
                                : dim3((G.nx + TL::T - 1) / TL::T, (G.ny + 1 + TL::F - 1) / TL::F);
        run(kind, [&] { k_faces2<DIR, STAGE, GT, TL, CH, SS, TW><<<g, FACE_THREADS, 0, s>>>(G, B); });
      };
      using CV = std::false_type;
      using CC = std::true_type;
      using NS = std::false_type;
      if (gp == 4) {
        using SV = std::true_type;
        if (G.charv) { if constexpr (DIR == 0) go(Tile4x16G4(), CC(), NS(), NS()); else go(Tile2x32G4(), CC(), NS(), NS()); }
        else if (G.sides) { if constexpr (DIR == 0) go(Tile4x16G4(), CV(), SV(), NS()); else go(Tile2x32G4(), CV(), SV(), NS()); }
        else if (G.tw) { if constexpr (DIR == 0) go(Tile4x16G4(), CV(), NS(), SV()); else go(Tile2x32G4(), CV(), NS(), SV()); }
        else { if constexpr (DIR == 0) go(Tile4x16G4(), CV(), NS(), NS()); else go(Tile2x32G4(), CV(), NS(), NS()); }
        return;
      }
      if (G.charv) {   // characteristic variables: one tile shape per direction
        if constexpr (DIR == 0) go(Tile4x32(), CC(), NS(), NS()); else go(Tile2x64(), CC(), NS(), NS());
        return;
      }
      if (G.tw) {      // the tangential-WENO variant: the 5-segment halo
        if constexpr (DIR == 0) go(Tile4x32W(), CV(), NS(), std::true_type()); else go(Tile2x64W(), CV(), NS(), std::true_type());
        return;
      }
      if (G.sides) {   // the side-slope variant: one tile shape per direction
        if constexpr (DIR == 0) go(Tile4x32(), CV(), std::true_type(), NS()); else go(Tile2x64(), CV(), std::true_type(), NS());
        return;
      }
      switch (tiles[DIR]) {
        case 1: go(Tile4x32(), CV(), NS(), NS()); break;
        case 2: go(Tile2x64(), CV(), NS(), NS()); break;
        default: go(Tile8x16(), CV(), NS(), NS()); break;
      }
    };
    using D0 = std::integral_constant<int, 0>;
    using D1 = std::integral_constant<int, 1>;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    auto stage_kernels = [&](auto gt) {
      using GT = decltype(gt);
      faces(D0(), S1(), gt, 0);
      faces(D1(), S1(), gt, 1);
      run(2, [&] { k_update2<1, GT><<<gu, 256, 0, s>>>(G, B); });
      faces(D0(), S2(), gt, 3);
      faces(D1(), S2(), gt, 4);
      run(5, [&] { k_update2<2, GT><<<gu, 256, 0, s>>>(G, B); });
    };
    if (storage == CGKS_FP32_STORAGE) stage_kernels(0.0f);
    else stage_kernels(0.0);
  } else {
    const unsigned nf = (unsigned)((G.nx + 1 + 255) / 256);
    run(0, [&] { k_faces1<1><<<nf, 256, 0, s>>>(G, B); });
    run(1, [&] { k_update1<1><<<gu, 256, 0, s>>>(G, B); });
    run(2, [&] { k_faces1<2><<<nf, 256, 0, s>>>(G, B); });
    run(3, [&] { k_update1<2><<<gu, 256, 0, s>>>(G, B); });
  }
  k_end<<<1, 64, 0, s>>>(B.sc);
}

static void launch_step(cgks_ctx* c) {
  launch_step_on(c->G, c->B, c->cfg.gauss_points, c->cfg.storage, c->tile, c->stream,
                 [c](int kind, auto&& launch) { timed(c, kind, launch); });
}

// 1D grids of at most this many cells run whole steps in one single-block
// launch (k_steps1) unless the kernels are being timed one by one: with one
// face per thread (nx + 1 <= 256) a step takes 17 instead of 25 us at 100
// cells; with two or more faces per thread the serial point evaluations cost
// more than the separate launches (34 against 29 us at 400 cells).
#ifndef CGKS_FUSED1D_MAX
#define CGKS_FUSED1D_MAX 255
#endif
constexpr long kStepsPerLaunch1D = 4096;   // bound on one fused launch's duration

static bool fused_1d(const cgks_ctx* c) {
  return c->G.dim == 1 && c->G.nx <= CGKS_FUSED1D_MAX && !c->profiling;
}

// n steps queued on the context's stream
static void launch_steps(cgks_ctx* c, long n) {
  if (fused_1d(c)) {
    const int nparts = (int)update_grid(c->G).x;
    while (n > 0) {
      const long k = n < kStepsPerLaunch1D ? n : kStepsPerLaunch1D;
      k_steps1<<<1, 256, 0, c->stream>>>(c->G, c->B, (int)k, nparts);
      n -= k;
    }
    return;
  }
  for (long k = 0; k < n; ++k) launch_step(c);
}

extern "C" int cgks_step_dt(cgks_ctx* c, double dt, double* dt_used) {
  if (!c) return CGKS_EINVAL;
  if (!c->has_state) return CGKS_ESTATE;
  int rc = push_params(c, INFINITY, dt > 0.0 ? dt : 0.0);
  if (rc) return rc;
  const long long before = c->host_sc->step;
  launch_steps(c, 1);
  HIPCHK(hipGetLastError());
  rc = pull_scalars(c);
  if (rc) return rc;
  if (c->host_sc->status) return c->host_sc->status;
  if (c->host_sc->step != before + 1) return CGKS_EDEVICE;
  if (dt_used) *dt_used = c->host_sc->last_dt;
  return CGKS_OK;
}

extern "C" int cgks_step(cgks_ctx* c, double* dt_used) { return cgks_step_dt(c, 0.0, dt_used); }

// Capture GRAPH_STEPS steps of the context into a graph.  Only on a stream
// that may be captured (not the legacy null stream) and with profiling off;
// returns false (and leaves eager launching) otherwise.
static bool ensure_graph(cgks_ctx* c) {
  if (c->exec) return true;
  if (!c->stream || c->profiling) return false;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  for (long k = 0; k < GRAPH_STEPS; ++k) launch_step(c);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  bool ok = e1 == hipSuccess && e2 == hipSuccess && g &&
            hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {
    c->exec = nullptr;
    (void)hipGetLastError();
  }
  return ok;
}

extern "C" int cgks_run_steps(cgks_ctx* c, long n) {
  if (!c || n < 0) return CGKS_EINVAL;
  if (!c->has_state) return CGKS_ESTATE;
  int rc = push_params(c, INFINITY, 0.0);
  if (rc) return rc;
  long k = 0;
  if (n >= GRAPH_STEPS && !c->profiling && !fused_1d(c) && ensure_graph(c))
    for (; k + GRAPH_STEPS <= n; k += GRAPH_STEPS) HIPCHK(hipGraphLaunch(c->exec, c->stream));
  launch_steps(c, n - k);
  HIPCHK(hipGetLastError());
  rc = pull_scalars(c);
  if (rc) return rc;
  return c->host_sc->status;
}

extern "C" int cgks_advance_to(cgks_ctx* c, double t_end, long max_steps, long* steps_taken) {
  if (!c) return CGKS_EINVAL;
  if (!c->has_state) return CGKS_ESTATE;
  int rc = push_params(c, t_end, 0.0);
  if (rc) return rc;
  const long long start = c->host_sc->step;
  long launched = 0;
  int chunk = 8;
  while (c->host_sc->t < t_end && c->host_sc->status == 0) {
    long n = chunk;
    if (max_steps > 0) n = n < max_steps - launched ? n : max_steps - launched;
    if (n <= 0) break;
    launch_steps(c, n);
    launched += n;
    HIPCHK(hipGetLastError());
    rc = pull_scalars(c);
    if (rc) return rc;
    if (chunk < 64) chunk *= 2;
  }
  if (steps_taken) *steps_taken = (long)(c->host_sc->step - start);
  return c->host_sc->status;
}

extern "C" int cgks_get_state(cgks_ctx* c, double* out, int on_device, double* t, long* step) {
  if (!c) return CGKS_EINVAL;
  if (!c->has_state) return CGKS_ESTATE;
  int rc = pull_scalars(c);
  if (rc) return rc;
  if (out) {
    const double* S = c->B.S[c->host_sc->cur];
    if (c->cfg.storage == CGKS_FP32_STORAGE) {
      // converted to FP64 straight into a device output, else via W* (free between steps)
      double* dst = on_device ? out : c->B.Ws;
      k_from_storage32<<<(unsigned)((c->N + 255) / 256), 256, 0, c->stream>>>(S, dst, c->N);
      HIPCHK(hipGetLastError());
      if (!on_device)
        HIPCHK(hipMemcpyAsync(out, c->B.Ws, c->nf * c->N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    } else {
      HIPCHK(hipMemcpyAsync(out, S, c->nf * c->N * sizeof(double),
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  if (t) *t = c->host_sc->t;
  if (step) *step = (long)c->host_sc->step;
  return CGKS_OK;
}

extern "C" int cgks_last_bad_cell(const cgks_ctx* c, long* cell) {
  if (!c || !cell) return CGKS_EINVAL;
  *cell = c->host_sc->bad_cell == ULLONG_MAX ? -1 : (long)c->host_sc->bad_cell;
  return CGKS_OK;
}

extern "C" int cgks_counters(cgks_ctx* c, cgks_counters_t* out) {
  if (!c || !out) return CGKS_EINVAL;
  int rc = pull_scalars(c);
  if (rc) return rc;
  out->steps = (long)c->host_sc->step;
  out->guard_w0 = (long)c->host_sc->guard_w0;
  out->guard_weno = (long)c->host_sc->guard_weno;
  out->last_dt = c->host_sc->last_dt;
  out->t = c->host_sc->t;
  return CGKS_OK;
}

extern "C" const char* cgks_strerror(int code) {
  switch (code) {
    case CGKS_OK: return "ok";
    case CGKS_EINVAL: return "invalid argument or configuration";
    case CGKS_ENOMEM: return "out of memory";
    case CGKS_EDEVICE: return "HIP runtime error";
    case CGKS_ENONPHYS: return "non-physical state (rho <= 0, p <= 0 or NaN); step not committed";
    case CGKS_EBUSY: return "no free slot or memory budget exhausted";
    case CGKS_ESTATE: return "no state loaded";
    default: return "unknown error";
  }
}

// ============================================================== step without allocation

// Scratch of cgks_step_noalloc: the intermediate state, the partial final
// update, the face results, the CFL partials and the step scalars of one step
// of at most CGKS_NOALLOC_MAX_CELLS cells (2D: 12 + 12 fields of 8 bytes,
// 16 x 2 face planes, a partial per 256 cells; 1D needs less).  One copy per
// GPU, for the life of the process.  Host code never passes the symbol itself:
// it takes the device address from hipGetSymbolAddress (per device).
constexpr size_t kScratchBytes = (size_t)600 * CGKS_NOALLOC_MAX_CELLS + ((size_t)1 << 16);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// the device address of this device's scratch (looked up once per device)
static int scratch_on_device(unsigned char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CGKS_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return CGKS_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return CGKS_OK;
}

// every field of the step scalars (the scratch keeps the last call's contents)
__global__ void k_noalloc_init(Scalars* sc, double cfl, double fixed_dt, double dt_override) {
  if (threadIdx.x != 0) return;
  sc->prm.t_end = INFINITY;
  sc->prm.dt_override = dt_override;
  sc->prm.max_step = LLONG_MAX;
  sc->t = 0.0;
  sc->dt = 0.0;
  sc->cfl = cfl;
  sc->fixed_dt = fixed_dt;
  sc->last_dt = 0.0;
  sc->bad_cell = ULLONG_MAX;
  sc->guard_w0 = 0;
  sc->guard_weno = 0;
  sc->step = 0;
  sc->status = 0;
  sc->active = 0;
  sc->last = 0;
  sc->cur = 0;
}

extern "C" int cgks_step_noalloc(const cgks_config* cfg, const double* in, double* out, double dt, void* hip_stream,
                                 double* dt_used) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!in || !out || in == out || cfg->storage != CGKS_FP64) return CGKS_EINVAL;
  cgks_config cf = *cfg;
  if (cf.dim == 1) cf.ny = 1;
  if (cf.gauss_points == 0) cf.gauss_points = 2;
  Geom G;
  make_geom(cf, G);
  const size_t N = (size_t)G.nx * G.ny;
  if (N > (size_t)CGKS_NOALLOC_MAX_CELLS) return CGKS_EINVAL;
  const size_t nf = cf.dim == 2 ? 12 : 6;
  const dim3 gu = update_grid(G);
  // carve the scratch: each piece 256-byte aligned
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
  const size_t o_ws = take(nf * N * sizeof(double));
  const size_t o_p = take(nf * N * sizeof(double));
  const size_t o_fx = take(cf.dim == 2 ? (size_t)16 * G.ny * (G.nx + 1) * sizeof(double)
                                       : (size_t)12 * (G.nx + 1) * sizeof(double));
  const size_t o_fy = take(cf.dim == 2 ? (size_t)16 * (G.ny + 1) * G.nx * sizeof(double) : sizeof(double));
  const size_t o_lam = take((size_t)gu.x * gu.y * sizeof(double));
  const size_t o_sc = take(sizeof(Scalars));
  if (off > kScratchBytes) return CGKS_EINVAL;
  unsigned char* base = nullptr;
  rc = scratch_on_device(&base);
  if (rc) return rc;
  Bufs B;
  B.S[0] = const_cast<double*>(in);   // only read: the step writes S[cur ^ 1] = out
  B.S[1] = out;
  B.Ws = reinterpret_cast<double*>(base + o_ws);
  B.P = reinterpret_cast<double*>(base + o_p);
  B.FX = reinterpret_cast<double*>(base + o_fx);
  B.FY = reinterpret_cast<double*>(base + o_fy);
  B.lam_part = reinterpret_cast<double*>(base + o_lam);
  B.sc = reinterpret_cast<Scalars*>(base + o_sc);
  hipStream_t s = (hipStream_t)hip_stream;
  int tiles[2] = {0, 0};
  if (cf.dim == 2) tuned_tiles(G.nx, G.ny, tiles);
  k_noalloc_init<<<1, 64, 0, s>>>(B.sc, cf.cfl, cf.fixed_dt, dt > 0.0 ? dt : 0.0);
  if (cf.dim == 2) k_scan<4><<<gu, 256, 0, s>>>(G, B);
  else k_scan<3><<<gu, 256, 0, s>>>(G, B);
  launch_step_on(G, B, cf.gauss_points, cf.storage, tiles, s, [](int, auto&& launch) { launch(); });
  HIPCHK(hipGetLastError());
  if (!dt_used) return CGKS_OK;
  Scalars h;
  HIPCHK(hipMemcpyAsync(&h, B.sc, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h.status) return h.status;
  if (h.step != 1) return CGKS_EDEVICE;
  *dt_used = h.last_dt;
  return CGKS_OK;
}

// ============================================================== batch (serving)

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator with coalescing over one device allocation.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> length, no two adjacent

  bool alloc(size_t n, size_t& off) {
    n = round_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      off = it->first;
      const size_t rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct SlotInfo {
  int used = 0;
  size_t off = 0, bytes = 0;
  size_t N = 0;
  int kind = 0;                    // BK_*
  int nb[2] = {0, 0}, nbu = 0;     // blocks of the x-face, y-face and update grids
};

// Face tile shape of a kind per direction: two points with FP64 storage and
// conservative variables use the batch's tuned shapes (0 = 8x16, 1 = 4x32,
// 2 = 2x64), the other two-point kinds 4x32 and 2x64, four points the
// four-point tiles.
struct TileDims { int F, T; };
static TileDims kind_tile(int kind, int dir, const int* tile) {
  if (kind_g4(kind))
    return dir == 0 ? TileDims{Tile4x16G4::F, Tile4x16G4::T} : TileDims{Tile2x32G4::F, Tile2x32G4::T};
  const int shape = kind == BK_G2 ? tile[dir] : (dir == 0 ? 1 : 2);
  switch (shape) {
    case 1: return TileDims{Tile4x32::F, Tile4x32::T};
    case 2: return TileDims{Tile2x64::F, Tile2x64::T};
    default: return TileDims{Tile8x16::F, Tile8x16::T};
  }
}

}  // namespace

struct cgks_batch {
  hipStream_t stream = nullptr;
  int own_stream = 0;
  int max_slots = 0;
  Arena arena;
  SlotDev* d_slots = nullptr;
  std::vector<SlotDev> h_slots;
  Scalars* d_sc = nullptr;
  Scalars* h_sc = nullptr;          // pinned mirror, refreshed after admit and run
  BatchTable* d_tab = nullptr;
  BatchTable* h_tab = nullptr;      // pinned
  std::vector<SlotInfo> info;
  std::vector<int> table;           // running slots in the current table
  int dirty = 1;                    // a slot was admitted or released since the table was built
  int cap_n = 0;                    // grid bucket of the begin/end launches
  int tile[2] = {1, 2};             // face tile shapes of the two-point FP64 slots
  hipGraphExec_t exec = nullptr;
  int graph_steps = 0;
  int cap_f[BK_KINDS][2] = {}, cap_u2[2] = {};   // face and update grid buckets per kind / storage
};

static int slot_state(const cgks_batch* b, int k) {
  if (!b->info[k].used) return CGKS_SLOT_FREE;
  const Scalars& h = b->h_sc[k];
  if (h.status != 0) return CGKS_SLOT_FAILED;
  if (h.step >= h.prm.max_step || !(h.prm.t_end - h.t > 0.0)) return CGKS_SLOT_DONE;
  return CGKS_SLOT_RUNNING;
}

static void drop_graph(cgks_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->graph_steps = 0;
}

extern "C" void cgks_batch_destroy(cgks_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  (void)hipFree(b->arena.base);
  (void)hipFree(b->d_slots);
  (void)hipFree(b->d_sc);
  (void)hipFree(b->d_tab);
  if (b->h_sc) (void)hipHostFree(b->h_sc);
  if (b->h_tab) (void)hipHostFree(b->h_tab);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

extern "C" int cgks_batch_create(size_t hbm_budget_bytes, int max_slots, void* hip_stream, cgks_batch** out) {
  if (!out) return CGKS_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > kMaxSlots || hbm_budget_bytes < kAlign) return CGKS_EINVAL;
  cgks_batch* b = new (std::nothrow) cgks_batch();
  if (!b) return CGKS_ENOMEM;
  b->max_slots = max_slots;
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return CGKS_EDEVICE;
    }
    b->own_stream = 1;
  }
  b->arena.size = hbm_budget_bytes / kAlign * kAlign;
  bool ok = hipMalloc(&b->arena.base, b->arena.size) == hipSuccess &&
            hipMalloc(&b->d_slots, sizeof(SlotDev) * max_slots) == hipSuccess &&
            hipMalloc(&b->d_sc, sizeof(Scalars) * max_slots) == hipSuccess &&
            hipMalloc(&b->d_tab, sizeof(BatchTable)) == hipSuccess &&
            hipHostMalloc(&b->h_sc, sizeof(Scalars) * max_slots, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_tab, sizeof(BatchTable), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    cgks_batch_destroy(b);
    return CGKS_ENOMEM;
  }
  b->arena.free_[0] = b->arena.size;
  b->tile[0] = kBatchTune.x;
  b->tile[1] = kBatchTune.y;
  b->h_slots.assign(max_slots, SlotDev());
  b->info.assign(max_slots, SlotInfo());
  std::memset(b->h_sc, 0, sizeof(Scalars) * max_slots);
  std::memset(b->h_tab, 0, sizeof(BatchTable));
  *out = b;
  return CGKS_OK;
}

extern "C" int cgks_batch_admit(cgks_batch* b, const cgks_config* cfg, const double* fields, int on_device,
                                double t_end, long max_steps, int* slot) {
  if (!b || !fields || !slot) return CGKS_EINVAL;
  int rc = validate(cfg);
  if (rc) return rc;
  if (cfg->dim != 2) return CGKS_EINVAL;
  if (!(t_end > 0.0) && max_steps <= 0) return CGKS_EINVAL;   // a request needs an end
  int k = 0;
  while (k < b->max_slots && b->info[k].used) ++k;
  if (k == b->max_slots) return CGKS_EBUSY;

  SlotDev& sd = b->h_slots[k];
  SlotInfo& in = b->info[k];
  const int gp = cfg->gauss_points ? cfg->gauss_points : 2;
  const int f32 = cfg->storage == CGKS_FP32_STORAGE;
  const int kind = (gp == 4 ? BK_G4 : BK_G2) | (f32 ? BK_G2_F32 : 0) |
                   (cfg->recon_vars == CGKS_CHARACTERISTIC ? BK_CHAR : 0) | (cfg->side_slopes ? BK_SIDE : 0) |
                   (cfg->tang_weno ? BK_TW : 0);
  make_geom(*cfg, sd.G);
  const Geom& G = sd.G;
  const size_t N = (size_t)G.nx * G.ny;
  const dim3 gu = update_grid(G);
  const size_t fbytes = round_up(12 * N * sizeof(double));
  const size_t fx = round_up((size_t)16 * G.ny * (G.nx + 1) * sizeof(double));
  const size_t fy = round_up((size_t)16 * (G.ny + 1) * G.nx * sizeof(double));
  const size_t lp = round_up(sizeof(double) * (size_t)gu.x * gu.y);
  const size_t bytes = 4 * fbytes + fx + fy + lp;
  size_t off = 0;
  if (!b->arena.alloc(bytes, off)) return CGKS_EBUSY;
  char* p = b->arena.base + off;
  sd.B.S[0] = (double*)p; p += fbytes;
  sd.B.S[1] = (double*)p; p += fbytes;
  sd.B.Ws = (double*)p; p += fbytes;
  sd.B.P = (double*)p; p += fbytes;
  sd.B.FX = (double*)p; p += fx;
  sd.B.FY = (double*)p; p += fy;
  sd.B.lam_part = (double*)p;
  sd.B.sc = b->d_sc + k;
  const TileDims tx = kind_tile(kind, 0, b->tile), ty = kind_tile(kind, 1, b->tile);
  sd.gw[0] = (G.nx + 1 + tx.F - 1) / tx.F;
  sd.gw[1] = (G.nx + ty.T - 1) / ty.T;
  sd.guw = (int)gu.x;
  sd.nparts = (int)(gu.x * gu.y);
  in.used = 1;
  in.off = off;
  in.bytes = bytes;
  in.N = N;
  in.kind = kind;
  in.nb[0] = sd.gw[0] * ((G.ny + tx.T - 1) / tx.T);
  in.nb[1] = sd.gw[1] * ((G.ny + 1 + ty.F - 1) / ty.F);
  in.nbu = sd.nparts;

  Scalars& h = b->h_sc[k];
  std::memset(&h, 0, sizeof h);
  h.prm.t_end = t_end > 0.0 ? t_end : INFINITY;
  h.prm.dt_override = 0.0;
  h.prm.max_step = max_steps > 0 ? (long long)max_steps : LLONG_MAX;
  h.cfl = cfg->cfl;
  h.fixed_dt = cfg->fixed_dt;
  h.bad_cell = ULLONG_MAX;
  bool ok;
  if (f32) {   // staged in W* (free between steps), then converted to the storage layout
    ok = hipMemcpyAsync(sd.B.Ws, fields, 12 * N * sizeof(double),
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, b->stream) == hipSuccess;
    if (ok) {
      k_to_storage32<<<(unsigned)((N + 255) / 256), 256, 0, b->stream>>>(sd.B.Ws, sd.B.S[0], N);
      ok = hipGetLastError() == hipSuccess;
    }
  } else {
    ok = hipMemcpyAsync(sd.B.S[0], fields, 12 * N * sizeof(double),
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, b->stream) == hipSuccess;
  }
  ok = ok && hipMemcpyAsync(b->d_sc + k, &h, sizeof h, hipMemcpyHostToDevice, b->stream) == hipSuccess &&
       hipMemcpyAsync(b->d_slots + k, &sd, sizeof sd, hipMemcpyHostToDevice, b->stream) == hipSuccess;
  if (ok) {
    k_scan<4><<<gu, 256, 0, b->stream>>>(sd.G, sd.B);
    ok = hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(&h, b->d_sc + k, sizeof h, hipMemcpyDeviceToHost, b->stream) == hipSuccess &&
         hipStreamSynchronize(b->stream) == hipSuccess;
  }
  if (!ok || h.status != 0) {
    b->arena.release(off, bytes);
    in = SlotInfo();
    return ok ? CGKS_ENONPHYS : CGKS_EDEVICE;
  }
  b->dirty = 1;
  *slot = k;
  return CGKS_OK;
}

// Work lists of the running slots (the graph reads them from device memory
// and needs no new capture while each list stays in its grid bucket).
static int refresh_table(cgks_batch* b) {
  std::vector<int> run;
  for (int k = 0; k < b->max_slots; ++k)
    if (slot_state(b, k) == CGKS_SLOT_RUNNING) run.push_back(k);
  // an admit or release may reuse a slot index with another grid: rebuild then too
  if (!b->dirty && run == b->table) return CGKS_OK;
  b->dirty = 0;
  b->table = run;
  BatchTable& t = *b->h_tab;
  t.n = (int)run.size();
  for (int q = 0; q < BK_KINDS; ++q) t.face[q].n = t.face[q].pre[0][0] = t.face[q].pre[1][0] = 0;
  for (int q = 0; q < 2; ++q) t.upd[q].n = t.upd[q].pre[0] = 0;
  for (int i = 0; i < t.n; ++i) {
    const SlotInfo& in = b->info[run[i]];
    t.slot[i] = run[i];
    FaceList& F = t.face[in.kind];
    F.slot[F.n] = run[i];
    F.pre[0][F.n + 1] = F.pre[0][F.n] + in.nb[0];
    F.pre[1][F.n + 1] = F.pre[1][F.n] + in.nb[1];
    ++F.n;
    UpdateList& U = t.upd[kind_f32(in.kind)];
    U.slot[U.n] = run[i];
    U.pre[U.n + 1] = U.pre[U.n] + in.nbu;
    ++U.n;
  }
  // grids: power-of-two buckets (0 for an empty list: its launches are left
  // out); a new graph only when a list leaves its bucket (buckets are
  // multiples of NXCD and >= NXCD * ceil(len / NXCD), as the face kernels'
  // XCD mapping needs)
  auto bucket = [](int len, int cap) {
    if (len == 0) return 0;
    const int need = (len + NXCD - 1) / NXCD * NXCD;
    if (cap > 0 && need <= cap && 4 * need > cap) return cap;
    int c = 64;
    while (c < need) c *= 2;
    return c;
  };
  bool changed = false;
  auto rebucket = [&](int len, int& cap) {
    const int c = bucket(len, cap);
    changed |= c != cap;
    cap = c;
  };
  rebucket(t.n, b->cap_n);
  for (int q = 0; q < BK_KINDS; ++q)
    for (int d = 0; d < 2; ++d) rebucket(t.face[q].pre[d][t.face[q].n], b->cap_f[q][d]);
  for (int q = 0; q < 2; ++q) rebucket(t.upd[q].pre[t.upd[q].n], b->cap_u2[q]);
  if (changed) drop_graph(b);
  HIPCHK(hipMemcpyAsync(b->d_tab, &t, sizeof t, hipMemcpyHostToDevice, b->stream));
  return CGKS_OK;
}

// One step of every running slot: begin, the face kernels of each kind present
// and the updates of each storage present for both stages, end.
static void launch_batch_step(cgks_batch* b) {
  hipStream_t s = b->stream;
  const SlotDev* sl = b->d_slots;
  const BatchTable* t = b->d_tab;
  kb_begin<<<b->cap_n, 256, 0, s>>>(sl, t);
  using D0 = std::integral_constant<int, 0>;
  using D1 = std::integral_constant<int, 1>;
  auto faces = [&](auto dir, auto stage) {
    constexpr int DIR = decltype(dir)::value, STAGE = decltype(stage)::value;
    for (int q = 0; q < BK_KINDS; ++q) {
      const int g = b->cap_f[q][DIR];
      if (!g) continue;
      using F = std::false_type;
      using T = std::true_type;
      auto go = [&](auto gt, auto tl, auto ch, auto ss, auto tw) {
        kb_faces<DIR, STAGE, decltype(gt), decltype(tl), decltype(ch)::value, decltype(ss)::value,
                 decltype(tw)::value><<<g, FACE_THREADS, 0, s>>>(sl, t, q);
      };
      // the tile shapes of kind_tile
      auto go_ch = [&](auto ch, auto ss) {
        if (kind_g4(q)) {
          if (!kind_f32(q)) { if constexpr (DIR == 0) go(0.0, Tile4x16G4(), ch, ss, F()); else go(0.0, Tile2x32G4(), ch, ss, F()); }
          else { if constexpr (DIR == 0) go(0.0f, Tile4x16G4(), ch, ss, F()); else go(0.0f, Tile2x32G4(), ch, ss, F()); }
        } else if (kind_f32(q)) {
          if constexpr (DIR == 0) go(0.0f, Tile4x32(), ch, ss, F()); else go(0.0f, Tile2x64(), ch, ss, F());
        } else {
          if constexpr (DIR == 0) go(0.0, Tile4x32(), ch, ss, F()); else go(0.0, Tile2x64(), ch, ss, F());
        }
      };
      if (kind_char(q)) {
        go_ch(T(), F());
      } else if (kind_side(q)) {
        go_ch(F(), T());
      } else if (kind_tw(q)) {   // two points: the 5-segment halo tiles; four: the four-point tiles
        if (kind_g4(q)) {
          if (kind_f32(q)) { if constexpr (DIR == 0) go(0.0f, Tile4x16G4(), F(), F(), T()); else go(0.0f, Tile2x32G4(), F(), F(), T()); }
          else { if constexpr (DIR == 0) go(0.0, Tile4x16G4(), F(), F(), T()); else go(0.0, Tile2x32G4(), F(), F(), T()); }
        } else if (kind_f32(q)) { if constexpr (DIR == 0) go(0.0f, Tile4x32W(), F(), F(), T()); else go(0.0f, Tile2x64W(), F(), F(), T()); }
        else { if constexpr (DIR == 0) go(0.0, Tile4x32W(), F(), F(), T()); else go(0.0, Tile2x64W(), F(), F(), T()); }
      } else if (q != BK_G2) {
        go_ch(F(), F());
      } else {
        switch (b->tile[DIR]) {
          case 1: go(0.0, Tile4x32(), F(), F(), F()); break;
          case 2: go(0.0, Tile2x64(), F(), F(), F()); break;
          default: go(0.0, Tile8x16(), F(), F(), F()); break;
        }
      }
    }
  };
  auto updates = [&](auto stage) {
    constexpr int STAGE = decltype(stage)::value;
    if (b->cap_u2[0]) kb_update<STAGE, double><<<b->cap_u2[0], 256, 0, s>>>(sl, t, 0);
    if (b->cap_u2[1]) kb_update<STAGE, float><<<b->cap_u2[1], 256, 0, s>>>(sl, t, 1);
  };
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  faces(D0(), S1());
  faces(D1(), S1());
  updates(S1());
  faces(D0(), S2());
  faces(D1(), S2());
  updates(S2());
  kb_end<<<b->cap_n, 64, 0, s>>>(sl, t);
}

extern "C" int cgks_batch_run(cgks_batch* b, int steps) {
  if (!b || steps < 1) return CGKS_EINVAL;
  int rc = refresh_table(b);
  if (rc) return rc;
  if (b->table.empty()) return CGKS_OK;
  if (!b->exec || b->graph_steps != steps) {
    drop_graph(b);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < steps; ++k) launch_batch_step(b);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e1 != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return CGKS_EDEVICE;
    }
    const hipError_t e3 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
      b->exec = nullptr;
      return CGKS_EDEVICE;
    }
    b->graph_steps = steps;
  }
  HIPCHK(hipGraphLaunch(b->exec, b->stream));
  HIPCHK(hipMemcpyAsync(b->h_sc, b->d_sc, sizeof(Scalars) * b->max_slots, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  return CGKS_OK;
}

extern "C" int cgks_batch_poll(cgks_batch* b, int slot, int* state, double* t, long* step) {
  if (!b || slot < 0 || slot >= b->max_slots) return CGKS_EINVAL;
  if (state) *state = slot_state(b, slot);
  if (t) *t = b->h_sc[slot].t;
  if (step) *step = (long)b->h_sc[slot].step;
  return CGKS_OK;
}

extern "C" int cgks_batch_read(cgks_batch* b, int slot, double* fields_out, int on_device) {
  if (!b || !fields_out || slot < 0 || slot >= b->max_slots) return CGKS_EINVAL;
  if (!b->info[slot].used) return CGKS_ESTATE;
  const SlotDev& sd = b->h_slots[slot];
  const size_t N = b->info[slot].N;
  const double* S = sd.B.S[b->h_sc[slot].cur];
  if (kind_f32(b->info[slot].kind)) {
    // converted to FP64 straight into a device output, else via W* (free between steps)
    double* dst = on_device ? fields_out : sd.B.Ws;
    k_from_storage32<<<(unsigned)((N + 255) / 256), 256, 0, b->stream>>>(S, dst, N);
    HIPCHK(hipGetLastError());
    if (!on_device)
      HIPCHK(hipMemcpyAsync(fields_out, sd.B.Ws, 12 * N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  } else {
    HIPCHK(hipMemcpyAsync(fields_out, S, 12 * N * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
  }
  HIPCHK(hipStreamSynchronize(b->stream));
  return CGKS_OK;
}

extern "C" int cgks_batch_set_tiles(cgks_batch* b, int x_shape, int y_shape) {
  if (!b || x_shape < 0 || x_shape >= kTileShapes || y_shape < 0 || y_shape >= kTileShapes) return CGKS_EINVAL;
  for (int k = 0; k < b->max_slots; ++k)
    if (b->info[k].used) return CGKS_ESTATE;
  b->tile[0] = x_shape;
  b->tile[1] = y_shape;
  drop_graph(b);
  return CGKS_OK;
}

extern "C" int cgks_batch_tuning(int* x_shape, int* y_shape, int* steps_per_run) {
  if (x_shape) *x_shape = kBatchTune.x;
  if (y_shape) *y_shape = kBatchTune.y;
  if (steps_per_run) *steps_per_run = kBatchTune.steps;
  return CGKS_OK;
}

extern "C" int cgks_batch_release(cgks_batch* b, int slot) {
  if (!b || slot < 0 || slot >= b->max_slots) return CGKS_EINVAL;
  SlotInfo& in = b->info[slot];
  if (!in.used) return CGKS_ESTATE;
  HIPCHK(hipStreamSynchronize(b->stream));
  b->arena.release(in.off, in.bytes);
  in = SlotInfo();
  std::memset(&b->h_sc[slot], 0, sizeof(Scalars));
  b->dirty = 1;
  return CGKS_OK;
}
