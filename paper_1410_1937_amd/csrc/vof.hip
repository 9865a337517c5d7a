// libnfa: operator-split VOF advection of the water fraction (Interface
// reconstruction and advection section: the transport of eq. vof in three
// one-directional sweeps with a dilation term, after the flux correction
// that restores eq. diverge cell by cell; piecewise-planar interfaces).
//
// One time step:  phi -> sweep(d1, explicit) -> sweep(d2, explicit) ->
// sweep(d3, implicit), with (d1, d2, d3) = (x, y, z) on even steps and
// (z, y, x) on odd ones.  In a sweep along d every active cell
//   - takes its face velocities uhat = dx_d F~ / V from the open-area fluxes
//     F = A u; on z-faces F~ carries the cell's share of its imbalance
//     E = sum over faces of (F+ - F-), split in proportion to the two z areas;
//   - passes across each of its two d-faces the water in the slab of
//     thickness |uhat| dt of the upwind cell next to that face: the slab's
//     volume times the part of it below the upwind cell's interface plane,
//     or times that cell's fraction when it has no plane;
//   - adds the dilation dt phi (uhat+ - uhat-) / dx_d with the sweep's input
//     fraction (explicit), or divides by 1 - dt (uhat+ - uhat-) / dx_d
//     (implicit, the last sweep).
// A cell with 0 < phi < 1 and a non-zero normal has a plane: the normal is
// -grad phi by central differences averaged across the difference direction
// with weights 1/4, 1/2, 1/4 over the 3x3x3 neighbourhood (beyond the domain
// the edge cell repeats; a neighbour inside the body takes the cell's own
// fraction); the plane constant puts the fraction phi of the cell below the
// plane, found by 64 bisection steps on the cube's volume function (the
// closed form of Scardovelli and Zaleski).  A fraction within 1e-12 of 0 or
// 1 counts as an empty or full cell without a plane.
//
// Work layout.  Interface cells are about 1 % of the grid, so a plane per
// thread of the sweep would leave most lanes of a wavefront idle through
// the bisection.  Each sweep therefore runs in two launches:
//   k_planes  each block scans its rows for active cells with
//             1e-12 < phi < 1 - 1e-12, stages them in LDS and solves them a
//             block at a time (normal, bisection), storing the plane in a
//             per-cell table (signed normal, constant);
//   k_sweep   one thread per cell, x fastest: face speeds, the two face
//             fluxes (reading the upwind cell's plane from the table), the
//             update.  All loads a cell may need are issued before any is
//             used, so a wavefront waits for memory about once per cell.
// Both take grid rows (x-lines) round robin.
//
// Built with -ffp-contract=off: every expression is rounded as written.
#include <cmath>

#include "device_util.h"
#include "nfa_internal.h"

namespace nfa {
namespace {

constexpr int kBisect = 64;
constexpr double kEps = 1e-12;   // fractions within kEps of 0 or 1 have no plane
constexpr int kRowBlocks = 4096;   // blocks of the row kernels

struct Sweep {
  int nx, ny, nz;
  const double* __restrict__ phi;   // fraction before the sweep
  double* __restrict__ out;         // fraction after it
  const unsigned char* __restrict__ act;
  const double* __restrict__ ox;    // open face areas
  const double* __restrict__ oy;
  const double* __restrict__ oz;
  const double* __restrict__ u;     // face velocities relative to the body
  const double* __restrict__ v;
  const double* __restrict__ w;
  const double* __restrict__ dx;    // cell widths
  const double* __restrict__ dy;
  const double* __restrict__ dz;
  const double* __restrict__ gx;    // normal-stencil spans
  const double* __restrict__ gy;
  const double* __restrict__ gz;
  double dt;
};

__device__ __forceinline__ double clip01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

__device__ __forceinline__ void sort3(double& a, double& b, double& c) {
  double t;
  if (b < a) { t = a; a = b; b = t; }
  if (c < b) { t = b; b = c; c = t; }
  if (b < a) { t = a; a = b; b = t; }
}

// Fraction of the unit cube with n1 x + n2 y + n3 z <= a, for
// 0 <= n1 <= n2 <= n3 and n1 + n2 + n3 = 1; the half a > 1/2 by V(a) = 1 - V(1 - a).
__device__ double unit_fraction(double n1, double n2, double n3, double a) {
  if (a <= 0.0) return 0.0;
  if (a >= 1.0) return 1.0;
  const bool low = a <= 0.5;
  const double s = low ? a : 1.0 - a;
  const double n12 = n1 + n2;
  double v;
  if (s <= 0.0) {
    v = 0.0;
  } else if (s <= n1) {      // a corner tetrahedron
    v = ((s * s) * s) / (((6.0 * n1) * n2) * n3);
  } else if (s <= n2) {      // the plane crosses the n1 edges
    v = ((s * (s - n1)) + ((n1 * n1) / 3.0)) / ((2.0 * n2) * n3);
  } else if (s <= fmin(n12, n3)) {
    v = ((((s * s) * ((3.0 * n12) - s)) + ((n1 * n1) * (n1 - (3.0 * s)))) + ((n2 * n2) * (n2 - (3.0 * s)))) /
        (((6.0 * n1) * n2) * n3);
  } else if (n3 < n12) {
    v = (((((s * s) * (3.0 - (2.0 * s))) + ((n1 * n1) * (n1 - (3.0 * s)))) + ((n2 * n2) * (n2 - (3.0 * s)))) +
         ((n3 * n3) * (n3 - (3.0 * s)))) /
        (((6.0 * n1) * n2) * n3);
  } else {                   // a slab of the n3 axis
    v = ((2.0 * s) - n12) / (2.0 * n3);
  }
  return low ? v : 1.0 - v;
}

__device__ __forceinline__ bool in_band(double phi) { return phi > kEps && phi < 1.0 - kEps; }

__device__ __forceinline__ long long cell(const Sweep& A, int i, int j, int k) {
  return ((long long)k * A.ny + j) * A.nx + i;
}

// -grad phi at (i, j, k) (x, y, z components).
__device__ void normal(const Sweep& A, int i, int j, int k, double m[3]) {
  const double pc = clip01(A.phi[cell(A, i, j, k)]);
  double P[3][3][3];   // [dz + 1][dy + 1][dx + 1]
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int kk = min(max(k + c - 1, 0), A.nz - 1);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int jj = min(max(j + b - 1, 0), A.ny - 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ii = min(max(i + a - 1, 0), A.nx - 1);
        const long long q = cell(A, ii, jj, kk);
        P[c][b][a] = A.act[q] ? clip01(A.phi[q]) : pc;
      }
    }
  }
  const double W[3] = {0.25, 0.5, 0.25};
  double ax = 0.0, ay = 0.0, az = 0.0;
  // x: across (y, z), outer loop over y, inner over z
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) ax = ax + (W[b] * W[c]) * (P[c][b][2] - P[c][b][0]);
  // y: across (x, z)
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) ay = ay + (W[a] * W[c]) * (P[c][2][a] - P[c][0][a]);
  // z: across (x, y)
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) az = az + (W[a] * W[b]) * (P[2][b][a] - P[0][b][a]);
  m[0] = -(ax / A.gx[i]);
  m[1] = -(ay / A.gy[j]);
  m[2] = -(az / A.gz[k]);
}

// Plane table entry of an in-band cell: the normalized normal n >= 0 (sum 1)
// of the reflected, scaled cube, with the sign bit set on a reflected axis
// (-0.0 for a reflected zero component), and the constant t in [0, 1] (water
// where n . xi <= t); t = -1 when the normal is zero (no plane).
__device__ double4 make_plane(const Sweep& A, int i, int j, int k, double phi) {
  double m[3];
  normal(A, i, j, k, m);
  if (!(((fabs(m[0]) + fabs(m[1])) + fabs(m[2])) > 0.0)) return make_double4(0.0, 0.0, 0.0, -1.0);
  const double dims[3] = {A.dx[i], A.dy[j], A.dz[k]};
  double nm[3], n[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) nm[e] = fabs(m[e]) * dims[e];
  const double S = (nm[0] + nm[1]) + nm[2];
#pragma unroll
  for (int e = 0; e < 3; ++e) n[e] = nm[e] / S;
  double n1 = n[0], n2 = n[1], n3 = n[2];
  sort3(n1, n2, n3);
  const double ph = clip01(phi);
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < kBisect; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (unit_fraction(n1, n2, n3, mid) < ph) lo = mid;
    else hi = mid;
  }
  return make_double4(m[0] < 0.0 ? -n[0] : n[0], m[1] < 0.0 ? -n[1] : n[1], m[2] < 0.0 ? -n[2] : n[2],
                      0.5 * (lo + hi));
}

// Water volume in the slab of thickness speed dt next to the upper (or
// lower) d-face of donor cell cd: width dw along d, volume vol, fraction phi.
__device__ __forceinline__ double water(const double4* __restrict__ planes, long long cd, double phi, double dw,
                                        double vol, int d, bool upper, double speed, double dt) {
  const double frac = fmin(speed * dt, dw) / dw;
  const double slab = frac * vol;
  if (!in_band(phi)) return slab * clip01(phi);
  const double4 P = planes[cd];
  if (!(P.w >= 0.0)) return slab * clip01(phi);
  const double pn[3] = {fabs(P.x), fabs(P.y), fabs(P.z)};
  double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {1.0, 1.0, 1.0};
  if (upper) lo[d] = 1.0 - frac;
  else hi[d] = frac;
  const double pd = d == 0 ? P.x : (d == 1 ? P.y : P.z);
  if (signbit(pd)) {
    const double l = 1.0 - hi[d], h = 1.0 - lo[d];
    lo[d] = l;
    hi[d] = h;
  }
  double nn[3], nl[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    nn[e] = pn[e] * (hi[e] - lo[e]);
    nl[e] = pn[e] * lo[e];
  }
  const double S = (nn[0] + nn[1]) + nn[2];
  const double tt = P.w - ((nl[0] + nl[1]) + nl[2]);
  double f;
  if (S > 0.0) {
    double q1 = nn[0] / S, q2 = nn[1] / S, q3 = nn[2] / S;
    sort3(q1, q2, q3);
    f = unit_fraction(q1, q2, q3, tt / S);
  } else {
    f = tt >= 0.0 ? 1.0 : 0.0;
  }
  return slab * f;
}

// Rows (x-lines, row r = k ny + j) are dealt to blocks round robin, so the
// free surface's band of rows spreads over every block and XCD; the logical
// block order is remapped so that the blocks of one XCD take neighbouring
// rows.
__device__ __forceinline__ int first_row() { return xcd_remap(blockIdx.x, gridDim.x); }

// The cells of a block, in chunks of blockDim: chunk q is part q % cpr of
// the block's row q / cpr (rows first_row(), first_row() + gridDim, ...).
struct Chunks {
  int r0, cpr, nq;
};

__device__ __forceinline__ Chunks block_chunks(int nx, int nrows) {
  Chunks C;
  C.r0 = first_row();
  C.cpr = (nx + blockDim.x - 1) / blockDim.x;
  const int nr = C.r0 < nrows ? (nrows - C.r0 + gridDim.x - 1) / gridDim.x : 0;
  C.nq = nr * C.cpr;
  return C;
}

// Row and x-index of this thread's cell in chunk q; valid = inside the grid.
__device__ __forceinline__ bool chunk_cell(const Chunks& C, int q, int nx, int nrows, int& r, int& i) {
  r = C.r0 + (q / C.cpr) * gridDim.x;
  i = (q % C.cpr) * blockDim.x + threadIdx.x;
  return q < C.nq && r < nrows && i < nx;
}

constexpr int kScanUnroll = 4;             // chunks loaded per barrier in the plane scan

// Planes of every active in-band cell.  Each block scans its rows (loading
// kScanUnroll chunks before it waits), stages the in-band cells in LDS and
// solves them a full block at a time (one cell per thread), so the bisection
// runs on dense wavefronts.
__global__ __launch_bounds__(kBlock) void k_planes(Sweep A, double4* __restrict__ planes) {
  __shared__ int s_list[(kScanUnroll + 1) * kBlock];
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const int nx = A.nx, nrows = A.ny * A.nz;
  const unsigned unx = nx, uny = A.ny;
  auto solve = [&](int e) {
    const unsigned c = s_list[e];
    const unsigned r = c / unx;
    const int i = (int)(c - r * unx);
    const int k = (int)(r / uny);
    const int j = (int)(r - (unsigned)k * uny);
    planes[c] = make_plane(A, i, j, k, A.phi[c]);
  };
  const Chunks C = block_chunks(nx, nrows);
  for (int q0 = 0; q0 < C.nq; q0 += kScanUnroll) {
    bool f[kScanUnroll];
    long long cc[kScanUnroll];
    double ph[kScanUnroll];
    unsigned char ac[kScanUnroll];
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      int r, i;
      f[u] = chunk_cell(C, q0 + u, nx, nrows, r, i);
      cc[u] = f[u] ? (long long)r * nx + i : 0;
      ph[u] = A.phi[cc[u]];
      ac[u] = A.act[cc[u]];
    }
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      const bool g = f[u] && ac[u] && in_band(ph[u]);
      const unsigned long long mask = __ballot(g);
      if (mask != 0) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((long long)mask) - 1;
        int b = 0;
        if (lane == leader) b = atomicAdd(&s_cnt, __popcll(mask));
        b = __shfl(b, leader, 64);
        if (g) s_list[b + __popcll(mask & ((1ull << lane) - 1ull))] = (int)cc[u];
      }
    }
    __syncthreads();
    const int m = s_cnt;
    const int full = m / (int)blockDim.x;
    if (full > 0) {                 // dense rounds; the remainder moves to the front
      for (int t = 0; t < full; ++t) solve(t * blockDim.x + threadIdx.x);
      const int rest = m - full * (int)blockDim.x;
      const int keep = (int)threadIdx.x < rest ? s_list[full * blockDim.x + threadIdx.x] : 0;
      __syncthreads();
      if ((int)threadIdx.x < rest) s_list[threadIdx.x] = keep;
      if (threadIdx.x == 0) s_cnt = rest;
    }
    __syncthreads();
  }
  const int m = s_cnt;
  if ((int)threadIdx.x < m) solve(threadIdx.x);
}

// What a sweep along D reads for one cell.
struct CellIn {
  long long c, cm, cp;        // the cell and its neighbours along D (itself beyond the domain)
  int i, j, k;
  bool valid, act;
  double phi, phim, phip;
  double dxc, dyc, dzc, wm, wp, vm, vp_;   // widths, neighbour widths along D, neighbour volumes' factors
  double a[12];               // face data
};

template <int D>
__device__ __forceinline__ void load_cell(const Sweep& A, const Chunks& C, int q, CellIn& X) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  int r, i;
  X.valid = chunk_cell(C, q, nx, ny * nz, r, i);
  if (!X.valid) {
    r = 0;
    i = 0;
  }
  const int k = r / ny, j = r - k * ny;
  X.i = i;
  X.j = j;
  X.k = k;
  const long long plane = (long long)nx * ny;
  const long long c = ((long long)k * ny + j) * nx + i;
  const int pos = D == 0 ? i : (D == 1 ? j : k);
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const long long sD = D == 0 ? 1 : (D == 1 ? nx : plane);
  const bool hasm = pos > 0, hasp = pos < nD - 1;
  X.c = c;
  X.cm = hasm ? c - sD : c;
  X.cp = hasp ? c + sD : c;
  X.phi = A.phi[c];
  X.act = A.act[c] != 0;
  X.phim = A.phi[X.cm];
  X.phip = A.phi[X.cp];
  X.dxc = A.dx[i];
  X.dyc = A.dy[j];
  X.dzc = A.dz[k];
  // the donor volumes (dz dy) dx of the two neighbours along D
  const int im = D == 0 && hasm ? i - 1 : i, ip = D == 0 && hasp ? i + 1 : i;
  const int jm = D == 1 && hasm ? j - 1 : j, jp = D == 1 && hasp ? j + 1 : j;
  const int km = D == 2 && hasm ? k - 1 : k, kp = D == 2 && hasp ? k + 1 : k;
  const double dxm = A.dx[im], dxp = A.dx[ip], dym = A.dy[jm], dyp = A.dy[jp], dzm = A.dz[km], dzp = A.dz[kp];
  X.wm = D == 0 ? dxm : (D == 1 ? dym : dzm);
  X.wp = D == 0 ? dxp : (D == 1 ? dyp : dzp);
  X.vm = (dzm * dym) * dxm;
  X.vp_ = (dzp * dyp) * dxp;
  const long long fxm = ((long long)k * ny + j) * (nx + 1) + i;
  const long long fym = ((long long)k * (ny + 1) + j) * nx + i;
  if (D == 0 || D == 2) {
    X.a[0] = A.ox[fxm];
    X.a[1] = A.u[fxm];
    X.a[2] = A.ox[fxm + 1];
    X.a[3] = A.u[fxm + 1];
  }
  if (D == 1 || D == 2) {
    X.a[4] = A.oy[fym];
    X.a[5] = A.v[fym];
    X.a[6] = A.oy[fym + nx];
    X.a[7] = A.v[fym + nx];
  }
  if (D == 2) {
    X.a[8] = A.oz[c];
    X.a[9] = A.w[c];
    X.a[10] = A.oz[c + plane];
    X.a[11] = A.w[c + plane];
  }
}

template <int D, bool IMPLICIT>
__device__ __forceinline__ void update_cell(const Sweep& A, const double4* __restrict__ planes, const CellIn& X) {
  if (!X.valid) return;
  if (!X.act) {
    A.out[X.c] = X.phi;
    return;
  }
  const double dt = A.dt;
  const double V = (X.dzc * X.dyc) * X.dxc;
  double lo, up;
  if (D == 0) {
    lo = (X.dxc * (X.a[0] * X.a[1])) / V;
    up = (X.dxc * (X.a[2] * X.a[3])) / V;
  } else if (D == 1) {
    lo = (X.dyc * (X.a[4] * X.a[5])) / V;
    up = (X.dyc * (X.a[6] * X.a[7])) / V;
  } else {
    const double Fxm = X.a[0] * X.a[1], Fxp = X.a[2] * X.a[3];
    const double Fym = X.a[4] * X.a[5], Fyp = X.a[6] * X.a[7];
    const double Azm = X.a[8], Azp = X.a[10];
    double Fzm = Azm * X.a[9], Fzp = Azp * X.a[11];
    const double E = ((Fxp - Fxm) + (Fyp - Fym)) + (Fzp - Fzm);
    const double den = Azp + Azm;
    if (den > 0.0) {
      Fzp = Fzp - (E * Azp) / den;
      Fzm = Fzm + (E * Azm) / den;
    }
    lo = (X.dzc * Fzm) / V;
    up = (X.dzc * Fzp) / V;
  }
  const double wc = D == 0 ? X.dxc : (D == 1 ? X.dyc : X.dzc);
  double f_up, f_lo;
  if (up > 0.0) f_up = water(planes, X.c, X.phi, wc, V, D, true, up, dt);
  else if (up < 0.0) f_up = -water(planes, X.cp, X.phip, X.wp, X.vp_, D, false, -up, dt);
  else f_up = 0.0;
  if (lo > 0.0) f_lo = water(planes, X.cm, X.phim, X.wm, X.vm, D, true, lo, dt);
  else if (lo < 0.0) f_lo = -water(planes, X.c, X.phi, wc, V, D, false, -lo, dt);
  else f_lo = 0.0;
  const double div = (up - lo) / wc;
  const double rest = X.phi - (f_up - f_lo) / V;
  A.out[X.c] = IMPLICIT ? rest / (1.0 - dt * div) : rest + (dt * X.phi) * div;
}

// Two chunks per iteration: both cells' loads are in flight before either
// is used.
template <int D, bool IMPLICIT>
__global__ __launch_bounds__(kBlock) void k_sweep(Sweep A, const double4* __restrict__ planes) {
  const Chunks C = block_chunks(A.nx, A.ny * A.nz);
  for (int q = 0; q < C.nq; q += 2) {
    CellIn X0, X1;
    load_cell<D>(A, C, q, X0);
    load_cell<D>(A, C, q + 1, X1);
    update_cell<D, IMPLICIT>(A, planes, X0);
    update_cell<D, IMPLICIT>(A, planes, X1);
  }
}

// What the z sweep loads for plane k of its column: the fraction above,
// the upper z-face, the flag and the x- and y-faces of the cell.
struct ZIn {
  double phip, Azp, wzp, ox0, u0, ox1, u1, oy0, v0, oy1, v1;
  unsigned char act;
};

__device__ __forceinline__ void load_z(const Sweep& A, long long c, int k, long long fxm, long long fym, ZIn& Z) {
  const long long plane = (long long)A.nx * A.ny;
  Z.phip = A.phi[k < A.nz - 1 ? c + plane : c];
  Z.Azp = A.oz[c + plane];
  Z.wzp = A.w[c + plane];
  Z.act = A.act[c];
  Z.ox0 = A.ox[fxm];
  Z.u0 = A.u[fxm];
  Z.ox1 = A.ox[fxm + 1];
  Z.u1 = A.u[fxm + 1];
  Z.oy0 = A.oy[fym];
  Z.v0 = A.v[fym];
  Z.oy1 = A.oy[fym + A.nx];
  Z.v1 = A.v[fym + A.nx];
}

// The z sweep marches up columns: a block takes one chunk of an x-line (j)
// over a segment of planes; the fraction below, the cell's own fraction and
// the lower z-face come from the previous plane in registers, so each is
// read from memory once, and the next plane's inputs are loaded before the
// current one is computed.  Neighbouring logical blocks take neighbouring j,
// so the y-faces a block shares with the next line are read on one XCD.
template <bool IMPLICIT>
__global__ __launch_bounds__(kBlock) void k_sweep_z(Sweep A, const double4* __restrict__ planes, int nseg) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int cpr = (nx + blockDim.x - 1) / blockDim.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = lb % cpr, j = (lb / cpr) % ny, seg = lb / (cpr * ny);
  const int per = (nz + nseg - 1) / nseg;
  const int k0 = seg * per, k1 = min(nz, k0 + per);
  if (seg >= nseg || k0 >= k1) return;
  const int i = chunk * (int)blockDim.x + threadIdx.x;
  const bool valid = i < nx;
  const int ic = valid ? i : 0;
  const long long plane = (long long)nx * ny;
  const double dxc = A.dx[ic], dyc = A.dy[j];
  long long c = ((long long)k0 * ny + j) * nx + ic;
  long long fxm = ((long long)k0 * ny + j) * (nx + 1) + ic;
  long long fym = ((long long)k0 * (ny + 1) + j) * nx + ic;
  const long long sfx = (long long)ny * (nx + 1), sfy = (long long)(ny + 1) * nx;
  double phim = A.phi[k0 > 0 ? c - plane : c];
  double phi = A.phi[c];
  double Azm = A.oz[c], wzm = A.w[c];
  ZIn cur, nxt;
  load_z(A, c, k0, fxm, fym, cur);
  for (int k = k0; k < k1; ++k) {
    if (k + 1 < k1) load_z(A, c + plane, k + 1, fxm + sfx, fym + sfy, nxt);
    const int km = k > 0 ? k - 1 : k, kp = k < nz - 1 ? k + 1 : k;
    CellIn X;
    X.valid = valid;
    X.i = ic;
    X.j = j;
    X.k = k;
    X.c = c;
    X.cm = k > 0 ? c - plane : c;
    X.cp = k < nz - 1 ? c + plane : c;
    X.act = cur.act != 0;
    X.phi = phi;
    X.phim = phim;
    X.phip = cur.phip;
    X.dxc = dxc;
    X.dyc = dyc;
    X.dzc = A.dz[k];
    const double dzm = A.dz[km], dzp = A.dz[kp];
    X.wm = dzm;
    X.wp = dzp;
    X.vm = (dzm * dyc) * dxc;
    X.vp_ = (dzp * dyc) * dxc;
    X.a[0] = cur.ox0;
    X.a[1] = cur.u0;
    X.a[2] = cur.ox1;
    X.a[3] = cur.u1;
    X.a[4] = cur.oy0;
    X.a[5] = cur.v0;
    X.a[6] = cur.oy1;
    X.a[7] = cur.v1;
    X.a[8] = Azm;
    X.a[9] = wzm;
    X.a[10] = cur.Azp;
    X.a[11] = cur.wzp;
    update_cell<2, IMPLICIT>(A, planes, X);
    phim = phi;
    phi = cur.phip;
    Azm = cur.Azp;
    wzm = cur.wzp;
    cur = nxt;
    c += plane;
    fxm += sfx;
    fym += sfy;
  }
}

// Segments of the z columns: enough blocks to fill the chip.
int z_segments(const Sweep& A) {
  const int cols = ((A.nx + kBlock - 1) / kBlock) * A.ny;
  return std::max(1, std::min(A.nz, (kRowBlocks + cols - 1) / cols));
}

void launch_sweep(const Sweep& A, int d, bool implicit, const double4* planes, hipStream_t s) {
  const int nb = std::min(kRowBlocks, A.ny * A.nz);
  k_planes<<<nb, kBlock, 0, s>>>(A, const_cast<double4*>(planes));
  if (d == 0) {
    if (implicit) k_sweep<0, true><<<nb, kBlock, 0, s>>>(A, planes);
    else k_sweep<0, false><<<nb, kBlock, 0, s>>>(A, planes);
  } else if (d == 1) {
    if (implicit) k_sweep<1, true><<<nb, kBlock, 0, s>>>(A, planes);
    else k_sweep<1, false><<<nb, kBlock, 0, s>>>(A, planes);
  } else {
    const int nseg = z_segments(A);
    const int nbz = ((A.nx + kBlock - 1) / kBlock) * A.ny * nseg;
    if (implicit) k_sweep_z<true><<<nbz, kBlock, 0, s>>>(A, planes, nseg);
    else k_sweep_z<false><<<nbz, kBlock, 0, s>>>(A, planes, nseg);
  }
}

Sweep make_sweep(const Grid& g, const double* u, const double* v, const double* w, double dt) {
  Sweep A;
  A.nx = g.nx;
  A.ny = g.ny;
  A.nz = g.nz;
  A.phi = nullptr;
  A.out = nullptr;
  A.act = g.active.as<unsigned char>();
  A.ox = g.open_x.as<double>();
  A.oy = g.open_y.as<double>();
  A.oz = g.open_z.as<double>();
  A.u = u;
  A.v = v;
  A.w = w;
  A.dx = g.d_dx.as<double>();
  A.dy = g.d_dy.as<double>();
  A.dz = g.d_dz.as<double>();
  A.gx = g.d_gx.as<double>();
  A.gy = g.d_gy.as<double>();
  A.gz = g.d_gz.as<double>();
  A.dt = dt;
  return A;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

}  // namespace
}  // namespace nfa

using namespace nfa;

// Work memory of the advection: the plane table and one fraction buffer.
struct nfa_vof_s {
  nfa::Grid* g = nullptr;
  nfa::DevBuf planes;    // double4 per cell
  nfa::DevBuf work;      // double per cell
};

extern "C" nfa_status nfa_vof_create(nfa_grid g, nfa_vof* out) {
  if (!out) return fail(NFA_ERR_INVALID, "nfa_vof_create: out is NULL");
  *out = nullptr;
  if (!g) return fail(NFA_ERR_INVALID, "nfa_vof_create: NULL grid");
  auto* v = new nfa_vof_s();
  v->g = g;
  const size_t n = (size_t)g->n;
  hipError_t e;
  if ((e = v->planes.alloc(n * sizeof(double4))) != hipSuccess || (e = v->work.alloc(n * 8)) != hipSuccess) {
    delete v;
    return fail(NFA_ERR_HIP, std::string("nfa_vof_create: ") + hipGetErrorString(e));
  }
  *out = v;
  return NFA_OK;
}

extern "C" void nfa_vof_destroy(nfa_vof v) { delete v; }

namespace {

nfa_status check(const char* who, nfa_vof vf, const double* phi, const double* u, const double* v,
                 const double* w, double dt, const double* phi_out) {
  if (!vf || !phi || !u || !v || !w || !phi_out) return fail(NFA_ERR_INVALID, std::string(who) + ": NULL argument");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(NFA_ERR_INVALID, std::string(who) + ": dt must be finite and > 0");
  if (overlap(phi, phi_out, (size_t)vf->g->n * 8))
    return fail(NFA_ERR_INVALID, std::string(who) + ": phi_out must not overlap phi");
  return NFA_OK;
}

}  // namespace

extern "C" nfa_status nfa_vof_sweep(nfa_vof vf, const double* phi, const double* u, const double* v,
                                    const double* w, double dt, int dir, int implicit, double* phi_out,
                                    nfa_stream s) {
  nfa_status e = check("nfa_vof_sweep", vf, phi, u, v, w, dt, phi_out);
  if (e != NFA_OK) return e;
  if (dir < 0 || dir > 2) return fail(NFA_ERR_INVALID, "nfa_vof_sweep: dir must be 0, 1 or 2");
  Sweep A = make_sweep(*vf->g, u, v, w, dt);
  A.phi = phi;
  A.out = phi_out;
  launch_sweep(A, dir, implicit != 0, vf->planes.as<double4>(), S(s));
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_vof_advect(nfa_vof vf, const double* phi, const double* u, const double* v,
                                     const double* w, double dt, int step, double* phi_out, nfa_stream s) {
  nfa_status e = check("nfa_vof_advect", vf, phi, u, v, w, dt, phi_out);
  if (e != NFA_OK) return e;
  const hipStream_t st = S(s);
  double* work = vf->work.as<double>();
  const int order[2][3] = {{0, 1, 2}, {2, 1, 0}};
  const int* o = order[step % 2 == 0 ? 0 : 1];
  // phi -> phi_out -> work -> phi_out
  const double* src[3] = {phi, phi_out, work};
  double* dst[3] = {phi_out, work, phi_out};
  Sweep A = make_sweep(*vf->g, u, v, w, dt);
  for (int p = 0; p < 3; ++p) {
    A.phi = src[p];
    A.out = dst[p];
    launch_sweep(A, o[p], p == 2, vf->planes.as<double4>(), st);
    NFA_CHECK_LAUNCH();
  }
  return NFA_OK;
}
