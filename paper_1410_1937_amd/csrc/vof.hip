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
//   k_planes  one thread per cell of a compact list of the active cells with
//             1e-12 < phi < 1 - 1e-12: normal, bisection, the plane stored
//             in a per-cell table (signed normal, constant);
//   k_sweep   one thread per cell, x fastest: face speeds, the two face
//             fluxes (reading the upwind cell's plane from the table), the
//             update; it appends the cells it leaves inside (1e-12, 1 - 1e-12)
//             to the list of the next sweep.
// The first list comes from k_scan.  Appends are staged in LDS and flushed
// with one global atomic per block and flush.  Blocks take grid rows
// (x-lines) round robin.
//
// Built with -ffp-contract=off: every expression is rounded as written.
#include <cmath>

#include "device_util.h"
#include "nfa_internal.h"

namespace nfa {
namespace {

constexpr int kBisect = 64;
constexpr double kEps = 1e-12;   // fractions within kEps of 0 or 1 have no plane
constexpr int kPlaneBlocks = 2048;
constexpr int kRowBlocks = 4096;   // blocks of the row kernels
constexpr int kStage = 2048;       // LDS list entries per block

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
// lower) d-face of cell (i, j, k).
__device__ double slab_water(const Sweep& A, const double4* __restrict__ planes, int d, int i, int j, int k,
                             bool upper, double speed) {
  const double dims[3] = {A.dx[i], A.dy[j], A.dz[k]};
  const double dw = dims[d];
  const double frac = fmin(speed * A.dt, dw) / dw;
  const double vol = (A.dz[k] * A.dy[j]) * A.dx[i];
  const double slab = frac * vol;
  const long long c = cell(A, i, j, k);
  const double phi = A.phi[c];
  if (!in_band(phi)) return slab * clip01(phi);
  const double4 P = planes[c];
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

// Face velocities uhat of cell (i, j, k) on its lower and upper d-faces.
__device__ void face_speeds(const Sweep& A, int d, int i, int j, int k, double& lo, double& up) {
  const int nx = A.nx, ny = A.ny;
  const long long fxm = ((long long)k * ny + j) * (nx + 1) + i;
  const long long fym = ((long long)k * (ny + 1) + j) * nx + i;
  const long long fzm = ((long long)k * ny + j) * nx + i;
  const long long plane = (long long)nx * ny;
  const double V = (A.dz[k] * A.dy[j]) * A.dx[i];
  if (d == 0) {
    lo = (A.dx[i] * (A.ox[fxm] * A.u[fxm])) / V;
    up = (A.dx[i] * (A.ox[fxm + 1] * A.u[fxm + 1])) / V;
  } else if (d == 1) {
    lo = (A.dy[j] * (A.oy[fym] * A.v[fym])) / V;
    up = (A.dy[j] * (A.oy[fym + nx] * A.v[fym + nx])) / V;
  } else {
    const double Fxm = A.ox[fxm] * A.u[fxm], Fxp = A.ox[fxm + 1] * A.u[fxm + 1];
    const double Fym = A.oy[fym] * A.v[fym], Fyp = A.oy[fym + nx] * A.v[fym + nx];
    const double Azm = A.oz[fzm], Azp = A.oz[fzm + plane];
    double Fzm = Azm * A.w[fzm], Fzp = Azp * A.w[fzm + plane];
    const double E = ((Fxp - Fxm) + (Fyp - Fym)) + (Fzp - Fzm);
    const double den = Azp + Azm;
    if (den > 0.0) {
      Fzp = Fzp - (E * Azp) / den;
      Fzm = Fzm + (E * Azm) / den;
    }
    lo = (A.dz[k] * Fzm) / V;
    up = (A.dz[k] * Fzp) / V;
  }
}

// A list staged in LDS (s_list, kStage entries): appended by wavefronts
// (one LDS atomic each), flushed to the global list with one global atomic
// per flush.  Every lane of the block must call these.
struct Stage {
  int cnt;
  int base;
};

__device__ __forceinline__ void stage_append(int* s_list, Stage& S, bool flag, int c) {
  const unsigned long long mask = __ballot(flag);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  int b = 0;
  if (lane == leader) b = atomicAdd(&S.cnt, __popcll(mask));
  b = __shfl(b, leader, 64);
  if (flag) s_list[b + __popcll(mask & ((1ull << lane) - 1ull))] = c;
}

// Flushes when forced or when the next chunk of blockDim appends might not fit.
__device__ __forceinline__ void stage_flush(const int* s_list, Stage& S, int* __restrict__ list, int* counter,
                                            bool force) {
  __syncthreads();
  const int m = S.cnt;
  __syncthreads();   // every thread has read S.cnt before the next append changes it
  if (m == 0 || (!force && m <= kStage - (int)blockDim.x)) return;
  if (threadIdx.x == 0) S.base = atomicAdd(counter, m);
  __syncthreads();
  const int base = S.base;
  for (int e = threadIdx.x; e < m; e += blockDim.x) list[base + e] = s_list[e];
  __syncthreads();
  if (threadIdx.x == 0) S.cnt = 0;
  __syncthreads();
}

// Rows (x-lines, row r = k ny + j) are dealt to blocks round robin, so the
// free surface's band of rows spreads over every block and XCD; the logical
// block order is remapped so that the blocks of one XCD take neighbouring
// rows.
__device__ __forceinline__ int first_row() { return xcd_remap(blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(64) void k_reset(int* counters) {
  if (threadIdx.x < 2) counters[threadIdx.x] = 0;
}

// The in-band active cells of phi.
__global__ __launch_bounds__(kBlock) void k_scan(int nx, int nrows, const double* __restrict__ phi,
                                                 const unsigned char* __restrict__ act, int* __restrict__ list,
                                                 int* counter) {
  __shared__ int s_list[kStage];
  __shared__ Stage S;
  if (threadIdx.x == 0) S.cnt = 0;
  __syncthreads();
  for (int r = first_row(); r < nrows; r += gridDim.x) {
    const long long row = (long long)r * nx;
    for (int i0 = 0; i0 < nx; i0 += blockDim.x) {
      const int i = i0 + threadIdx.x;
      const long long c = row + i;
      const bool f = i < nx && act[c] && in_band(phi[c]);
      stage_append(s_list, S, f, (int)c);
      stage_flush(s_list, S, list, counter, false);
    }
  }
  stage_flush(s_list, S, list, counter, true);
}

// Planes of the listed cells; also clears the counter of the next list.
__global__ __launch_bounds__(kBlock) void k_planes(Sweep A, const int* __restrict__ list, const int* count,
                                                   double4* __restrict__ planes, int* next_counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *next_counter = 0;
  const int m = *count;
  const unsigned nx = A.nx, ny = A.ny;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    const unsigned c = list[e];
    const unsigned r = c / nx;
    const int i = (int)(c - r * nx);
    const int k = (int)(r / ny);
    const int j = (int)(r - (unsigned)k * ny);
    planes[c] = make_plane(A, i, j, k, A.phi[c]);
  }
}

template <int D, bool IMPLICIT, bool APPEND>
__global__ __launch_bounds__(kBlock) void k_sweep(Sweep A, const double4* __restrict__ planes,
                                                  int* __restrict__ list, int* counter) {
  __shared__ int s_list[APPEND ? kStage : 1];
  __shared__ Stage S;
  if (APPEND) {
    if (threadIdx.x == 0) S.cnt = 0;
    __syncthreads();
  }
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  for (int r = first_row(); r < ny * nz; r += gridDim.x) {
    const int k = r / ny, j = r - k * ny;
    const long long row = (long long)r * nx;
    for (int i0 = 0; i0 < nx; i0 += blockDim.x) {
      const int i = i0 + threadIdx.x;
      const long long c = row + i;
      bool listed = false;
      if (i < nx) {
        const double phi = A.phi[c];
        if (!A.act[c]) {
          A.out[c] = phi;
        } else {
          double lo, up;
          face_speeds(A, D, i, j, k, lo, up);
          // the neighbours along D (a face on the domain boundary draws from the cell itself)
          const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
          const int pos = D == 0 ? i : (D == 1 ? j : k);
          const int pm = pos > 0 ? pos - 1 : pos, pp = pos < nD - 1 ? pos + 1 : pos;
          const int im = D == 0 ? pm : i, jm = D == 1 ? pm : j, km = D == 2 ? pm : k;
          const int ip = D == 0 ? pp : i, jp = D == 1 ? pp : j, kp = D == 2 ? pp : k;
          double f_up, f_lo;
          if (up > 0.0) f_up = slab_water(A, planes, D, i, j, k, true, up);
          else if (up < 0.0) f_up = -slab_water(A, planes, D, ip, jp, kp, false, -up);
          else f_up = 0.0;
          if (lo > 0.0) f_lo = slab_water(A, planes, D, im, jm, km, true, lo);
          else if (lo < 0.0) f_lo = -slab_water(A, planes, D, i, j, k, false, -lo);
          else f_lo = 0.0;
          const double width = D == 0 ? A.dx[i] : (D == 1 ? A.dy[j] : A.dz[k]);
          const double V = (A.dz[k] * A.dy[j]) * A.dx[i];
          const double div = (up - lo) / width;
          const double rest = phi - (f_up - f_lo) / V;
          const double nw = IMPLICIT ? rest / (1.0 - A.dt * div) : rest + (A.dt * phi) * div;
          A.out[c] = nw;
          listed = in_band(nw);
        }
      }
      if (APPEND) {
        stage_append(s_list, S, listed, (int)c);
        stage_flush(s_list, S, list, counter, false);
      }
    }
  }
  if (APPEND) stage_flush(s_list, S, list, counter, true);
}

void launch_sweep(const Sweep& A, int d, bool implicit, bool append_next, const double4* planes, int* list,
                  int* counter, hipStream_t s) {
  const int nb = std::min(kRowBlocks, A.ny * A.nz);
#define NFA_SWEEP(D, I, P) k_sweep<D, I, P><<<nb, kBlock, 0, s>>>(A, planes, list, counter)
  if (append_next) {
    if (d == 0) { if (implicit) NFA_SWEEP(0, true, true); else NFA_SWEEP(0, false, true); }
    else if (d == 1) { if (implicit) NFA_SWEEP(1, true, true); else NFA_SWEEP(1, false, true); }
    else { if (implicit) NFA_SWEEP(2, true, true); else NFA_SWEEP(2, false, true); }
  } else {
    if (d == 0) { if (implicit) NFA_SWEEP(0, true, false); else NFA_SWEEP(0, false, false); }
    else if (d == 1) { if (implicit) NFA_SWEEP(1, true, false); else NFA_SWEEP(1, false, false); }
    else { if (implicit) NFA_SWEEP(2, true, false); else NFA_SWEEP(2, false, false); }
  }
#undef NFA_SWEEP
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

// Work memory of the advection: the plane table, two cell lists, their
// counters and one fraction buffer.
struct nfa_vof_s {
  nfa::Grid* g = nullptr;
  nfa::DevBuf planes;    // double4 per cell
  nfa::DevBuf lists;     // 2 x int32 per cell
  nfa::DevBuf counters;  // 2 x int32
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
  if ((e = v->planes.alloc(n * sizeof(double4))) != hipSuccess || (e = v->lists.alloc(2 * n * 4)) != hipSuccess ||
      (e = v->counters.alloc(256)) != hipSuccess || (e = v->work.alloc(n * 8)) != hipSuccess) {
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

// Lists and planes of the sweeps: list 0 and counter 0 hold the cells of
// phi, the sweep appends those of its output to list 1 and counter 1.
struct Work {
  double4* planes;
  int* list[2];
  int* count[2];
};

Work work_of(nfa_vof v) {
  Work W;
  W.planes = v->planes.as<double4>();
  W.list[0] = v->lists.as<int>();
  W.list[1] = v->lists.as<int>() + v->g->n;
  W.count[0] = v->counters.as<int>();
  W.count[1] = v->counters.as<int>() + 1;
  return W;
}

}  // namespace

extern "C" nfa_status nfa_vof_sweep(nfa_vof vf, const double* phi, const double* u, const double* v,
                                    const double* w, double dt, int dir, int implicit, double* phi_out,
                                    nfa_stream s) {
  nfa_status e = check("nfa_vof_sweep", vf, phi, u, v, w, dt, phi_out);
  if (e != NFA_OK) return e;
  if (dir < 0 || dir > 2) return fail(NFA_ERR_INVALID, "nfa_vof_sweep: dir must be 0, 1 or 2");
  const Grid& g = *vf->g;
  const hipStream_t st = S(s);
  Work W = work_of(vf);
  Sweep A = make_sweep(g, u, v, w, dt);
  A.phi = phi;
  A.out = phi_out;
  k_reset<<<1, 64, 0, st>>>(W.count[0]);
  k_scan<<<std::min(kRowBlocks, g.ny * g.nz), kBlock, 0, st>>>(g.nx, g.ny * g.nz, phi, g.active.as<unsigned char>(),
                                                               W.list[0], W.count[0]);
  k_planes<<<kPlaneBlocks, kBlock, 0, st>>>(A, W.list[0], W.count[0], W.planes, W.count[1]);
  launch_sweep(A, dir, implicit != 0, false, W.planes, nullptr, nullptr, st);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_vof_advect(nfa_vof vf, const double* phi, const double* u, const double* v,
                                     const double* w, double dt, int step, double* phi_out, nfa_stream s) {
  nfa_status e = check("nfa_vof_advect", vf, phi, u, v, w, dt, phi_out);
  if (e != NFA_OK) return e;
  const Grid& g = *vf->g;
  const hipStream_t st = S(s);
  Work W = work_of(vf);
  double* work = vf->work.as<double>();
  const int order[2][3] = {{0, 1, 2}, {2, 1, 0}};
  const int* o = order[step % 2 == 0 ? 0 : 1];
  // phi -> phi_out -> work -> phi_out; the lists alternate 0, 1, 0
  const double* src[3] = {phi, phi_out, work};
  double* dst[3] = {phi_out, work, phi_out};
  Sweep A = make_sweep(g, u, v, w, dt);
  k_reset<<<1, 64, 0, st>>>(W.count[0]);
  k_scan<<<std::min(kRowBlocks, g.ny * g.nz), kBlock, 0, st>>>(g.nx, g.ny * g.nz, phi, g.active.as<unsigned char>(),
                                                               W.list[0], W.count[0]);
  for (int p = 0; p < 3; ++p) {
    const int cur = p & 1, nxt = cur ^ 1;
    A.phi = src[p];
    A.out = dst[p];
    k_planes<<<kPlaneBlocks, kBlock, 0, st>>>(A, W.list[cur], W.count[cur], W.planes, W.count[nxt]);
    launch_sweep(A, o[p], p == 2, p < 2, W.planes, W.list[nxt], W.count[nxt], st);
    NFA_CHECK_LAUNCH();
  }
  return NFA_OK;
}
