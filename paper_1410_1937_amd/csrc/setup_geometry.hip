// libnfa: set-up geometry -- the one-dimensional grid stretching of the
// Gridding section (eq. grid) and the signed distance psi of a triangulated
// body surface (Enforcement of Body Boundary Conditions section).
//
// Stretching runs on the host: a 1-D tridiagonal iteration over at most a
// few thousand nodes has no parallel work to give a GPU.  The conservative
// form w(m_{i+1/2}) (x_{i+1} - x_i) = w(m_{i-1/2}) (x_i - x_{i-1}) (m the
// midpoints) is iterated Picard-style: weights frozen at the current
// midpoints, the interior nodes solved exactly (Thomas algorithm; the matrix
// is symmetric, positive definite and weakly diagonally dominant).
//
// The signed distance runs on the GPU, one thread per grid node in bricks of
// 8 x 8 x 4 nodes, the panels sorted along a Morton curve of their centroids
// and streamed through LDS in tiles of 128 (each block derives a tile's edge
// vectors and normal once).  A brick skips a whole tile when the tile's box
// is farther from the brick's box than an upper bound of every node's
// distance (the nearest sub-tile vertex), unless the brick meets the panels'
// bounding box, where every node needs every tile's solid angle; a node
// skips each 32-panel sub-tile whose box is farther than its best distance
// so far, which starts at its own bound.  Per node:
//   - the least squared distance to the panels: to the foot of the
//     perpendicular when it falls inside the triangle, else to the nearest
//     of its three edges; a tile whose bounding box is farther than the best
//     distance so far is skipped (it cannot hold the minimum);
//   - inside or outside by Gauss's theorem on the solid angle: the panels of
//     a closed surface subtend 4 pi at an inside point and 0 outside (Van
//     Oosterom and Strackee's closed form per triangle); a node outside the
//     mesh's bounding box is outside and skips the sum.
// psi = -sqrt(d2) inside, +sqrt(d2) outside, in FP64.
//
// Built with -ffp-contract=off; the signed-distance kernel alone allows FMA
// contraction.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "nfa_internal.h"

namespace nfa {
namespace {

// ------------------------------------------------------------ stretching
double stretch_weight(double x, int nz, const double* lv, const double* zn) {
  double w = lv[0];
  for (int k = 0; k < nz; ++k) {
    const double x0 = zn[2 * k], x1 = zn[2 * k + 1], wa = lv[k], wb = lv[k + 1];
    if (x < x0) continue;
    if (x <= x1) {
      const double t = (M_PI * (x - x0)) / (x1 - x0);
      w = ((wa - wb) / 2.0) * (1.0 + std::cos(t)) + wb;
    } else {
      w = wb;
    }
  }
  return w;
}

// ------------------------------------------------------- signed distance
constexpr int kPsiBlock = 256;
constexpr int kTile = 128;
constexpr int kSub = 32;        // panels per culling sub-tile (kTile / kSub per tile)

struct Box {
  double lo[3], hi[3];
};

// Bounding box of all panel vertices (one block).
__global__ __launch_bounds__(kPsiBlock) void k_panel_box(const double* __restrict__ tri, long long m, Box* out) {
  __shared__ double s_lo[3][kPsiBlock], s_hi[3][kPsiBlock];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (long long v = threadIdx.x; v < 3 * m; v += blockDim.x)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double c = tri[3 * v + d];
      lo[d] = fmin(lo[d], c);
      hi[d] = fmax(hi[d], c);
    }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    s_lo[d][threadIdx.x] = lo[d];
    s_hi[d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    double l = INFINITY, h = -INFINITY;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      l = fmin(l, s_lo[d][t]);
      h = fmax(h, s_hi[d][t]);
    }
    out->lo[d] = l;
    out->hi[d] = h;
  }
}

__device__ __forceinline__ double seg_d2(double qx, double qy, double qz, double ex, double ey, double ez,
                                         double inv_l2) {
  double t = ((qx * ex + qy * ey) + qz * ez) * inv_l2;
  t = fmin(fmax(t, 0.0), 1.0);
  const double dx = qx - t * ex, dy = qy - t * ey, dz = qz - t * ez;
  return (dx * dx + dy * dy) + dz * dz;
}

// Bounding box of each sub-tile of kSub consecutive (sorted) panels.
__global__ __launch_bounds__(kPsiBlock) void k_tile_boxes(const double* __restrict__ tri, int m, Box* __restrict__ out) {
  const int ntiles = (m + kSub - 1) / kSub;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    Box B;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      B.lo[d] = INFINITY;
      B.hi[d] = -INFINITY;
    }
    const int p1 = min(m, (t + 1) * kSub);
    for (int p = t * kSub; p < p1; ++p)
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double c = tri[9LL * p + 3 * v + d];
          B.lo[d] = fmin(B.lo[d], c);
          B.hi[d] = fmax(B.hi[d], c);
        }
    out[t] = B;
  }
}

// Node bricks of 8 x 8 x 4.
constexpr int kBx = 8, kBy = 8, kBz = 4;

__global__ __launch_bounds__(kPsiBlock) void k_psi(int nx1, int ny1, int nz1, const double* __restrict__ xf,
                                                   const double* __restrict__ yf, const double* __restrict__ zf,
                                                   const double* __restrict__ tri, int m,
                                                   const Box* __restrict__ subs, const Box* __restrict__ box,
                                                   double* __restrict__ psi) {
  // psi is held to the oracle by tolerance, not bitwise, so products and
  // sums may fuse into FMAs here (the library is otherwise built without)
#pragma clang fp contract(fast)
  // tile of panels: vertices, edge vectors, scaled in-plane coordinate
  // vectors u1 = (e1 x n)/|n|^2, u2 = (n x e0)/|n|^2, normal, 1/|n|^2 and
  // the inverse squared edge lengths
  __shared__ double s_a[3][kTile], s_b[3][kTile], s_c[3][kTile], s_e0[3][kTile], s_e1[3][kTile], s_e2[3][kTile];
  __shared__ double s_u1[3][kTile], s_u2[3][kTile], s_n[3][kTile], s_inn[kTile], s_il[3][kTile];
  __shared__ double s_red[kPsiBlock];
  const int nbx = (nx1 + kBx - 1) / kBx, nby = (ny1 + kBy - 1) / kBy;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
  const int i = bx * kBx + threadIdx.x % kBx, j = by * kBy + (threadIdx.x / kBx) % kBy,
            k = bz * kBz + threadIdx.x / (kBx * kBy);
  const bool valid = i < nx1 && j < ny1 && k < nz1;
  const double px = xf[min(i, nx1 - 1)], py = yf[min(j, ny1 - 1)], pz = zf[min(k, nz1 - 1)];
  // the brick's box
  const double blo[3] = {xf[bx * kBx], yf[by * kBy], zf[bz * kBz]};
  const double bhi[3] = {xf[min(bx * kBx + kBx - 1, nx1 - 1)], yf[min(by * kBy + kBy - 1, ny1 - 1)],
                         zf[min(bz * kBz + kBz - 1, nz1 - 1)]};
  const bool maybe_inside = px >= box->lo[0] && px <= box->hi[0] && py >= box->lo[1] && py <= box->hi[1] &&
                            pz >= box->lo[2] && pz <= box->hi[2];
  bool brick_meets_box = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) brick_meets_box = brick_meets_box && bhi[d] >= box->lo[d] && blo[d] <= box->hi[d];
  const int ntiles = (m + kTile - 1) / kTile, nsubs = (m + kSub - 1) / kSub;
  // an upper bound of each node's distance: the nearest of the sub-tiles'
  // first vertices (all on the surface); the brick takes the largest
  double ub = INFINITY;
  for (int t = 0; t < nsubs; ++t) {
    const double* v = tri + 9LL * t * kSub;
    const double dx = px - v[0], dy = py - v[1], dz = pz - v[2];
    ub = fmin(ub, (dx * dx + dy * dy) + dz * dz);
  }
  s_red[threadIdx.x] = valid ? ub : 0.0;
  __syncthreads();
  for (int w = kPsiBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_red[threadIdx.x] = fmax(s_red[threadIdx.x], s_red[threadIdx.x + w]);
    __syncthreads();
  }
  const double brick_ub = s_red[0];
  // the node's own bound starts its running minimum: the tile holding the
  // true minimum is never culled (its box is no farther than that minimum)
  double best = ub, omega = 0.0;
  for (int tile = 0; tile < ntiles; ++tile) {
    const int s0 = tile * (kTile / kSub), s1 = min(nsubs, s0 + kTile / kSub);
    Box T = subs[s0];
    for (int u = s0 + 1; u < s1; ++u) {
      const Box U = subs[u];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        T.lo[d] = fmin(T.lo[d], U.lo[d]);
        T.hi[d] = fmax(T.hi[d], U.hi[d]);
      }
    }
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double gap = fmax(fmax(T.lo[d] - bhi[d], 0.0), blo[d] - T.hi[d]);
      g2 = g2 + gap * gap;
    }
    // no node of the brick can have its minimum in this tile, and no node
    // needs the tile's solid angle: skip it (a uniform branch)
    if (g2 > brick_ub && !brick_meets_box) continue;
    const int t0 = tile * kTile;
    const int nt = min(kTile, m - t0);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const double* P = tri + 9LL * (t0 + t);
      double a[3], b[3], c[3], e0[3], e1[3], n[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        a[d] = P[d];
        b[d] = P[3 + d];
        c[d] = P[6 + d];
        e0[d] = b[d] - a[d];
        e1[d] = c[d] - a[d];
      }
      n[0] = e0[1] * e1[2] - e0[2] * e1[1];
      n[1] = e0[2] * e1[0] - e0[0] * e1[2];
      n[2] = e0[0] * e1[1] - e0[1] * e1[0];
      const double n2 = (n[0] * n[0] + n[1] * n[1]) + n[2] * n[2];
      const double inn = n2 > 0.0 ? 1.0 / n2 : 0.0;
      const double u1[3] = {(e1[1] * n[2] - e1[2] * n[1]) * inn, (e1[2] * n[0] - e1[0] * n[2]) * inn,
                            (e1[0] * n[1] - e1[1] * n[0]) * inn};
      const double u2[3] = {(n[1] * e0[2] - n[2] * e0[1]) * inn, (n[2] * e0[0] - n[0] * e0[2]) * inn,
                            (n[0] * e0[1] - n[1] * e0[0]) * inn};
      const double e2[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
      const double l0 = (e0[0] * e0[0] + e0[1] * e0[1]) + e0[2] * e0[2];
      const double l1 = (e2[0] * e2[0] + e2[1] * e2[1]) + e2[2] * e2[2];
      const double l2 = (e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        s_a[d][t] = a[d];
        s_b[d][t] = b[d];
        s_c[d][t] = c[d];
        s_e0[d][t] = e0[d];
        s_e1[d][t] = e1[d];
        s_e2[d][t] = e2[d];
        s_u1[d][t] = u1[d];
        s_u2[d][t] = u2[d];
        s_n[d][t] = n[d];
      }
      s_inn[t] = n2 > 0.0 ? inn : -1.0;   // -1: degenerate, edges only
      s_il[0][t] = l0 > 0.0 ? 1.0 / l0 : 0.0;
      s_il[1][t] = l1 > 0.0 ? 1.0 / l1 : 0.0;
      s_il[2][t] = l2 > 0.0 ? 1.0 / l2 : 0.0;
    }
    __syncthreads();
    if (!valid) continue;
    // distance: skip a sub-tile when its box is farther than this node's best
    for (int u = s0; u < s1; ++u) {
      const Box U = subs[u];
      const double gx = fmax(fmax(U.lo[0] - px, 0.0), px - U.hi[0]);
      const double gy = fmax(fmax(U.lo[1] - py, 0.0), py - U.hi[1]);
      const double gz = fmax(fmax(U.lo[2] - pz, 0.0), pz - U.hi[2]);
      const double box_d2 = (gx * gx + gy * gy) + gz * gz;
      if (box_d2 > best) continue;
      const int ta = (u - s0) * kSub, tb = min(nt, ta + kSub);
      for (int t = ta; t < tb; ++t) {
        const double ax = px - s_a[0][t], ay = py - s_a[1][t], az = pz - s_a[2][t];
        const double inn = s_inn[t];
        double d2;
        const double s = (ax * s_u1[0][t] + ay * s_u1[1][t]) + az * s_u1[2][t];
        const double tt = (ax * s_u2[0][t] + ay * s_u2[1][t]) + az * s_u2[2][t];
        if (inn > 0.0 && s >= 0.0 && tt >= 0.0 && s + tt <= 1.0) {
          const double pn = (ax * s_n[0][t] + ay * s_n[1][t]) + az * s_n[2][t];
          d2 = (pn * pn) * inn;
        } else {
          const double bx2 = px - s_b[0][t], by2 = py - s_b[1][t], bz2 = pz - s_b[2][t];
          const double d0 = seg_d2(ax, ay, az, s_e0[0][t], s_e0[1][t], s_e0[2][t], s_il[0][t]);
          const double d1 = seg_d2(bx2, by2, bz2, s_e2[0][t], s_e2[1][t], s_e2[2][t], s_il[1][t]);
          // edge c -> a: from c, direction -e1
          const double cx = px - s_c[0][t], cy = py - s_c[1][t], cz = pz - s_c[2][t];
          const double d3 = seg_d2(cx, cy, cz, -s_e1[0][t], -s_e1[1][t], -s_e1[2][t], s_il[2][t]);
          d2 = fmin(fmin(d0, d1), d3);
        }
        best = fmin(best, d2);
      }
    }
    if (maybe_inside) {
      for (int t = 0; t < nt; ++t) {
        const double rax = s_a[0][t] - px, ray = s_a[1][t] - py, raz = s_a[2][t] - pz;
        const double rbx = s_b[0][t] - px, rby = s_b[1][t] - py, rbz = s_b[2][t] - pz;
        const double rcx = s_c[0][t] - px, rcy = s_c[1][t] - py, rcz = s_c[2][t] - pz;
        const double la = sqrt((rax * rax + ray * ray) + raz * raz);
        const double lb = sqrt((rbx * rbx + rby * rby) + rbz * rbz);
        const double lc = sqrt((rcx * rcx + rcy * rcy) + rcz * rcz);
        const double num = (rax * (rby * rcz - rbz * rcy) + ray * (rbz * rcx - rbx * rcz)) +
                           raz * (rbx * rcy - rby * rcx);
        const double ab = (rax * rbx + ray * rby) + raz * rbz;
        const double ac = (rax * rcx + ray * rcy) + raz * rcz;
        const double bc = (rbx * rcx + rby * rcy) + rbz * rcz;
        const double den = ((la * lb * lc + ab * lc) + ac * lb) + bc * la;
        omega += 2.0 * atan2(num, den);
      }
    }
  }
  if (valid) {
    const double d = sqrt(best);
    psi[((long long)k * ny1 + j) * nx1 + i] = fabs(omega) > 2.0 * M_PI ? -d : d;
  }
}

// Panels reordered along a Morton curve of their centroids, so that a tile
// of consecutive panels is compact and its bounding box culls well.
std::vector<double> morton_order(const std::vector<double>& t, long long m) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  std::vector<double> cen(3 * m);
  for (long long p = 0; p < m; ++p)
    for (int d = 0; d < 3; ++d) {
      const double c = (t[9 * p + d] + t[9 * p + 3 + d] + t[9 * p + 6 + d]) / 3.0;
      cen[3 * p + d] = c;
      lo[d] = std::fmin(lo[d], c);
      hi[d] = std::fmax(hi[d], c);
    }
  std::vector<std::pair<unsigned long long, long long>> key(m);
  for (long long p = 0; p < m; ++p) {
    unsigned long long code = 0;
    unsigned q[3];
    for (int d = 0; d < 3; ++d) {
      const double span = hi[d] - lo[d];
      const double u = span > 0 ? (cen[3 * p + d] - lo[d]) / span : 0.0;
      q[d] = (unsigned)std::fmin(std::fmax(u * 2097151.0, 0.0), 2097151.0);
    }
    for (int b = 20; b >= 0; --b)
      for (int d = 0; d < 3; ++d) code = (code << 1) | ((q[d] >> b) & 1u);
    key[p] = {code, p};
  }
  std::sort(key.begin(), key.end());
  std::vector<double> out(9 * m);
  for (long long p = 0; p < m; ++p)
    for (int v = 0; v < 9; ++v) out[9 * p + v] = t[9 * key[p].second + v];
  return out;
}

// Work memory of nfa_panels_psi_noalloc, one copy per device for the life
// of the process: the panels' bounding box, the sub-tile boxes and the
// Morton-sorted panels of at most kScratchPanels panels.  The array's name is
// a host-side stand-in in host code: kernels receive the device address
// hipGetSymbolAddress gives for it (scratch_base), never the name.
constexpr long long kScratchPanels = 1LL << 16;
constexpr size_t kScratchBoxOff = 0;
constexpr size_t kScratchTileOff = 256;
constexpr size_t kScratchTriOff =
    kScratchTileOff + ((sizeof(Box) * (kScratchPanels / kSub) + 255) / 256) * 256;
constexpr size_t kScratchBytes = kScratchTriOff + 9 * sizeof(double) * kScratchPanels;

}  // namespace
}  // namespace nfa

using namespace nfa;

static __device__ __align__(256) unsigned char scratch[nfa::kScratchBytes];

extern "C" nfa_status nfa_stretch_axis(double a, double b, int n, int nzones, const double* levels,
                                       const double* zones, double tol, int max_iter, double* nodes,
                                       int* iterations) {
  if (!nodes || !levels || (nzones > 0 && !zones) || !iterations)
    return fail(NFA_ERR_INVALID, "nfa_stretch_axis: NULL argument");
  if (n < 1 || nzones < 0 || !(a < b) || !std::isfinite(a) || !std::isfinite(b) || !(tol > 0) || max_iter < 1)
    return fail(NFA_ERR_INVALID, "nfa_stretch_axis: needs n >= 1, finite a < b, tol > 0, max_iter >= 1");
  for (int k = 0; k <= nzones; ++k)
    if (!(levels[k] > 0) || !std::isfinite(levels[k]))
      return fail(NFA_ERR_INVALID, "nfa_stretch_axis: weight levels must be finite and > 0");
  for (int k = 0; k < nzones; ++k)
    if (!(zones[2 * k] < zones[2 * k + 1]) || !std::isfinite(zones[2 * k]) || !std::isfinite(zones[2 * k + 1]) ||
        (k > 0 && zones[2 * k] < zones[2 * k - 1]))
      return fail(NFA_ERR_INVALID, "nfa_stretch_axis: transition zones must be increasing and not overlap");
  std::vector<double> x(n + 1), xn(n + 1), wm(n), cp(n), dp(n);
  for (int i = 0; i <= n; ++i) x[i] = a + ((b - a) * i) / n;
  for (int it = 1; it <= max_iter; ++it) {
    for (int i = 0; i < n; ++i) wm[i] = stretch_weight(0.5 * (x[i] + x[i + 1]), nzones, levels, zones);
    if (n == 1) {
      for (int i = 0; i <= n; ++i) nodes[i] = x[i];
      *iterations = it;
      return NFA_OK;
    }
    // rows r = 0..n-2 for node r+1: -wm[r] x[r] + (wm[r] + wm[r+1]) x[r+1] - wm[r+1] x[r+2] = 0
    const int rows = n - 1;
    for (int r = 0; r < rows; ++r) {
      const double sub = r > 0 ? -wm[r] : 0.0, diag = wm[r] + wm[r + 1], sup = -wm[r + 1];
      double rhs = 0.0;
      if (r == 0) rhs += wm[0] * a;
      if (r == rows - 1) rhs += wm[n - 1] * b;
      const double den = r > 0 ? diag - sub * cp[r - 1] : diag;
      cp[r] = sup / den;
      dp[r] = (r > 0 ? rhs - sub * dp[r - 1] : rhs) / den;
    }
    xn[0] = a;
    xn[n] = b;
    xn[rows] = dp[rows - 1];
    for (int r = rows - 2; r >= 0; --r) xn[r + 1] = dp[r] - cp[r] * xn[r + 2];
    double moved = 0.0;
    for (int i = 0; i <= n; ++i) moved = std::fmax(moved, std::fabs(xn[i] - x[i]));
    x.swap(xn);
    if (moved <= tol * (b - a)) {
      for (int i = 0; i <= n; ++i) nodes[i] = x[i];
      *iterations = it;
      return NFA_OK;
    }
  }
  for (int i = 0; i <= n; ++i) nodes[i] = x[i];
  *iterations = max_iter;
  return NFA_NOT_CONVERGED;
}

namespace nfa {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// with that device current.
nfa_status scratch_base(void** out) {
  int dev = 0;
  NFA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NFA_ERR_INVALID, "nfa_panels_psi_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    NFA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(NFA_ERR_HIP, "nfa_panels_psi_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NFA_OK;
}

nfa_status psi_check(nfa_grid g, const double* panels, long long m, double* psi, const char* who) {
  if (!g || !psi || (m > 0 && !panels)) return fail(NFA_ERR_INVALID, std::string(who) + ": NULL argument");
  if (m < 1 || m > (1LL << 30)) return fail(NFA_ERR_INVALID, std::string(who) + ": needs 1 <= m <= 2^30 panels");
  return NFA_OK;
}

// The panels in Morton order of their centroids, read back from the device.
nfa_status psi_sorted_panels(const double* panels, long long m, hipStream_t st, std::vector<double>& sorted) {
  std::vector<double> host(9 * m);
  NFA_HIP(hipMemcpyAsync(host.data(), panels, 9 * m * sizeof(double), hipMemcpyDeviceToHost, st));
  NFA_HIP(hipStreamSynchronize(st));
  sorted = morton_order(host, m);
  return NFA_OK;
}

// Uploads the sorted panels into tri and runs the three kernels; returns once
// the stream has finished them.
nfa_status psi_run(const Grid& g, const std::vector<double>& sorted, long long m, double* tri, Box* box, Box* tiles,
                   double* psi, hipStream_t st) {
  NFA_HIP(hipMemcpyAsync(tri, sorted.data(), 9 * m * sizeof(double), hipMemcpyHostToDevice, st));
  k_panel_box<<<1, kPsiBlock, 0, st>>>(tri, m, box);
  NFA_CHECK_LAUNCH();
  const int nsubs = (int)((m + kSub - 1) / kSub);
  k_tile_boxes<<<(nsubs + kPsiBlock - 1) / kPsiBlock, kPsiBlock, 0, st>>>(tri, (int)m, tiles);
  NFA_CHECK_LAUNCH();
  const int nx1 = g.nx + 1, ny1 = g.ny + 1, nz1 = g.nz + 1;
  const long long nb = (long long)((nx1 + kBx - 1) / kBx) * ((ny1 + kBy - 1) / kBy) * ((nz1 + kBz - 1) / kBz);
  k_psi<<<(unsigned)nb, kPsiBlock, 0, st>>>(nx1, ny1, nz1, g.d_xf.as<double>(), g.d_yf.as<double>(),
                                           g.d_zf.as<double>(), tri, (int)m, tiles, box, psi);
  NFA_CHECK_LAUNCH();
  NFA_HIP(hipStreamSynchronize(st));
  return NFA_OK;
}

}  // namespace
}  // namespace nfa

extern "C" nfa_status nfa_panels_psi(nfa_grid g, const double* panels, long long m, double* psi, nfa_stream s) {
  if (const nfa_status e = psi_check(g, panels, m, psi, "nfa_panels_psi")) return e;
  const hipStream_t st = S(s);
  std::vector<double> sorted;
  if (const nfa_status e = psi_sorted_panels(panels, m, st, sorted)) return e;
  DevBuf box, tri, tiles;
  NFA_HIP(box.alloc(sizeof(Box)));
  NFA_HIP(tri.alloc(9 * m * sizeof(double)));
  NFA_HIP(tiles.alloc((size_t)((m + kSub - 1) / kSub) * sizeof(Box)));
  // the work buffers are freed on return, after the stream has finished
  return psi_run(*g, sorted, m, tri.as<double>(), box.as<Box>(), tiles.as<Box>(), psi, st);
}

extern "C" nfa_status nfa_panels_psi_noalloc(nfa_grid g, const double* panels, long long m, double* psi,
                                             nfa_stream s) {
  if (const nfa_status e = psi_check(g, panels, m, psi, "nfa_panels_psi_noalloc")) return e;
  if (m > kScratchPanels)
    return fail(NFA_ERR_INVALID, "nfa_panels_psi_noalloc: at most " + std::to_string(kScratchPanels) +
                                     " panels (the size of its static work memory); got " + std::to_string(m));
  void* base = nullptr;
  if (const nfa_status e = scratch_base(&base)) return e;
  const hipStream_t st = S(s);
  std::vector<double> sorted;
  if (const nfa_status e = psi_sorted_panels(panels, m, st, sorted)) return e;
  unsigned char* b = static_cast<unsigned char*>(base);
  // every kernel writes its part of the work memory in full before reading it
  return psi_run(*g, sorted, m, reinterpret_cast<double*>(b + kScratchTriOff),
                 reinterpret_cast<Box*>(b + kScratchBoxOff), reinterpret_cast<Box*>(b + kScratchTileOff), psi, st);
}
