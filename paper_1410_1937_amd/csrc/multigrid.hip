// libnfa: aggregation multigrid preconditioner for the projection's CG solve
// (Introduction: preconditioned conjugate gradients; the preconditioner is
// not named -- Jacobi is the default, this is the stronger option).
//
// Hierarchy (rebuilt from the FP64 coefficients after every assembly):
//   level 0  the merged operator A' over the reduced unknowns;
//   level 1  blocks of 2 x 2 x 2 cells; an unknown belongs to the block of
//            its own cell; A_1 = P^T A' P assembled face by face: a face of a
//            merge group's member whose other side belongs (through its root)
//            to another block adds T to the block's diagonal and -T to the
//            coupling with that block; a face to a block more than one away
//            (only through long merge chains) keeps its diagonal term and
//            drops the coupling; Dirichlet faces add to the diagonal;
//   level l+1  the Galerkin sum of level l's 27-point stencil over 2 x 2 x 2
//            children (exact: a 27-point stencil aggregates to 27 points);
//   coarsest  at most 600 cells (at least one coarsening): a dense FP64
//            inverse, formed on the host, with empty rows made identity rows and, when
//            every boundary is Neumann, c v v^T added (v the non-empty rows,
//            c their mean diagonal).
// Each thread assembles one coarse row, summing in a fixed order in FP64:
// the hierarchy is bitwise reproducible.  Stencils are stored structure of
// arrays, entry o = (dz+1) 9 + (dy+1) 3 + (dx+1) of cell c at [o n + c], in
// FP64 (for building the next level and for export).
//
// Cycle storage of a level l >= 1 (FP32): a Galerkin product of a 7-point
// operator over 2 x 2 x 2 blocks is again 7-point; couplings outside the
// 7 points come only from merge groups, so each cell keeps one float4
// (D^-1, a(+x), a(+y), a(+z)) -- the coupling to a lower neighbour is that
// neighbour's upper one (the operator is symmetric) -- and the rare rows with
// other couplings are flagged by a negative D^-1 and hold their 20 remaining
// entries in a side list sorted by cell (found by binary search).
//
// V-cycle in FP32, symmetric (damped Jacobi, omega = 0.9, one sweep before
// and one after the coarse correction; restriction = transpose of the
// piecewise-constant prolongation), so the solve may use it in (flexible)
// CG.  On levels >= 1 the pre-smoothed z = omega D^-1 r is never stored:
//   down   r_{l+1} = P^T (r - A z) = P^T ((1 - omega) r - omega N (D^-1 r)),
//   up     z' = z + alpha P z_{l+1};  zt = (1 - omega) z' + omega D^-1 (r - N z'),
// N the off-diagonal part (the diagonal terms cancel against D^-1 exactly in
// exact arithmetic), z' formed on the fly at each neighbour.  Rows without
// an unknown keep z' (zero coupling).  The levels from the first one with at
// most `tail` cells down run in one workgroup with their vectors in LDS,
// ending in the dense FP64 coarsest solve.
//
// Level 0 (the merged operator, read from the operator's FP32 face
// coefficients) runs as two fused sweeps that march z-columns: down forms
// omega D^-1 r, applies the operator and restricts; up prolongs, applies the
// operator, post-smooths and sums z.q for the flexible CG.  Both treat every
// cell on its own; the rows this gets wrong (roots, which carry their
// slaves' rows, and unknowns next to a slave) are corrected afterwards from
// lists built when the body is set.  Every kernel returns at once when the
// solve has converged.
//
// Built with -ffp-contract=off.
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "device_util.h"
#include "nfa_internal.h"

namespace nfa {
namespace {

constexpr int kMaxLevels = 16;
constexpr long long kMinCoarse = 600;
constexpr double kDefaultOmega = 0.9;    // damping of the Jacobi sweeps
constexpr double kDefaultAlpha = 1.0;    // scale of the coarse correction

// Cycle parameters as the kernels take them.
struct Cyc {
  float w, a;   // omega, alpha
};

struct Dims {
  int nx, ny, nz;
  long long n;
};

Dims make_dims(int nx, int ny, int nz) { return {nx, ny, nz, (long long)nx * ny * nz}; }
Dims coarser(const Dims& d) { return make_dims((d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2); }

#define MG_STRIDE(idx, n) \
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (n); idx += (long long)gridDim.x * blockDim.x)

// FP32 -> BF16, round to nearest even (the upper 16 bits of the rounded value).
__global__ void k_to_bf16(long long n, const float* __restrict__ src, unsigned short* __restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned u = __float_as_uint(src[i]);
    dst[i] = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
}

__global__ void k_fill_int(long long n, int v, int* a) {
  MG_STRIDE(i, n) a[i] = v;
}

// dst[t] = src[idx[t]]
__global__ void k_gather_int(int n, const int* __restrict__ idx, const int* __restrict__ src, int* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[idx[t]];
}

__global__ void k_group_of(int ng, const int* __restrict__ groot, int* __restrict__ group_of) {
  for (int gi = blockIdx.x * blockDim.x + threadIdx.x; gi < ng; gi += gridDim.x * blockDim.x)
    group_of[groot[gi]] = gi;
}

// The 20 stencil entries outside the 7 points (o != 4, 10, 12, 13, 14, 16, 22).
constexpr int kXSlots = 20;
__host__ __device__ constexpr int xoff(int t) {
  return t < 4 ? t : t < 9 ? t + 1 : t == 9 ? 11 : t == 10 ? 15 : t < 16 ? t + 6 : t + 7;
}
__host__ __device__ constexpr bool in7(int o) {
  return o == 4 || o == 10 || o == 12 || o == 13 || o == 14 || o == 16 || o == 22;
}

__device__ __forceinline__ void store_row(long long n, long long B, const double* acc, double* A64, float4* S) {
  bool extra = false;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    A64[o * n + B] = acc[o];
    if (!in7(o) && acc[o] != 0.0) extra = true;
  }
  const float dv = acc[13] > 0.0 ? (float)(1.0 / acc[13]) : 0.0f;
  S[B] = make_float4(extra ? -dv : dv, (float)acc[14], (float)acc[16], (float)acc[22]);
}

// Level 1 from the faces of level 0 (see the file head).
__global__ void k_level1(Dims f, Dims c, const double* __restrict__ tx, const double* __restrict__ txb,
                         const double* __restrict__ ty, const double* __restrict__ tz,
                         const unsigned char* __restrict__ reduced, const int* __restrict__ root,
                         const int* __restrict__ group_of, const int* __restrict__ g_off,
                         const int* __restrict__ g_mem, double* A64, float4* S) {
  const long long fplane = (long long)f.nx * f.ny;
  MG_STRIDE(B, c.n) {
    const int I = (int)(B % c.nx);
    const long long rr = B / c.nx;
    const int J = (int)(rr % c.ny), K = (int)(rr / c.ny);
    // acc takes the couplings whose target block is fixed by the face (a
    // neighbour that is its own root), dyn the ones through merge groups;
    // only dyn is indexed at run time, so acc stays in registers
    double acc[27], dyn[27];
    bool has_dyn = false;   // dyn is zeroed and read only when a merge touches the block
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = 0.0;
    // a face of member m (cell indices im, jm, km) to a cell whose root is rn
    auto merged_face = [&](double T, int rn) {
      if (rn < 0) return;
      const int in = rn % f.nx;
      const int rrn = rn / f.nx;
      const int jn = rrn % f.ny, kn = rrn / f.ny;
      const int dK = (kn >> 1) - K, dJ = (jn >> 1) - J, dI = (in >> 1) - I;
      if (dK == 0 && dJ == 0 && dI == 0) return;
      acc[13] += T;
      if (dK >= -1 && dK <= 1 && dJ >= -1 && dJ <= 1 && dI >= -1 && dI <= 1) {
        if (!has_dyn) {
          for (int o = 0; o < 27; ++o) dyn[o] = 0.0;
          has_dyn = true;
        }
        dyn[(dK + 1) * 9 + (dJ + 1) * 3 + (dI + 1)] -= T;
      }
    };
    auto face_of = [&](long long m, int im, int jm, int km, long long rm, int face, double& T) -> long long {
      long long nb = -1;
      if (face == 0) {
        T = tx[m];
        if (im > 0) nb = m - 1;
      } else if (face == 1) {
        T = im < f.nx - 1 ? tx[m + 1] : txb[rm];
        if (im < f.nx - 1) nb = m + 1;
      } else if (face == 2) {
        T = ty[((long long)km * (f.ny + 1) + jm) * f.nx + im];
        if (jm > 0) nb = m - f.nx;
      } else if (face == 3) {
        T = ty[((long long)km * (f.ny + 1) + jm + 1) * f.nx + im];
        if (jm < f.ny - 1) nb = m + f.nx;
      } else if (face == 4) {
        T = tz[m];
        if (km > 0) nb = m - fplane;
      } else {
        T = tz[m + fplane];
        if (km < f.nz - 1) nb = m + fplane;
      }
      return nb;
    };
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
          const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
          if (k >= f.nz || j >= f.ny || i >= f.nx) continue;
          const long long cidx = ((long long)k * f.ny + j) * f.nx + i;
          if (!reduced[cidx]) continue;
          const long long rm0 = cidx / f.nx;
#pragma unroll
          for (int face = 0; face < 6; ++face) {
            double T;
            const long long nb = face_of(cidx, i, j, k, rm0, face, T);
            if (!(T > 0.0)) continue;
            if (nb < 0) {          // a Dirichlet boundary face
              acc[13] += T;
              continue;
            }
            const int rn = root[nb];
            if (rn < 0 || (long long)rn == cidx) continue;
            if ((long long)rn == nb) {
              // the neighbour carries its own unknown: its block follows from the face
              const int dI = face == 0 ? (ii - 1) >> 1 : face == 1 ? (ii + 1) >> 1 : 0;
              const int dJ = face == 2 ? (jj - 1) >> 1 : face == 3 ? (jj + 1) >> 1 : 0;
              const int dK = face == 4 ? (kk - 1) >> 1 : face == 5 ? (kk + 1) >> 1 : 0;
              if (dK == 0 && dJ == 0 && dI == 0) continue;
              acc[13] += T;
              acc[(dK + 1) * 9 + (dJ + 1) * 3 + (dI + 1)] -= T;
            } else {
              merged_face(T, rn);
            }
          }
          // the faces of the cell's slaves, through their roots
          const int gi = group_of[cidx];
          if (gi >= 0)
            for (int e = g_off[gi]; e < g_off[gi + 1]; ++e) {
              const long long m = g_mem[e];
              const int im = (int)(m % f.nx);
              const long long rm = m / f.nx;
              const int jm = (int)(rm % f.ny), km = (int)(rm / f.ny);
              for (int face = 0; face < 6; ++face) {
                double T;
                const long long nb = face_of(m, im, jm, km, rm, face, T);
                if (!(T > 0.0)) continue;
                if (nb < 0) {
                  acc[13] += T;
                  continue;
                }
                const int rn = root[nb];
                if (rn < 0 || (long long)rn == cidx) continue;
                merged_face(T, rn);
              }
            }
        }
    if (has_dyn) {
#pragma unroll
      for (int o = 0; o < 27; ++o) acc[o] += dyn[o];
    }
    store_row(c.n, B, acc, A64, S);
  }
}

// Level l+1 as the Galerkin sum of level l's 27-point stencil.
__global__ void k_coarsen(Dims f, Dims c, const double* __restrict__ Af, double* A64, float4* S) {
  MG_STRIDE(B, c.n) {
    const int I = (int)(B % c.nx);
    const long long rr = B / c.nx;
    const int J = (int)(rr % c.ny), K = (int)(rr / c.ny);
    double acc[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = 0.0;
    // child (kk, jj, ii) and fine offset o fix the coarse offset, so every
    // index into acc is a constant once the loops are unrolled
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
          const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
          if (k >= f.nz || j >= f.ny || i >= f.nx) continue;
          const long long cidx = ((long long)k * f.ny + j) * f.nx + i;
#pragma unroll
          for (int o = 0; o < 27; ++o) {
            const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
            const int kn = k + dz, jn = j + dy, in = i + dx;
            if (kn < 0 || kn >= f.nz || jn < 0 || jn >= f.ny || in < 0 || in >= f.nx) continue;
            const double a = Af[o * f.n + cidx];
            if (a != 0.0) acc[(((kk + dz) >> 1) + 1) * 9 + (((jj + dy) >> 1) + 1) * 3 + (((ii + dx) >> 1) + 1)] += a;
          }
        }
    store_row(c.n, B, acc, A64, S);
  }
}

// ---------------------------------------------------- side list of rows
// Flagged rows per block of kBlock cells.
__global__ void k_xcount(long long n, const float4* __restrict__ S, int* cnt) {
  const long long c = blockIdx.x * (long long)kBlock + threadIdx.x;
  const int f = c < n && S[c].x < 0.0f;
  const int total = __syncthreads_count(f);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// Flagged rows in cell order: xcell[e] = c, xval[e * 20 + t] = A(c, xoff(t)).
__global__ void k_xscatter(long long n, const float4* __restrict__ S, const double* __restrict__ A64,
                           const int* __restrict__ off, int* xcell, float* xval) {
  __shared__ int wcount[kBlock / 64];
  const long long c = blockIdx.x * (long long)kBlock + threadIdx.x;
  const bool f = c < n && S[c].x < 0.0f;
  const unsigned long long ballot = __ballot(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wcount[w] = __popcll(ballot);
  __syncthreads();
  int e = off[blockIdx.x] + __popcll(ballot & ((1ull << lane) - 1ull));
  for (int q = 0; q < w; ++q) e += wcount[q];
  if (f) {
    xcell[e] = (int)c;
#pragma unroll
    for (int t = 0; t < kXSlots; ++t) xval[(long long)e * kXSlots + t] = (float)A64[xoff(t) * n + c];
  }
}

// ------------------------------------------------------------------ cycle
// One level of the cycle as the kernels see it (levels >= 1).
struct LevelView {
  int nx, ny, nz, m;            // m flagged rows
  const float4* S;
  const int* xcell;
  const float* xval;
};

// sum over the couplings of row c outside the 7 points of a * w(nb, kn, jn, in)
template <class W>
__device__ __forceinline__ float extras_sum(const LevelView& L, int c, int k, int j, int i, W w) {
  int lo = 0, hi = L.m - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (L.xcell[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  const float* v = L.xval + (long long)lo * kXSlots;
  float s = 0.0f;
#pragma unroll
  for (int t = 0; t < kXSlots; ++t) {
    const int o = xoff(t);
    const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
    const float a = v[t];
    const int kn = k + dz, jn = j + dy, in = i + dx;
    if (a == 0.0f || kn < 0 || kn >= L.nz || jn < 0 || jn >= L.ny || in < 0 || in >= L.nx) continue;
    s += a * w(c + (dz * L.ny + dy) * L.nx + dx, kn, jn, in);
  }
  return s;
}

// (N w)_c: the off-diagonal part of row c applied to the cell function w
// (x-, x+, y-, y+, z-, z+, then the side list), s4 = S[c].
template <class W>
__device__ __forceinline__ float offdiag(const LevelView& L, const float4& s4, int c, int k, int j, int i, W w) {
  const int nx = L.nx, plane = L.nx * L.ny;
  float s = 0.0f;
  if (i > 0) s += L.S[c - 1].y * w(c - 1, k, j, i - 1);
  if (i + 1 < nx) s += s4.y * w(c + 1, k, j, i + 1);
  if (j > 0) s += L.S[c - nx].z * w(c - nx, k, j - 1, i);
  if (j + 1 < L.ny) s += s4.z * w(c + nx, k, j + 1, i);
  if (k > 0) s += L.S[c - plane].w * w(c - plane, k - 1, j, i);
  if (k + 1 < L.nz) s += s4.w * w(c + plane, k + 1, j, i);
  if (s4.x < 0.0f) s += extras_sum(L, c, k, j, i, w);
  return s;
}

// Fine-cell term of the restriction: r - A z with z = omega D^-1 r.
__device__ __forceinline__ float down_value(const LevelView& L, Cyc p, const float* r, int c, int k, int j, int i) {
  const float4 s4 = L.S[c];
  const float rc = r[c];
  if (s4.x == 0.0f) return rc;
  const float n = offdiag(L, s4, c, k, j, i, [&](int nb, int, int, int) { return fabsf(L.S[nb].x) * r[nb]; });
  return (1.0f - p.w) * rc - p.w * n;
}

// Post-smoothed z of a fine cell, z' = omega D^-1 r + alpha z_{l+1}(parent).
__device__ __forceinline__ float up_value(const LevelView& L, Cyc p, const float* r, const float* zc, int cnx,
                                          int cny, int c, int k, int j, int i) {
  auto zp = [&](int nb, int kn, int jn, int in) {
    return p.w * (fabsf(L.S[nb].x) * r[nb]) + p.a * zc[((kn >> 1) * cny + (jn >> 1)) * cnx + (in >> 1)];
  };
  const float4 s4 = L.S[c];
  const float z0 = zp(c, k, j, i);
  if (s4.x == 0.0f) return z0;
  const float n = offdiag(L, s4, c, k, j, i, zp);
  return (1.0f - p.w) * z0 + p.w * (fabsf(s4.x) * (r[c] - n));
}

// Launch geometry shared by the grid-wide level kernels: a workgroup of
// 64 x 2 x 2 fine cells (x fastest), i.e. 32 coarse cells of one coarse
// row; the 8 children of a coarse cell are lanes 2I, 2I+1 of 4 wavefronts.
struct Tile {
  int i, j, k, I, J, K, lane, w;
};
__device__ __forceinline__ Tile tile_of(int tiles_x, int cny) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  Tile t;
  const int bx = blk % tiles_x, rest = blk / tiles_x;
  t.J = rest % cny;
  t.K = rest / cny;
  t.lane = threadIdx.x & 63;
  t.w = threadIdx.x >> 6;
  t.i = bx * 64 + t.lane;
  t.j = 2 * t.J + (t.w & 1);
  t.k = 2 * t.K + (t.w >> 1);
  t.I = bx * 32 + (t.lane >> 1);
  return t;
}

// rc[coarse] = sum of v over its (up to) 8 children; v in every thread.
__device__ __forceinline__ void restrict_store(const Tile& t, float v, int cnx, int cny, float* rc) {
  __shared__ float red[4][32];
  v += __shfl_xor(v, 1, 64);
  if ((t.lane & 1) == 0) red[t.w][t.lane >> 1] = v;
  __syncthreads();
  if (threadIdx.x < 32) {
    const int I = t.I - (t.lane >> 1) + threadIdx.x;   // wave 0: lane == threadIdx.x
    if (I < cnx) rc[((long long)t.K * cny + t.J) * cnx + I] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                            (red[2][threadIdx.x] + red[3][threadIdx.x]);
  }
}

// The seven cells of a fine cell's 7-point neighbourhood (x-, x+, y-, y+,
// z-, z+ and the cell), loaded up front: S and r, plus (up) the parents'
// corrections; zero beyond the domain.
template <bool UP>
struct Hood {
  float4 s[7];
  float r[7], z[7];
};
template <bool UP>
__device__ __forceinline__ void load_hood(const LevelView& L, const float* __restrict__ r, const float* __restrict__ zc,
                                          int cnx, int cny, int c, int k, int j, int i, Hood<UP>& h) {
  const int nx = L.nx, plane = L.nx * L.ny;
  const bool ok[6] = {i > 0, i + 1 < nx, j > 0, j + 1 < L.ny, k > 0, k + 1 < L.nz};
  const int off[6] = {-1, 1, -nx, nx, -plane, plane};
  const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
  // every load unconditional, so that all of them are in flight at once: a
  // neighbour beyond the domain reads the cell itself and is multiplied by 0
  // (a product the compiler may not fold, unlike a select, which it would
  // turn back into a branch around the load)
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    const bool v = f == 6 || ok[f];
    const float m = v ? 1.0f : 0.0f;
    const int nb = v && f < 6 ? c + off[f] : c;
    const float4 sv = L.S[nb];
    h.s[f] = make_float4(sv.x * m, sv.y * m, sv.z * m, sv.w * m);
    h.r[f] = r[nb] * m;
    if (UP) {
      const int kn = v && f < 6 ? k + dk[f] : k, jn = v && f < 6 ? j + dj[f] : j, in = v && f < 6 ? i + di[f] : i;
      h.z[f] = zc[((kn >> 1) * cny + (jn >> 1)) * cnx + (in >> 1)] * m;
    }
  }
}
// (N w)_c from a loaded neighbourhood: couplings x-: S[x-].y, x+: S[c].y,
// y-: S[y-].z, y+: S[c].z, z-: S[z-].w, z+: S[c].w.
__device__ __forceinline__ float hood_offdiag(const float4* s, const float* w) {
  float n = s[0].y * w[0];
  n += s[6].y * w[1];
  n += s[2].z * w[2];
  n += s[6].z * w[3];
  n += s[4].w * w[4];
  n += s[6].w * w[5];
  return n;
}

// level l -> l+1 (l >= 1): r_{l+1} = P^T (r - A omega D^-1 r)
__global__ __launch_bounds__(256) void k_down(LevelView L, Cyc p, int tiles_x, int cnx, int cny,
                                              const float* __restrict__ r, float* rc, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  const Tile t = tile_of(tiles_x, cny);
  float v = 0.0f;
  if (t.i < L.nx && t.j < L.ny && t.k < L.nz) {
    const int c = (t.k * L.ny + t.j) * L.nx + t.i;
    Hood<false> h;
    load_hood<false>(L, r, nullptr, cnx, cny, c, t.k, t.j, t.i, h);
    float w[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) w[f] = fabsf(h.s[f].x) * h.r[f];
    // computed for every row and selected (a branch would let the compiler
    // sink the neighbour loads behind the load of the row's own entry)
    float n = hood_offdiag(h.s, w);
    if (h.s[6].x < 0.0f)
      n += extras_sum(L, c, t.k, t.j, t.i, [&](int nb, int, int, int) { return fabsf(L.S[nb].x) * r[nb]; });
    const float full = (1.0f - p.w) * h.r[6] - p.w * n;
    v = h.s[6].x == 0.0f ? h.r[6] : full;
  }
  restrict_store(t, v, cnx, cny, rc);
}

// level l+1 -> l (l >= 1): zt = post-smoothed (omega D^-1 r + alpha P z_{l+1})
__global__ __launch_bounds__(256) void k_up(LevelView L, Cyc p, int tiles_x, int cnx, int cny,
                                            const float* __restrict__ r, const float* __restrict__ zc, float* zt,
                                            const SolveScalars* sc) {
  if (solve_done(sc)) return;
  const Tile t = tile_of(tiles_x, cny);
  if (t.i < L.nx && t.j < L.ny && t.k < L.nz) {
    const int c = (t.k * L.ny + t.j) * L.nx + t.i;
    Hood<true> h;
    load_hood<true>(L, r, zc, cnx, cny, c, t.k, t.j, t.i, h);
    float w[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) w[f] = p.w * (fabsf(h.s[f].x) * h.r[f]) + p.a * h.z[f];
    float n = hood_offdiag(h.s, w);
    if (h.s[6].x < 0.0f)
      n += extras_sum(L, c, t.k, t.j, t.i, [&](int nb, int kn, int jn, int in) {
        return p.w * (fabsf(L.S[nb].x) * r[nb]) + p.a * zc[((kn >> 1) * cny + (jn >> 1)) * cnx + (in >> 1)];
      });
    const float full = (1.0f - p.w) * w[6] + p.w * (fabsf(h.s[6].x) * (h.r[6] - n));
    zt[c] = h.s[6].x == 0.0f ? w[6] : full;
  }
}

// ------------------------------------------------------------- level 0
// Level 0 in two fused sweeps, each marching a 64 x 4 tile of (i, j)
// columns up a chunk of z-planes (an even number) with the plane's values in
// LDS (halo included, double-buffered) and the column's z-neighbours in
// registers:
//   down  zt = omega D^-1 r formed per cell, q = A zt, and
//         r_1 = P^T (r - q) over the unknowns (pairs of planes summed in
//         registers, pairs of columns by a shuffle, pairs of rows in LDS);
//   up    zp = omega D^-1 r + alpha P z_1 formed per cell, q = A zp, and
//         z = zp + omega D^-1 (r - q) on the unknowns (0 elsewhere).
// Both treat every cell on its own: a slave's value is taken as 0 and its
// row is not moved to its root.  The rows this changes (roots, and unknowns
// next to a slave) are corrected to the merged operator (slaves take their
// root's value, roots add their slaves' rows) from term lists built when the
// body is set: trailing workgroups of each sweep's launch form the terms, a
// small kernel after it adds them in.
template <class C>
struct L0 {
  int nx, ny, nz, kchunk, tiles_x, tiles_y;
  const C *tx, *txb, *ty, *tz, *dinv;   // coefficients: FP32, or their BF16 roundings
  const float* r;
  const unsigned char* red;
  Cyc p;
  int cnx, cny;            // level 1
  const float* zc;         // level-1 correction (up)
};

// A coefficient as FP32: itself, or a BF16 (stored as its upper 16 bits).
__device__ __forceinline__ float cf(float v) { return v; }
__device__ __forceinline__ float cf(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
// Four consecutive coefficients (16- or 8-byte aligned).
__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ float4 ld4(const unsigned short* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}

constexpr int L0X = 64, L0Y = 4;

// What a cell's value is formed from: r, D^-1, the unknown flag and (up)
// the level-1 correction of its parent; loaded unconditionally so that the
// loads of one plane are independent.
struct Raw {
  float r, d, z;
  int m;
};

template <bool UP, class C>
__device__ __forceinline__ Raw l0_raw(const L0<C>& a, long long c, int i, int j, int k) {
  Raw w;
  w.r = a.r[c];
  w.d = cf(a.dinv[c]);
  w.m = a.red[c];
  w.z = UP ? a.zc[((long long)(k >> 1) * a.cny + (j >> 1)) * a.cnx + (i >> 1)] : 0.0f;
  return w;
}

template <bool UP, class C>
__device__ __forceinline__ float l0_val(const L0<C>& a, const Raw& w) {
  const float v = a.p.w * (w.d * w.r);
  return UP && w.m ? v + a.p.a * w.z : v;
}

template <bool UP, class C>
__device__ __forceinline__ float l0_value(const L0<C>& a, long long c, int i, int j, int k) {
  return l0_val<UP>(a, l0_raw<UP>(a, c, i, j, k));
}

// The five face coefficients of a cell other than its lower z-face.
struct Faces {
  float txm, txp, tym, typ, tzp;
};
template <class C>
__device__ __forceinline__ Faces l0_faces(const L0<C>& a, long long c, long long yi, int i, int j, int k) {
  const long long plane = (long long)a.nx * a.ny;
  Faces f;
  f.txm = cf(a.tx[c]);
  f.txp = i < a.nx - 1 ? cf(a.tx[c + 1]) : cf(a.txb[(long long)k * a.ny + j]);
  f.tym = cf(a.ty[yi]);
  f.typ = cf(a.ty[yi + a.nx]);
  f.tzp = cf(a.tz[c + plane]);
  return f;
}

// The fix-ups' terms, formed by the workgroups of a level-0 sweep's launch
// that follow the sweep's own (ids from nsweep on): they read only the
// inputs of the cycle's level 0 (r, D^-1, the coefficients, the roots and,
// up, the level-1 correction), never what the sweep writes, so they need no
// launch of their own.
struct Fix {
  int nsweep = 0;                  // workgroups of the sweep itself
  int n = 0;                       // terms (0: none)
  const int4* terms = nullptr;     // the listed terms (FixTerm)
  float* val = nullptr;            // one value per term
};
template <bool UP, class C> __device__ void l0_fix_block(const L0<C>& a, const Fix& F, int b);

template <bool UP, class C>
__global__ __launch_bounds__(L0X* L0Y) void k_l0(L0<C> a, float* out, const float* __restrict__ q,
                                                double* __restrict__ part, Fix fx, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  if ((int)blockIdx.x >= fx.nsweep) {
    l0_fix_block<UP>(a, fx, (int)blockIdx.x - fx.nsweep);
    return;
  }
  __shared__ float pl[2][L0Y + 2][L0X + 2];
  __shared__ float rb[2][L0Y][L0X / 2];
  const int blk = xcd_remap(blockIdx.x, fx.nsweep);
  const int bx = blk % a.tiles_x, rest = blk / a.tiles_x;
  const int by = rest % a.tiles_y, bz = rest / a.tiles_y;
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  const int i = bx * L0X + lx, j = by * L0Y + ly;
  const int k0 = bz * a.kchunk, k1 = min(a.nz, k0 + a.kchunk);
  const bool in = i < a.nx && j < a.ny;
  const long long plane = (long long)a.nx * a.ny;
  // halo cell of this thread (if any): rows below / above the tile from
  // waves 0 / 3, the columns left / right from lanes 0-3 / 4-7 of wave 1
  int hi = 0, hj = 0, hy = 0, hx = 0;
  bool has_halo = true;
  if (ly == 0) {
    hi = i; hj = by * L0Y - 1; hy = 0; hx = lx + 1;
  } else if (ly == L0Y - 1) {
    hi = i; hj = by * L0Y + L0Y; hy = L0Y + 1; hx = lx + 1;
  } else if (ly == 1 && lx < 2 * L0Y) {
    hi = lx < L0Y ? bx * L0X - 1 : bx * L0X + L0X;
    hj = by * L0Y + (lx & (L0Y - 1));
    hy = (lx & (L0Y - 1)) + 1;
    hx = lx < L0Y ? 0 : L0X + 1;
  } else {
    has_halo = false;
  }
  const bool halo_in = has_halo && hi >= 0 && hi < a.nx && hj >= 0 && hj < a.ny;
  const long long hc0 = (long long)hj * a.nx + hi;
  const Raw zero{0.0f, 0.0f, 0.0f, 0};
  long long c = (long long)k0 * plane + (long long)j * a.nx + i;
  long long yi = ((long long)k0 * (a.ny + 1) + j) * a.nx + i;
  const long long yplane = (long long)(a.ny + 1) * a.nx;
  // software pipeline: the cell's own values at k and k+1, its faces at k,
  // the halo's values at k
  float vm = 0.0f, tzm = 0.0f;
  Raw cur = zero, nxt = zero, hcur = zero;
  Faces f{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (k0 < a.nz) {
    if (in) {
      if (k0 > 0) vm = l0_value<UP>(a, c - plane, i, j, k0 - 1);
      cur = l0_raw<UP>(a, c, i, j, k0);
      if (k0 + 1 < a.nz) nxt = l0_raw<UP>(a, c + plane, i, j, k0 + 1);
      tzm = cf(a.tz[c]);
      f = l0_faces(a, c, yi, i, j, k0);
    }
    if (halo_in) hcur = l0_raw<UP>(a, (long long)k0 * plane + hc0, hi, hj, k0);
  }
  float acc = 0.0f;
  double dot = 0.0;
  for (int k = k0; k < k1; ++k, c += plane, yi += yplane) {
    const int b = (k - k0) & 1;
    const float vc = in ? l0_val<UP>(a, cur) : 0.0f;
    pl[b][ly + 1][lx + 1] = vc;
    if (has_halo) pl[b][hy][hx] = halo_in ? l0_val<UP>(a, hcur) : 0.0f;
    // prefetch the next plane before waiting
    Raw nn = zero, hnext = zero;
    Faces fn = f;
    if (in && k + 1 < k1) {
      if (k + 2 < a.nz) nn = l0_raw<UP>(a, c + 2 * plane, i, j, k + 2);
      fn = l0_faces(a, c + plane, yi + yplane, i, j, k + 1);
    }
    if (halo_in && k + 1 < k1) hnext = l0_raw<UP>(a, (long long)(k + 1) * plane + hc0, hi, hj, k + 1);
    __syncthreads();
    const float vp = (in && k + 1 < a.nz) ? l0_val<UP>(a, nxt) : 0.0f;
    float w = 0.0f;
    if (in) {
      float aq = f.txm * (vc - pl[b][ly + 1][lx]);
      aq = aq + f.txp * (vc - pl[b][ly + 1][lx + 2]);
      aq = aq + f.tym * (vc - pl[b][ly][lx + 1]);
      aq = aq + f.typ * (vc - pl[b][ly + 2][lx + 1]);
      aq = aq + tzm * (vc - vm);
      aq = aq + f.tzp * (vc - vp);
      if (UP) {
        const float zo = cur.m ? vc + a.p.w * (cur.d * (cur.r - aq)) : 0.0f;
        out[c] = zo;
        if (part) dot += (double)zo * (double)q[c];
      } else if (cur.m) {
        w = cur.r - aq;
      }
    }
    if (!UP) {
      acc += w;
      if (((k - k0) & 1) == 1 || k == a.nz - 1) {   // a pair of planes (or the last, odd one) done
        const int pb = ((k - k0) >> 1) & 1;
        const float v2 = acc + __shfl_xor(acc, 1, 64);
        if ((lx & 1) == 0) rb[pb][ly][lx >> 1] = v2;
        acc = 0.0f;
        __syncthreads();
        if (lx < 32 && ly < L0Y / 2) {
          const int I = bx * (L0X / 2) + lx, J = by * (L0Y / 2) + ly, K = k >> 1;
          if (I < a.cnx && J < a.cny)
            out[((long long)K * a.cny + J) * a.cnx + I] = rb[pb][2 * ly][lx] + rb[pb][2 * ly + 1][lx];
        }
      }
    }
    vm = vc;
    tzm = f.tzp;
    cur = nxt;
    nxt = nn;
    hcur = hnext;
    f = fn;
  }
  if (UP && part) {
    __shared__ double red[L0X * L0Y / 64];
    const double t = block_sum(dot, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// The same two sweeps with 4 consecutive cells per lane (nx a multiple of
// 4, arrays 16-byte aligned): a workgroup marches a 256 x 4 tile, every
// per-cell array is read with one 16-byte load per lane, so that a plane
// costs about 3 vector memory instructions per cell instead of 12.
struct Raw4 {
  float4 r, d, z;   // z: parents' corrections of cells 0-1 and 2-3 in z.x, z.y
  uchar4 m;
};

template <bool UP, class C>
__device__ __forceinline__ Raw4 l0_raw4(const L0<C>& a, long long c, int i0, int j, int k) {
  Raw4 w;
  w.r = *reinterpret_cast<const float4*>(a.r + c);
  w.d = ld4(a.dinv + c);
  w.m = *reinterpret_cast<const uchar4*>(a.red + c);
  if (UP) {
    const float2 zz =
        *reinterpret_cast<const float2*>(a.zc + ((long long)(k >> 1) * a.cny + (j >> 1)) * a.cnx + (i0 >> 1));
    w.z = make_float4(zz.x, zz.y, 0.0f, 0.0f);
  } else {
    w.z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  return w;
}

template <bool UP, class C>
__device__ __forceinline__ float4 l0_val4(const L0<C>& a, const Raw4& w) {
  float4 v = make_float4(a.p.w * (w.d.x * w.r.x), a.p.w * (w.d.y * w.r.y), a.p.w * (w.d.z * w.r.z),
                         a.p.w * (w.d.w * w.r.w));
  if (UP) {
    v.x = w.m.x ? v.x + a.p.a * w.z.x : v.x;
    v.y = w.m.y ? v.y + a.p.a * w.z.x : v.y;
    v.z = w.m.z ? v.z + a.p.a * w.z.y : v.z;
    v.w = w.m.w ? v.w + a.p.a * w.z.y : v.w;
  }
  return v;
}

struct Faces4 {
  float4 txm, tym, typ, tzp;
  float tx4;   // the +x face of the last cell
};
template <class C>
__device__ __forceinline__ Faces4 l0_faces4(const L0<C>& a, long long c, long long yi, int i0, int j, int k) {
  const long long plane = (long long)a.nx * a.ny;
  Faces4 f;
  f.txm = ld4(a.tx + c);
  const bool last = i0 + 4 >= a.nx;
  const float t4 = cf(a.tx[last ? c : c + 4]);
  const float tb = cf(a.txb[(long long)k * a.ny + j]);
  const float ml = last ? 1.0f : 0.0f;
  f.tx4 = t4 * (1.0f - ml) + tb * ml;
  f.tym = ld4(a.ty + yi);
  f.typ = ld4(a.ty + yi + a.nx);
  f.tzp = ld4(a.tz + c + plane);
  return f;
}

__device__ __forceinline__ float4 f4(float v) { return make_float4(v, v, v, v); }
__device__ __forceinline__ float comp(const float4& v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }

template <bool UP, class C>
__global__ __launch_bounds__(L0X* L0Y) void k_l0_x4(L0<C> a, float* out, const float* __restrict__ q,
                                               double* __restrict__ part, Fix fx, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  if ((int)blockIdx.x >= fx.nsweep) {
    l0_fix_block<UP>(a, fx, (int)blockIdx.x - fx.nsweep);
    return;
  }
  constexpr int W = 4 * L0X;   // cells of a tile row
  __shared__ float pl[2][L0Y + 2][W + 2];
  __shared__ float rb[2][L0Y][W / 2];
  const int blk = xcd_remap(blockIdx.x, fx.nsweep);
  const int bx = blk % a.tiles_x, rest = blk / a.tiles_x;
  const int by = rest % a.tiles_y, bz = rest / a.tiles_y;
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  const int i0 = bx * W + 4 * lx, j = by * L0Y + ly;
  const int k0 = bz * a.kchunk, k1 = min(a.nz, k0 + a.kchunk);
  const bool in = i0 < a.nx && j < a.ny;
  const long long plane = (long long)a.nx * a.ny;
  // halo: rows below / above from waves 0 / 3 (4 cells per lane), the
  // columns left / right from lanes 0-3 / 4-7 of wave 1 (one cell each)
  int hj = 0, hi = 0, hy = 0, hx = 0, hkind = 0;   // 1: 4-cell row segment, 2: single cell
  if (ly == 0 || ly == L0Y - 1) {
    hkind = 1;
    hi = i0;
    hj = ly == 0 ? by * L0Y - 1 : by * L0Y + L0Y;
    hy = ly == 0 ? 0 : L0Y + 1;
    hx = 4 * lx + 1;
  } else if (ly == 1 && lx < 2 * L0Y) {
    hkind = 2;
    hi = lx < L0Y ? bx * W - 1 : bx * W + W;
    hj = by * L0Y + (lx & (L0Y - 1));
    hy = (lx & (L0Y - 1)) + 1;
    hx = lx < L0Y ? 0 : W + 1;
  }
  const bool halo_in = hkind != 0 && hi >= 0 && hi < a.nx && hj >= 0 && hj < a.ny;
  const long long hc0 = (long long)hj * a.nx + hi;
  Raw4 zero4;
  zero4.r = zero4.d = zero4.z = f4(0.0f);
  zero4.m = make_uchar4(0, 0, 0, 0);
  const Raw zero1{0.0f, 0.0f, 0.0f, 0};
  long long c = (long long)k0 * plane + (long long)j * a.nx + i0;
  long long yi = ((long long)k0 * (a.ny + 1) + j) * a.nx + i0;
  const long long yplane = (long long)(a.ny + 1) * a.nx;
  float4 vm = f4(0.0f), tzm = f4(0.0f);
  Raw4 cur = zero4, nxt = zero4, hc4 = zero4;
  Raw hc1 = zero1;
  Faces4 f{f4(0.0f), f4(0.0f), f4(0.0f), f4(0.0f), 0.0f};
  if (k0 < a.nz) {
    if (in) {
      if (k0 > 0) vm = l0_val4<UP>(a, l0_raw4<UP>(a, c - plane, i0, j, k0 - 1));
      cur = l0_raw4<UP>(a, c, i0, j, k0);
      if (k0 + 1 < a.nz) nxt = l0_raw4<UP>(a, c + plane, i0, j, k0 + 1);
      tzm = ld4(a.tz + c);
      f = l0_faces4(a, c, yi, i0, j, k0);
    }
    if (halo_in) {
      if (hkind == 1) hc4 = l0_raw4<UP>(a, (long long)k0 * plane + hc0, hi, hj, k0);
      else hc1 = l0_raw<UP>(a, (long long)k0 * plane + hc0, hi, hj, k0);
    }
  }
  float acc0 = 0.0f, acc1 = 0.0f;
  double dot = 0.0;
  for (int k = k0; k < k1; ++k, c += plane, yi += yplane) {
    const int b = (k - k0) & 1;
    const float4 vc = in ? l0_val4<UP>(a, cur) : f4(0.0f);
    float* row = &pl[b][ly + 1][4 * lx + 1];
    row[0] = vc.x; row[1] = vc.y; row[2] = vc.z; row[3] = vc.w;
    if (hkind == 1) {
      const float4 hv = halo_in ? l0_val4<UP>(a, hc4) : f4(0.0f);
      float* hr = &pl[b][hy][hx];
      hr[0] = hv.x; hr[1] = hv.y; hr[2] = hv.z; hr[3] = hv.w;
    } else if (hkind == 2) {
      pl[b][hy][hx] = halo_in ? l0_val<UP>(a, hc1) : 0.0f;
    }
    // prefetch the next plane before waiting
    Raw4 nn = zero4, hn4 = zero4;
    Raw hn1 = zero1;
    Faces4 fn = f;
    if (in && k + 1 < k1) {
      if (k + 2 < a.nz) nn = l0_raw4<UP>(a, c + 2 * plane, i0, j, k + 2);
      fn = l0_faces4(a, c + plane, yi + yplane, i0, j, k + 1);
    }
    if (halo_in && k + 1 < k1) {
      if (hkind == 1) hn4 = l0_raw4<UP>(a, (long long)(k + 1) * plane + hc0, hi, hj, k + 1);
      else hn1 = l0_raw<UP>(a, (long long)(k + 1) * plane + hc0, hi, hj, k + 1);
    }
    __syncthreads();
    const float4 vp = (in && k + 1 < a.nz) ? l0_val4<UP>(a, nxt) : f4(0.0f);
    float w[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (in) {
      const float xl = pl[b][ly + 1][4 * lx], xr = pl[b][ly + 1][4 * lx + 5];
      float o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float ve = comp(vc, e);
        const float vxm = e == 0 ? xl : comp(vc, e - 1);
        const float vxp = e == 3 ? xr : comp(vc, e + 1);
        const float txp = e == 3 ? f.tx4 : comp(f.txm, e + 1);
        float q = comp(f.txm, e) * (ve - vxm);
        q = q + txp * (ve - vxp);
        q = q + comp(f.tym, e) * (ve - pl[b][ly][4 * lx + 1 + e]);
        q = q + comp(f.typ, e) * (ve - pl[b][ly + 2][4 * lx + 1 + e]);
        q = q + comp(tzm, e) * (ve - comp(vm, e));
        q = q + comp(f.tzp, e) * (ve - comp(vp, e));
        const int me = e == 0 ? cur.m.x : e == 1 ? cur.m.y : e == 2 ? cur.m.z : cur.m.w;
        if (UP)
          o[e] = me ? ve + a.p.w * (comp(cur.d, e) * (comp(cur.r, e) - q)) : 0.0f;
        else
          w[e] = me ? comp(cur.r, e) - q : 0.0f;
      }
      if (UP) {
        *reinterpret_cast<float4*>(out + c) = make_float4(o[0], o[1], o[2], o[3]);
        if (part) {
          const float4 q4 = *reinterpret_cast<const float4*>(q + c);
          dot += (double)o[0] * (double)q4.x + (double)o[1] * (double)q4.y + (double)o[2] * (double)q4.z +
                 (double)o[3] * (double)q4.w;
        }
      }
    }
    if (!UP) {
      acc0 += w[0] + w[1];
      acc1 += w[2] + w[3];
      if (((k - k0) & 1) == 1 || k == a.nz - 1) {   // a pair of planes (or the last, odd one) done
        const int pb = ((k - k0) >> 1) & 1;
        rb[pb][ly][2 * lx] = acc0;
        rb[pb][ly][2 * lx + 1] = acc1;
        acc0 = acc1 = 0.0f;
        __syncthreads();
        if (ly < L0Y / 2) {
          const int I = bx * (W / 2) + 2 * lx, J = by * (L0Y / 2) + ly, K = k >> 1;
          if (I < a.cnx && J < a.cny) {
            const long long o = ((long long)K * a.cny + J) * a.cnx + I;
            out[o] = rb[pb][2 * ly][2 * lx] + rb[pb][2 * ly + 1][2 * lx];
            if (I + 1 < a.cnx) out[o + 1] = rb[pb][2 * ly][2 * lx + 1] + rb[pb][2 * ly + 1][2 * lx + 1];
          }
        }
      }
    }
    vm = vc;
    tzm = f.tzp;
    cur = nxt;
    nxt = nn;
    hc4 = hn4;
    hc1 = hn1;
    f = fn;
  }
  if (UP && part) {
    __shared__ double red[L0X * L0Y / 64];
    const double t = block_sum(dot, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// Coordinates of a cell from its linear index.  The fix-up kernels below
// index in 32 bits: a grid has fewer than 2^31 nodes, so every cell and face
// index fits.
struct Ijk {
  int i, j, k;
};
template <class C> __device__ __forceinline__ Ijk ijk_of(const L0<C>& a, unsigned c) {
  const unsigned nx = a.nx, ny = a.ny;
  const unsigned row = c / nx, k = row / ny;
  return {(int)(c - row * nx), (int)(row - k * ny), (int)k};
}

// v[e0] + ... + v[e1 - 1], added left to right, four loads issued at a time
__device__ __forceinline__ float sum_in_order(const float* __restrict__ v, int e0, int e1) {
  float d = 0.0f;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    const float a = v[e], b = v[e + 1], c = v[e + 2], w = v[e + 3];
    d = d + a;
    d = d + b;
    d = d + c;
    d = d + w;
  }
  for (; e < e1; ++e) d = d + v[e];
  return d;
}

// Down fix-up.  Per entry the merged operator owes q~_c - q_c: an unknown c
// next to a slave, or a root, sum over its faces to slaves of T_f z(root of
// the slave); a slave s (listed with its root's level-1 cell) minus its row
// with merged values, sum_f T_f (z(root) - z(neighbour's root)).  The terms
// are formed by trailing workgroups of the down sweep; then one thread per
// level-1 cell adds its entries' terms in order.
__global__ void k_l0_fix_sum(int nblk, const int* __restrict__ blk, const int* __restrict__ off,
                             const float* __restrict__ term, float* rc, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblk) return;
  rc[blk[t]] += sum_in_order(term, off[t], off[t + 1]);
}


// Up fix-up.  The up sweep formed z = z' + omega D^-1 (r - q^) with a
// slave's value taken as 0 and a root without its slaves' rows.  With the
// merged operator q' = q^ + dq, where dq takes -T_f z'(root of the slave) for
// each face of the row to a slave and, on a root, adds its slaves' rows
// sum_f T_f (z'(root) - z'(neighbour's root)); so z -= omega D^-1 dq.

// A term of either fix-up: s T (z(y1) - z(y2)), listed when the body is set.
struct FixTerm {
  int face;   // coefficient array (0 tx, 1 txb, 2 ty, 3 tz) + 4 for a negative sign
  int idx;    // index in that array
  int y1, y2;  // unknowns (y2 < 0: none)
};
static_assert(sizeof(FixTerm) == sizeof(int4), "a FixTerm is read on the device as one int4");

// z of an unknown y: omega D^-1 r after pre-smoothing (down); plus alpha
// times its parent's level-1 correction before post-smoothing (up)
template <bool UP, class C> __device__ __forceinline__ float zfix(const L0<C>& a, unsigned y) {
  const float v = a.p.w * (cf(a.dinv[y]) * a.r[y]);
  if constexpr (!UP) return v;
  const Ijk p = ijk_of(a, y);
  const unsigned par = ((unsigned)(p.k >> 1) * a.cny + (unsigned)(p.j >> 1)) * a.cnx + (unsigned)(p.i >> 1);
  return v + a.p.a * a.zc[par];
}

// the value of one term
template <bool UP, class C> __device__ __forceinline__ float fix_term(const L0<C>& a, const int4 t) {
  const int arr = t.x & 3;
  const C* base = arr == 0 ? a.tx : arr == 1 ? a.txb : arr == 2 ? a.ty : a.tz;
  const float T = cf(base[(unsigned)t.y]);
  const float z1 = zfix<UP>(a, (unsigned)t.z);
  const float z2 = zfix<UP>(a, t.w < 0 ? 0u : (unsigned)t.w) * (t.w < 0 ? 0.0f : 1.0f);
  const float v = T * (z1 - z2);
  return (t.x & 4) ? -v : v;
}

// The fix-up workgroups of a level-0 sweep: one thread per term.
template <bool UP, class C> __device__ void l0_fix_block(const L0<C>& a, const Fix& F, int b) {
  const int t = b * (L0X * L0Y) + (int)threadIdx.x;
  if (t < F.n) F.val[t] = fix_term<UP>(a, F.terms[t]);
}

// step 2 (after the up sweep and its trailing workgroups): one thread per
// listed row adds its terms in order and applies
// z -= omega D^-1 dq.  The up sweep summed z_old . q for the row; the z.q
// partial takes the difference.
template <class C>
__global__ __launch_bounds__(256) void k_l0_up_fix(L0<C> a, int nrow, const int* __restrict__ rows,
                                                   const int* __restrict__ off, const float* __restrict__ val, float* z,
                                                   const float* __restrict__ qv, double* __restrict__ part,
                                                   const SolveScalars* sc) {
  if (solve_done(sc)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double dd = 0.0;
  if (t < nrow) {
    const unsigned c = (unsigned)rows[t];
    const float dq = sum_in_order(val, off[t], off[t + 1]);
    const float zold = z[c];
    const float znew = zold - a.p.w * (cf(a.dinv[c]) * dq);
    z[c] = znew;
    if (part) dd = ((double)znew - (double)zold) * (double)qv[c];
  }
  if (part) {
    __shared__ double red2[256 / 64];
    const double s2 = block_sum(dd, red2);
    if (threadIdx.x == 0) part[blockIdx.x] = s2;
  }
}

// The levels from `first` down, in one workgroup: vectors of level l in LDS
// at [off[l], off[l] + n_l) (r) and [off[l] + n_l, off[l] + 2 n_l) (z).
struct TailArgs {
  int first, last;                 // last = the coarsest level
  int off[kMaxLevels];
  int soff[kMaxLevels];            // LDS copy of S of level l < last at [soff[l], soff[l] + 4 n_l) (16-byte aligned)
  LevelView lv[kMaxLevels];
  Cyc p;
  const float* rin;                // r of level `first`
  float* zout;                     // z of level `first`
  const double* minv;              // coarsest dense inverse (row-major)
};

__global__ __launch_bounds__(1024) void k_tail(TailArgs A, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  extern __shared__ float lds[];
  const int t = threadIdx.x, nt = blockDim.x;
  auto cells = [&](int l) { return A.lv[l].nx * A.lv[l].ny * A.lv[l].nz; };
  // r of the first level and the cycle storage of every level but the
  // coarsest, into LDS in one round of loads; the levels' views then read S
  // there (their side lists stay in global memory)
  for (int c = t; c < cells(A.first); c += nt) lds[A.off[A.first] + c] = A.rin[c];
  for (int l = A.first; l < A.last; ++l) {
    float4* s = reinterpret_cast<float4*>(lds + A.soff[l]);
    for (int c = t; c < cells(l); c += nt) s[c] = A.lv[l].S[c];
  }
  __syncthreads();
  auto view = [&](int l) {
    LevelView v = A.lv[l];
    if (l < A.last) v.S = reinterpret_cast<const float4*>(lds + A.soff[l]);
    return v;
  };
  // down: a thread per fine cell (its term parked in the level's z slot,
  // unused until the way up), then a thread per coarse cell sums 8 terms
  for (int l = A.first; l < A.last; ++l) {
    const LevelView F = view(l);
    const LevelView& C = A.lv[l + 1];
    const float* r = lds + A.off[l];
    float* v = lds + A.off[l] + cells(l);
    float* rc = lds + A.off[l + 1];
    for (int c = t; c < cells(l); c += nt) {
      const int i = c % F.nx, rr = c / F.nx, j = rr % F.ny, k = rr / F.ny;
      v[c] = down_value(F, A.p, r, c, k, j, i);
    }
    __syncthreads();
    for (int B = t; B < cells(l + 1); B += nt) {
      const int I = B % C.nx, rr = B / C.nx, J = rr % C.ny, K = rr / C.ny;
      float s = 0.0f;
      for (int kk = 0; kk < 2; ++kk)
        for (int jj = 0; jj < 2; ++jj)
          for (int ii = 0; ii < 2; ++ii) {
            const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
            if (k < F.nz && j < F.ny && i < F.nx) s += v[(k * F.ny + j) * F.nx + i];
          }
      rc[B] = s;
    }
    __syncthreads();
  }
  // coarsest: z = M r in FP64, G lanes per row (G a power of two dividing 64)
  {
    const int N = cells(A.last);
    const float* r = lds + A.off[A.last];
    float* z = lds + A.off[A.last] + N;
    int G = 1;
    while (G < 64 && 2 * G * N <= nt) G *= 2;
    const int i = t / G, q = t % G;
    double s = 0.0;
    if (i < N)
      for (int jc = q; jc < N; jc += G) s += A.minv[(long long)i * N + jc] * (double)r[jc];
    for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m, 64);
    if (i < N && q == 0) z[i] = (float)s;
  }
  __syncthreads();
  for (int l = A.last - 1; l >= A.first; --l) {
    const LevelView F = view(l);
    const LevelView& C = A.lv[l + 1];
    const float* r = lds + A.off[l];
    float* z = lds + A.off[l] + cells(l);
    const float* zc = lds + A.off[l + 1] + cells(l + 1);
    for (int c = t; c < cells(l); c += nt) {
      const int i = c % F.nx, rr = c / F.nx, j = rr % F.ny, k = rr / F.ny;
      z[c] = up_value(F, A.p, r, zc, C.nx, C.ny, c, k, j, i);
    }
    __syncthreads();
  }
  for (int c = t; c < cells(A.first); c += nt) A.zout[c] = lds[A.off[A.first] + cells(A.first) + c];
}

// Inverse of a dense symmetric positive definite matrix (Cholesky).
bool spd_inverse(std::vector<double>& a, int n) {
  // a = L L^T in the lower triangle
  for (int j = 0; j < n; ++j) {
    double d = a[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    const double l = std::sqrt(d);
    a[(size_t)j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double s = a[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
      a[(size_t)i * n + j] = s / l;
    }
  }
  // columns of the inverse: solve L L^T x = e_c
  std::vector<double> inv((size_t)n * n), y(n);
  for (int col = 0; col < n; ++col) {
    for (int i = 0; i < n; ++i) {
      double s = i == col ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= a[(size_t)i * n + k] * y[k];
      y[i] = s / a[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= a[(size_t)k * n + i] * inv[(size_t)col * n + k];
      inv[(size_t)col * n + i] = s / a[(size_t)i * n + i];
    }
  }
  a.swap(inv);
  return true;
}

struct Level {
  Dims d;
  DevBuf A64;                   // 27 x n FP64 stencil
  DevBuf S;                     // float4 per cell: cycle storage
  DevBuf xcell, xval;           // side list of rows with couplings outside the 7 points
  int m = 0;                    // its length
  long long xcap = 0;           // its capacity (rows)
  DevBuf r, zt;                 // cycle vectors: right-hand side, corrected z
  LevelView view() const {
    return {d.nx, d.ny, d.nz, m, S.as<float4>(), xcell.as<int>(), xval.as<float>()};
  }
};

constexpr int kTailThreads = 1024;
constexpr int kTailLdsBytes = 64 * 1024;
constexpr int kDefaultTailCells = 1024;

}  // namespace
}  // namespace nfa

using namespace nfa;

struct nfa_mg_s {
  Poisson* op = nullptr;
  int L = 0;                    // levels including level 0
  Level lv[kMaxLevels];         // lv[0]: dims only
  DevBuf group_of, minv, xcnt;
  DevBuf tx16, txb16, ty16, tz16, d16;   // level-0 coefficients and D^-1 rounded to BF16
  bool coef16 = false;          // the cycle's level 0 reads the BF16 copies
  DevBuf fblk, foff, fterm, fval;   // level-0 down fix-up: level-1 cells, CSR offsets, terms (FixTerm), values
  int nfblk = 0, nfterm = 0;
  DevBuf uoff, uterm, uval;         // level-0 up fix-up: CSR offsets per listed row, terms (FixTerm), values
  int nuterm = 0;
  int body_version = -1;        // grid body the fix-up lists belong to
  int ncoarse = 0;
  int cus = 1;                  // compute units of the device the handle was made on
  int tail_cells = kDefaultTailCells;
  double omega = kDefaultOmega, alpha = kDefaultAlpha;
  int first_tail = 1;           // first level run by the one-workgroup tail kernel
  int built_version = -1;       // op->version the coarse operators belong to
};

namespace nfa {
namespace {

// The first level of the tail: the coarsest, or further up while each level
// has at most tail_cells cells and the tail's vectors fit in LDS.
void plan_tail(nfa_mg_s& mg) {
  int first = mg.L - 1;
  // LDS floats: r and z of every tail level, a float4 copy of S of each
  // but the coarsest, and 3 floats of alignment padding
  long long floats = 2 * mg.lv[first].d.n + 3;
  while (first > 1) {
    const long long n = mg.lv[first - 1].d.n;
    if (n > mg.tail_cells || (floats + 6 * n) * 4 > kTailLdsBytes) break;
    floats += 6 * n;
    --first;
  }
  mg.first_tail = first;
}

// Side list of level l: count per block, scan on the host, scatter in cell
// order.  Grows the list's storage when the merge set needs more rows.
nfa_status build_side_list(nfa_mg_s& mg, Level& C, hipStream_t st) {
  const long long nb = (C.d.n + kBlock - 1) / kBlock;
  int* cnt = mg.xcnt.as<int>();
  k_xcount<<<(int)nb, kBlock, 0, st>>>(C.d.n, C.S.as<float4>(), cnt);
  NFA_CHECK_LAUNCH();
  std::vector<int> h(nb);
  NFA_HIP(hipMemcpyAsync(h.data(), cnt, nb * sizeof(int), hipMemcpyDeviceToHost, st));
  NFA_HIP(hipStreamSynchronize(st));
  long long m = 0;
  for (long long b = 0; b < nb; ++b) {
    const int c = h[b];
    h[b] = (int)m;
    m += c;
  }
  C.m = (int)m;
  if (m == 0) return NFA_OK;
  if (m > C.xcap) {
    // creation reserves min(n, 12 slaves + 256) rows; the rows a merge set
    // couples beyond 7 points are at most 8 per slave on level 1 (the root's
    // block and the blocks of the slave's neighbours and its own) and, on a
    // coarser level, the blocks that hold such rows of the level below
    C.m = 0;
    return fail(NFA_ERR_NOMEM, "multigrid: side list longer than its reserved bound");
  }
  NFA_HIP(hipMemcpyAsync(cnt + nb, h.data(), nb * sizeof(int), hipMemcpyHostToDevice, st));
  k_xscatter<<<(int)nb, kBlock, 0, st>>>(C.d.n, C.S.as<float4>(), C.A64.as<double>(), cnt + nb, C.xcell.as<int>(),
                                         C.xval.as<float>());
  NFA_CHECK_LAUNCH();
  NFA_HIP(hipStreamSynchronize(st));   // h must outlive the copy
  return NFA_OK;
}

}  // namespace

// The merge fix-ups' term lists of the grid's current body, built when the
// handle is created (the roots they need are gathered on the device).
nfa_status build_fixups(nfa_mg_s& mg, hipStream_t st) {
  Grid& g = *mg.op->g;
  // Every term is
  // s T_f (z(y1) - z(y2)) with a face coefficient, a sign and one or two
  // unknowns (y2 < 0: none); z is an unknown's value after pre-smoothing
  // (down) or before post-smoothing (up).
  const long long plane = (long long)g.nx * g.ny;
  // face f of cell c: coefficient array and index, whether it lies inside the domain, the neighbour
  auto face = [&](long long c, int f, int* arr, long long* idx, bool* in, long long* nb) {
    const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / plane);
    const long long yi = ((long long)k * (g.ny + 1) + j) * g.nx + i;
    switch (f) {
      case 0: *arr = 0; *idx = c; *in = i > 0; *nb = c - 1; break;
      case 1:
        if (i < g.nx - 1) { *arr = 0; *idx = c + 1; } else { *arr = 1; *idx = (long long)k * g.ny + j; }
        *in = i < g.nx - 1; *nb = c + 1; break;
      case 2: *arr = 2; *idx = yi; *in = j > 0; *nb = c - g.nx; break;
      case 3: *arr = 2; *idx = yi + g.nx; *in = j < g.ny - 1; *nb = c + g.nx; break;
      case 4: *arr = 3; *idx = c; *in = k > 0; *nb = c - plane; break;
      default: *arr = 3; *idx = c + plane; *in = k < g.nz - 1; *nb = c + plane; break;
    }
  };
  // each root's slaves, ascending
  std::map<int, std::vector<int>> members;
  for (size_t t = 0; t < g.h_scell.size(); ++t) members[g.h_sroot[t]].push_back(g.h_scell[t]);
  for (auto& m : members) std::sort(m.second.begin(), m.second.end());
  auto upload = [&](DevBuf& b, const std::vector<int>& v) -> hipError_t {
    hipError_t e2 = b.alloc(std::max<size_t>(1, v.size()) * sizeof(int));
    if (e2 != hipSuccess || v.empty()) return e2;
    return hipMemcpy(b.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
  };
  // the roots the terms need (of the neighbours of the listed rows and of
  // the slaves), gathered on the device
  std::vector<int> need;
  for (const std::vector<int>* list : {&g.h_fix, &g.h_scell})
    for (int c : *list)
      for (int f = 0; f < 6; ++f) {
        int arr; long long idx, nb; bool in;
        face(c, f, &arr, &idx, &in, &nb);
        if (in) need.push_back((int)nb);
      }
  std::sort(need.begin(), need.end());
  need.erase(std::unique(need.begin(), need.end()), need.end());
  std::vector<int> need_root(need.size());
  if (!need.empty()) {
    DevBuf d_need, d_out;
    NFA_HIP(upload(d_need, need));
    NFA_HIP(d_out.alloc(need.size() * sizeof(int)));
    k_gather_int<<<blocks_for((long long)need.size()), kBlock, 0, st>>>((int)need.size(), d_need.as<int>(),
                                                                        g.root.as<int>(), d_out.as<int>());
    NFA_CHECK_LAUNCH();
    NFA_HIP(hipMemcpyAsync(need_root.data(), d_out.p, need.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    NFA_HIP(hipStreamSynchronize(st));
  }
  auto root_of = [&](long long x) {
    return need_root[std::lower_bound(need.begin(), need.end(), (int)x) - need.begin()];
  };
  // terms of a row's faces to slaves: s T_f z(root of the slave)
  auto slave_faces = [&](int c, int sign, std::vector<FixTerm>& out) {
    for (int f = 0; f < 6; ++f) {
      int arr; long long idx, nb; bool in;
      face(c, f, &arr, &idx, &in, &nb);
      if (!in) continue;
      const int rt = root_of(nb);
      if (rt >= 0 && rt != nb) out.push_back({arr | sign, (int)idx, rt, -1});
    }
  };
  // terms of slave m's row with merged values: s T_f (z(root) - z(root of the neighbour))
  auto slave_row = [&](int m, int rm, int sign, std::vector<FixTerm>& out) {
    for (int f = 0; f < 6; ++f) {
      int arr; long long idx, nb; bool in;
      face(m, f, &arr, &idx, &in, &nb);
      const int rt = in ? root_of(nb) : -1;
      if (rt == rm) continue;   // T (z(r) - z(r)) = 0
      out.push_back({arr | sign, (int)idx, rm, rt});
    }
  };
  // down: q~ - q per entry, entries grouped by level-1 cell in a fixed
  // order (the listed rows ascending, then the slaves by their root's cell)
  const Dims& C = mg.lv[1].d;
  auto blk0 = [&](long long c) {
    const long long i = c % g.nx, j = (c / g.nx) % g.ny, k = c / plane;
    return (int)(((k >> 1) * C.ny + (j >> 1)) * C.nx + (i >> 1));
  };
  std::vector<std::pair<int, int>> ent;
  for (int c : g.h_fix) ent.push_back({blk0(c), c});
  for (size_t t = 0; t < g.h_scell.size(); ++t) ent.push_back({blk0(g.h_sroot[t]), -(int)t - 1});
  std::stable_sort(ent.begin(), ent.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  std::vector<int> fb, fo;
  std::vector<FixTerm> dt;
  for (size_t e = 0; e < ent.size(); ++e) {
    if (e == 0 || ent[e].first != ent[e - 1].first) {
      fb.push_back(ent[e].first);
      fo.push_back((int)dt.size());
    }
    const int code = ent[e].second;
    if (code >= 0) slave_faces(code, 0, dt);   // an unknown's faces to slaves
    else slave_row(g.h_scell[-code - 1], g.h_sroot[-code - 1], 4, dt);   // minus a slave's row
  }
  fo.push_back((int)dt.size());
  // up: dq per listed row, its faces to slaves, then (a root) its slaves' rows
  std::vector<int> uo(1, 0);
  std::vector<FixTerm> ut;
  for (int c : g.h_fix) {
    slave_faces(c, 4, ut);
    auto it = members.find(c);
    if (it != members.end())
      for (int m : it->second) slave_row(m, c, 0, ut);
    uo.push_back((int)ut.size());
  }
  auto upload_terms = [&](DevBuf& b, const std::vector<FixTerm>& v) -> hipError_t {
    hipError_t e2 = b.alloc(std::max<size_t>(1, v.size()) * sizeof(FixTerm));
    if (e2 != hipSuccess || v.empty()) return e2;
    return hipMemcpy(b.p, v.data(), v.size() * sizeof(FixTerm), hipMemcpyHostToDevice);
  };
  NFA_HIP(upload(mg.fblk, fb));
  NFA_HIP(upload(mg.foff, fo));
  NFA_HIP(upload_terms(mg.fterm, dt));
  NFA_HIP(mg.fval.alloc(std::max<size_t>(1, dt.size()) * sizeof(float)));
  mg.nfblk = (int)fb.size();
  mg.nfterm = (int)dt.size();
  NFA_HIP(upload(mg.uoff, uo));
  NFA_HIP(upload_terms(mg.uterm, ut));
  NFA_HIP(mg.uval.alloc(std::max<size_t>(1, ut.size()) * sizeof(float)));
  mg.nuterm = (int)ut.size();
  mg.body_version = g.body_version;
  return NFA_OK;
}

nfa_status mg_setup(nfa_mg_s& mg, hipStream_t st) {
  Poisson& op = *mg.op;
  Grid& g = *op.g;
  if (const nfa_status e = require_assembled(op, "multigrid")) return e;
  k_fill_int<<<blocks_for(g.n), kBlock, 0, st>>>(g.n, -1, mg.group_of.as<int>());
  if (g.n_groups > 0)
    k_group_of<<<blocks_for(g.n_groups), kBlock, 0, st>>>(g.n_groups, g.g_root.as<int>(), mg.group_of.as<int>());
  const Coeffs<double> c = op.c64();
  for (int l = 1; l < mg.L; ++l) {
    Level& C = mg.lv[l];
    if (l == 1)
      k_level1<<<blocks_for(C.d.n), kBlock, 0, st>>>(mg.lv[0].d, C.d, c.tx, c.txb, c.ty, c.tz,
                                                     g.reduced.as<unsigned char>(), g.root.as<int>(),
                                                     mg.group_of.as<int>(), g.g_off.as<int>(), g.g_mem.as<int>(),
                                                     C.A64.as<double>(), C.S.as<float4>());
    else
      k_coarsen<<<blocks_for(C.d.n), kBlock, 0, st>>>(mg.lv[l - 1].d, C.d, mg.lv[l - 1].A64.as<double>(),
                                                      C.A64.as<double>(), C.S.as<float4>());
    NFA_CHECK_LAUNCH();
  }
  for (int l = 1; l < mg.L - 1; ++l) {
    const nfa_status e = build_side_list(mg, mg.lv[l], st);
    if (e != NFA_OK) return e;
  }
  if (mg.coef16) {
    if (!mg.d16.p) return fail(NFA_ERR_INVALID, "multigrid: BF16 coefficients not allocated");
    const Coeffs<float> c32 = op.c32();
    const float* src[5] = {c32.tx, c32.txb, c32.ty, c32.tz, c32.dinv};
    DevBuf* dst[5] = {&mg.tx16, &mg.txb16, &mg.ty16, &mg.tz16, &mg.d16};
    const long long cnt[5] = {g.n, (long long)g.nz * g.ny, g.nfy(), g.nfz(), g.n};
    for (int t = 0; t < 5; ++t)
      k_to_bf16<<<blocks_for(cnt[t]), kBlock, 0, st>>>(cnt[t], src[t], dst[t]->as<unsigned short>());
    NFA_CHECK_LAUNCH();
  }
  if (mg.body_version != g.body_version)
    return fail(NFA_ERR_INVALID, "multigrid: the grid's body was set after the handle was created; create it again");
  // the coarsest level: dense, regularized, inverted on the host
  const Level& Z = mg.lv[mg.L - 1];
  const int N = (int)Z.d.n;
  std::vector<double> st27((size_t)27 * N);
  NFA_HIP(hipMemcpyAsync(st27.data(), Z.A64.p, st27.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  NFA_HIP(hipStreamSynchronize(st));
  std::vector<double> M((size_t)N * N, 0.0);
  std::vector<char> empty(N, 0);
  double dsum = 0.0;
  int dcount = 0;
  for (int row = 0; row < N; ++row) {
    const int i = row % Z.d.nx, rr = row / Z.d.nx, j = rr % Z.d.ny, k = rr / Z.d.ny;
    for (int o = 0; o < 27; ++o) {
      const double a = st27[(size_t)o * N + row];
      if (a == 0.0) continue;
      const int kn = k + o / 9 - 1, jn = j + (o / 3) % 3 - 1, in = i + o % 3 - 1;
      if (kn < 0 || kn >= Z.d.nz || jn < 0 || jn >= Z.d.ny || in < 0 || in >= Z.d.nx) continue;
      M[(size_t)row * N + ((size_t)kn * Z.d.ny + jn) * Z.d.nx + in] += a;
    }
    const double d = M[(size_t)row * N + row];
    if (d > 0.0) {
      dsum += d;
      ++dcount;
    } else {
      empty[row] = 1;
    }
  }
  if (g.all_neumann() && dcount > 0) {
    const double cc = dsum / dcount;
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b)
        if (!empty[a] && !empty[b]) M[(size_t)a * N + b] += cc;
  }
  for (int a = 0; a < N; ++a)
    if (empty[a])
      for (int b = 0; b < N; ++b) M[(size_t)a * N + b] = M[(size_t)b * N + a] = (a == b) ? 1.0 : 0.0;
  if (!spd_inverse(M, N)) return fail(NFA_ERR_NUMERIC, "multigrid: coarsest matrix is not positive definite");
  // the inverse comes column by column; the tail kernel reads it by rows
  // (consecutive lanes, consecutive columns)
  std::vector<double> Mt((size_t)N * N);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) Mt[(size_t)a * N + b] = M[(size_t)b * N + a];
  NFA_HIP(hipMemcpyAsync(mg.minv.p, Mt.data(), Mt.size() * sizeof(double), hipMemcpyHostToDevice, st));
  NFA_HIP(hipStreamSynchronize(st));
  mg.built_version = op.version;
  return NFA_OK;
}

// Level 0 of the cycle, down: the fused sweep, whose trailing workgroups
// form the merged rows' fix-up terms, then the terms' sums into level 1.
template <class C>
void l0_down(nfa_mg_s& mg, const L0<C>& a, bool x4, int nb0, const SolveScalars* sc, hipStream_t st) {
  Poisson& op = *mg.op;
  Fix fx;
  fx.nsweep = nb0;
  if (mg.nfblk > 0) {
    fx.n = mg.nfterm;
    fx.terms = mg.fterm.as<int4>();
    fx.val = mg.fval.as<float>();
  }
  const int nb = nb0 + (fx.n + L0X * L0Y - 1) / (L0X * L0Y);
  const bool rec = prof_begin(op, st);
  if (x4)
    k_l0_x4<false, C><<<nb, L0X * L0Y, 0, st>>>(a, mg.lv[1].r.as<float>(), nullptr, nullptr, fx, sc);
  else
    k_l0<false, C><<<nb, L0X * L0Y, 0, st>>>(a, mg.lv[1].r.as<float>(), nullptr, nullptr, fx, sc);
  prof_end(op, rec, kProfMgDown, st);
  if (mg.nfblk > 0)
    k_l0_fix_sum<<<(mg.nfblk + 255) / 256, 256, 0, st>>>(mg.nfblk, mg.fblk.as<int>(), mg.foff.as<int>(),
                                                         mg.fval.as<float>(), mg.lv[1].r.as<float>(), sc);
}

// Level 0 of the cycle, up: the fused sweep (with the z.q partials when
// parts is given, nb0 of them, the fix-up's after them), whose trailing
// workgroups form the fix-up's terms, then the fix-up.
template <class C>
void l0_up(nfa_mg_s& mg, const L0<C>& a, bool x4, int nb0, float* z0, const float* qdot, double* parts,
           const SolveScalars* sc, hipStream_t st) {
  Poisson& op = *mg.op;
  Grid& g = *op.g;
  const int nfix = (int)g.h_fix.size();
  Fix fx;
  fx.nsweep = nb0;
  if (nfix > 0) {
    fx.n = mg.nuterm;
    fx.terms = mg.uterm.as<int4>();
    fx.val = mg.uval.as<float>();
  }
  const int nb = nb0 + (fx.n + L0X * L0Y - 1) / (L0X * L0Y);
  const bool rec = prof_begin(op, st);
  if (x4)
    k_l0_x4<true, C><<<nb, L0X * L0Y, 0, st>>>(a, z0, qdot, parts, fx, sc);
  else
    k_l0<true, C><<<nb, L0X * L0Y, 0, st>>>(a, z0, qdot, parts, fx, sc);
  prof_end(op, rec, kProfMgUp, st);
  if (nfix > 0) {
    k_l0_up_fix<C><<<(nfix + 255) / 256, 256, 0, st>>>(a, nfix, g.fix_rows.as<int>(), mg.uoff.as<int>(),
                                                        mg.uval.as<float>(), z0, qdot, parts ? parts + nb0 : nullptr, sc);
  }
}

// One V-cycle: z = M r on the reduced unknowns of level 0 (FP32).
nfa_status mg_vcycle(nfa_mg_s& mg, const float* r0, float* z0, const float* qdot, double* parts, int* np,
                     const SolveScalars* sc, hipStream_t st) {
  Poisson& op = *mg.op;
  Grid& g = *op.g;
  const Coeffs<float> c32 = op.c32();
  const unsigned char* red = g.reduced.as<unsigned char>();
  const Dims d0 = mg.lv[0].d;
  // the grid of a fine level l in 64 x 2 x 2 tiles
  auto tiles = [&](int l, int* tx) {
    *tx = (mg.lv[l].d.nx + 63) / 64;
    return (int)((long long)*tx * mg.lv[l + 1].d.ny * mg.lv[l + 1].d.nz);
  };
  int tx;
  const Cyc p{(float)mg.omega, (float)mg.alpha};
  const Dims& C1 = mg.lv[1].d;
  // 4 cells per lane when rows and every per-cell array allow 16-byte loads
  const bool x4 = d0.nx % 4 == 0 && ((uintptr_t)r0 % 16) == 0 && ((uintptr_t)z0 % 16) == 0;
  const int tw = x4 ? 4 * L0X : L0X;
  // planes per workgroup: 32 (fewer re-read chunk-boundary planes) when the
  // sweep still has a workgroup for each of the 3 resident slots per CU, else 16
  const long long cols = (long long)((d0.nx + tw - 1) / tw) * ((d0.ny + L0Y - 1) / L0Y);
  const int kchunk = cols * ((d0.nz + 31) / 32) >= 3LL * mg.cus ? 32 : 16;
  L0<float> a32{d0.nx, d0.ny, d0.nz, kchunk, (d0.nx + tw - 1) / tw, (d0.ny + L0Y - 1) / L0Y, c32.tx, c32.txb, c32.ty,
                c32.tz, c32.dinv, r0, red, p, C1.nx, C1.ny, nullptr};
  L0<unsigned short> a16{d0.nx, d0.ny, d0.nz, kchunk, a32.tiles_x, a32.tiles_y, mg.tx16.as<unsigned short>(),
                         mg.txb16.as<unsigned short>(), mg.ty16.as<unsigned short>(), mg.tz16.as<unsigned short>(),
                         mg.d16.as<unsigned short>(), r0, red, p, C1.nx, C1.ny, nullptr};
  const int nb0 = a32.tiles_x * a32.tiles_y * ((d0.nz + a32.kchunk - 1) / a32.kchunk);
  // z.q of the flexible direction summed by the up sweep and the up fix-up
  const int nfix_blocks = ((int)g.h_fix.size() + 255) / 256;
  const bool dot = qdot && parts && nb0 + nfix_blocks <= kMaxPartials;
  if (np) *np = 0;
  if (mg.coef16)
    l0_down(mg, a16, x4, nb0, sc, st);
  else
    l0_down(mg, a32, x4, nb0, sc, st);
  // grid-wide levels, down
  const int T = mg.first_tail;
  for (int l = 1; l < T; ++l) {
    const int nb = tiles(l, &tx);
    const Dims& C = mg.lv[l + 1].d;
    k_down<<<nb, 256, 0, st>>>(mg.lv[l].view(), p, tx, C.nx, C.ny, mg.lv[l].r.as<float>(),
                               mg.lv[l + 1].r.as<float>(), sc);
  }
  // the tail: levels T.. in one workgroup
  {
    TailArgs A{};
    A.first = T;
    A.last = mg.L - 1;
    int off = 0;
    for (int l = T; l < mg.L; ++l) {
      A.off[l] = off;
      A.lv[l] = mg.lv[l].view();
      off += 2 * (int)mg.lv[l].d.n;
    }
    off = (off + 3) & ~3;   // 16-byte alignment of the S copies
    for (int l = T; l < mg.L - 1; ++l) {
      A.soff[l] = off;
      off += 4 * (int)mg.lv[l].d.n;
    }
    A.p = p;
    A.rin = mg.lv[T].r.as<float>();
    A.zout = mg.lv[T].zt.as<float>();
    A.minv = mg.minv.as<double>();
    k_tail<<<1, kTailThreads, off * sizeof(float), st>>>(A, sc);
  }
  // grid-wide levels, up
  for (int l = T - 1; l >= 1; --l) {
    const int nb = tiles(l, &tx);
    const Dims& C = mg.lv[l + 1].d;
    k_up<<<nb, 256, 0, st>>>(mg.lv[l].view(), p, tx, C.nx, C.ny, mg.lv[l].r.as<float>(),
                             mg.lv[l + 1].zt.as<float>(), mg.lv[l].zt.as<float>(), sc);
  }
  // level 0, up
  a32.zc = a16.zc = mg.lv[1].zt.as<float>();
  const int nfix = (int)g.h_fix.size();
  if (mg.coef16)
    l0_up(mg, a16, x4, nb0, z0, qdot, dot ? parts : nullptr, sc, st);
  else
    l0_up(mg, a32, x4, nb0, z0, qdot, dot ? parts : nullptr, sc, st);
  if (np) *np = dot ? nb0 + (nfix > 0 ? (nfix + 255) / 256 : 0) : 0;
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

nfa_status mg_precond_apply(void* mgh, Poisson& op, const float* r, float* z, const float* q, double* parts, int* np,
                            const SolveScalars* sc, hipStream_t st) {
  if (!mgh) return fail(NFA_ERR_INVALID, "multigrid preconditioner: no handle");
  nfa_mg_s& mg = *static_cast<nfa_mg_s*>(mgh);
  if (mg.op != &op) return fail(NFA_ERR_INVALID, "multigrid preconditioner: built for another operator");
  if (mg.built_version != op.version) return fail(NFA_ERR_INVALID, "multigrid preconditioner: not set up");
  return mg_vcycle(mg, r, z, q, parts, np, sc, st);
}

nfa_status mg_ensure(void* mgh, Poisson& op, hipStream_t st) {
  if (!mgh) return fail(NFA_ERR_INVALID, "multigrid preconditioner: no handle");
  nfa_mg_s& mg = *static_cast<nfa_mg_s*>(mgh);
  if (mg.op != &op) return fail(NFA_ERR_INVALID, "multigrid preconditioner: built for another operator");
  return mg.built_version == op.version && mg.body_version == op.g->body_version ? NFA_OK : mg_setup(mg, st);
}

}  // namespace nfa

extern "C" nfa_status nfa_mg_create(nfa_poisson op, nfa_mg* out) {
  if (!out) return fail(NFA_ERR_INVALID, "nfa_mg_create: out is NULL");
  *out = nullptr;
  if (!op) return fail(NFA_ERR_INVALID, "nfa_mg_create: NULL operator");
  auto* mg = new nfa_mg_s();
  mg->op = op;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      mg->cus = cus;
  }
  Grid& g = *op->g;
  mg->lv[0].d = make_dims(g.nx, g.ny, g.nz);
  mg->L = 1;
  Dims d = mg->lv[0].d;
  while ((mg->L == 1 || d.n > kMinCoarse) && (d.nx > 1 || d.ny > 1 || d.nz > 1) && mg->L < kMaxLevels) {
    d = coarser(d);
    mg->lv[mg->L++].d = d;
  }
  auto bad = [&](hipError_t e) {
    delete mg;
    return fail(NFA_ERR_HIP, std::string("nfa_mg_create: ") + hipGetErrorString(e));
  };
  if (mg->L < 2) {
    delete mg;
    return fail(NFA_ERR_INVALID, "nfa_mg_create: the grid has a single cell");
  }
  hipError_t e;
  if ((e = mg->group_of.alloc(g.n * 4)) != hipSuccess ||
      (e = mg->xcnt.alloc(2 * ((mg->lv[1].d.n + kBlock - 1) / kBlock) * sizeof(int))) != hipSuccess)
    return bad(e);
  for (int l = 1; l < mg->L; ++l) {
    Level& C = mg->lv[l];
    const size_t n = (size_t)C.d.n;
    if ((e = C.A64.alloc(27 * n * 8)) != hipSuccess || (e = C.S.alloc(n * sizeof(float4))) != hipSuccess ||
        (e = C.r.alloc(n * 4)) != hipSuccess || (e = C.zt.alloc(n * 4)) != hipSuccess)
      return bad(e);
    // side-list rows reserved for the merge set at creation (grown by set-up)
    const long long cap = std::min<long long>((long long)n, 12LL * g.n_slaves + 256);
    if (l < mg->L - 1) {
      if ((e = C.xcell.alloc(cap * sizeof(int))) != hipSuccess ||
          (e = C.xval.alloc(cap * kXSlots * sizeof(float))) != hipSuccess)
        return bad(e);
      C.xcap = cap;
    }
  }
  mg->ncoarse = (int)mg->lv[mg->L - 1].d.n;
  if ((e = mg->minv.alloc((size_t)mg->ncoarse * mg->ncoarse * 8)) != hipSuccess) return bad(e);
  plan_tail(*mg);
  const nfa_status fe = build_fixups(*mg, nullptr);
  if (fe != NFA_OK) {
    delete mg;
    return fe;
  }
  *out = mg;
  return NFA_OK;
}

extern "C" void nfa_mg_destroy(nfa_mg mg) { delete mg; }

extern "C" nfa_status nfa_mg_setup(nfa_mg mg, nfa_stream s) {
  if (!mg) return fail(NFA_ERR_INVALID, "nfa_mg_setup: NULL handle");
  return mg_setup(*mg, S(s));
}

extern "C" nfa_status nfa_mg_apply(nfa_mg mg, const float* r, float* z, nfa_stream s) {
  if (!mg || !r || !z) return fail(NFA_ERR_INVALID, "nfa_mg_apply: NULL argument");
  if (r == z) return fail(NFA_ERR_INVALID, "nfa_mg_apply: r and z must differ");
  if (mg->built_version != mg->op->version || mg->body_version != mg->op->g->body_version)
    return fail(NFA_ERR_INVALID, "nfa_mg_apply: call nfa_mg_setup after the last assembly (and after a new body)");
  const nfa_status e = mg_vcycle(*mg, r, z, nullptr, nullptr, nullptr, nullptr, S(s));
  if (e != NFA_OK) return e;
  launch_merge_copy<float>(*mg->op->g, z, S(s), nullptr);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_mg_set_tail(nfa_mg mg, int max_cells) {
  if (!mg) return fail(NFA_ERR_INVALID, "nfa_mg_set_tail: NULL handle");
  mg->tail_cells = max_cells < 0 ? kDefaultTailCells : max_cells;
  plan_tail(*mg);
  return NFA_OK;
}

extern "C" nfa_status nfa_mg_set_params(nfa_mg mg, double omega, double alpha) {
  if (!mg) return fail(NFA_ERR_INVALID, "nfa_mg_set_params: NULL handle");
  if (!(omega > 0.0 && omega < 1.0) || !(alpha > 0.0 && alpha < 2.0))
    return fail(NFA_ERR_INVALID, "nfa_mg_set_params: need 0 < omega < 1 and 0 < alpha < 2");
  mg->omega = omega;
  mg->alpha = alpha;
  return NFA_OK;
}

extern "C" nfa_status nfa_mg_set_coef(nfa_mg mg, int dtype) {
  if (!mg) return fail(NFA_ERR_INVALID, "nfa_mg_set_coef: NULL handle");
  if (dtype != NFA_F32 && dtype != NFA_BF16) return fail(NFA_ERR_INVALID, "nfa_mg_set_coef: NFA_F32 or NFA_BF16");
  const bool c16 = dtype == NFA_BF16;
  if (c16 && !mg->d16.p) {   // the BF16 copies are allocated here, not by a set-up
    const Grid& g = *mg->op->g;
    if (mg->tx16.alloc(g.n * 2) != hipSuccess || mg->txb16.alloc((size_t)g.nz * g.ny * 2) != hipSuccess ||
        mg->ty16.alloc(g.nfy() * 2) != hipSuccess || mg->tz16.alloc(g.nfz() * 2) != hipSuccess ||
        mg->d16.alloc(g.n * 2) != hipSuccess) {
      mg->d16.release();
      return fail(NFA_ERR_HIP, "nfa_mg_set_coef: out of device memory for the BF16 coefficients");
    }
  }
  if (c16 != mg->coef16) {
    mg->coef16 = c16;
    mg->built_version = -1;   // the BF16 copies are made by the next set-up
  }
  return NFA_OK;
}

extern "C" nfa_status nfa_mg_side_rows(nfa_mg mg, int level, int* rows) {
  if (!mg || !rows) return fail(NFA_ERR_INVALID, "nfa_mg_side_rows: NULL argument");
  if (level < 1 || level >= mg->L) return fail(NFA_ERR_INVALID, "nfa_mg_side_rows: level out of range");
  *rows = mg->lv[level].m;
  return NFA_OK;
}

extern "C" nfa_status nfa_mg_info(nfa_mg mg, int* levels, int* dims) {
  if (!mg || !levels) return fail(NFA_ERR_INVALID, "nfa_mg_info: NULL argument");
  *levels = mg->L;
  if (dims)
    for (int l = 0; l < mg->L; ++l) {
      dims[3 * l] = mg->lv[l].d.nz;
      dims[3 * l + 1] = mg->lv[l].d.ny;
      dims[3 * l + 2] = mg->lv[l].d.nx;
    }
  return NFA_OK;
}

extern "C" nfa_status nfa_mg_export(nfa_mg mg, int level, double* dst, nfa_stream s) {
  if (!mg || !dst) return fail(NFA_ERR_INVALID, "nfa_mg_export: NULL argument");
  if (level < 1 || level >= mg->L) return fail(NFA_ERR_INVALID, "nfa_mg_export: level out of range");
  const Level& C = mg->lv[level];
  NFA_HIP(hipMemcpyAsync(dst, C.A64.p, (size_t)27 * C.d.n * sizeof(double), hipMemcpyDeviceToDevice, S(s)));
  return NFA_OK;
}
