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
// FP64 (for building the next level) and FP32 (for the cycle).
//
// V-cycle in FP32, symmetric (damped Jacobi, omega = 0.7, one sweep before
// and one after the coarse correction; restriction = transpose of the
// piecewise-constant prolongation), so the solve may use it in (flexible)
// CG.  Every kernel returns at once when the solve has converged.
//
// Built with -ffp-contract=off.
#include <cmath>
#include <vector>

#include "device_util.h"
#include "nfa_internal.h"

namespace nfa {
namespace {

constexpr int kMaxLevels = 16;
constexpr long long kMinCoarse = 600;
constexpr float kOmega = 0.7f;

struct Dims {
  int nx, ny, nz;
  long long n;
};

Dims make_dims(int nx, int ny, int nz) { return {nx, ny, nz, (long long)nx * ny * nz}; }
Dims coarser(const Dims& d) { return make_dims((d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2); }

#define MG_STRIDE(idx, n) \
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (n); idx += (long long)gridDim.x * blockDim.x)

__global__ void k_fill_int(long long n, int v, int* a) {
  MG_STRIDE(i, n) a[i] = v;
}

__global__ void k_group_of(int ng, const int* __restrict__ groot, int* __restrict__ group_of) {
  for (int gi = blockIdx.x * blockDim.x + threadIdx.x; gi < ng; gi += gridDim.x * blockDim.x)
    group_of[groot[gi]] = gi;
}

__device__ __forceinline__ void store_row(long long n, long long B, const double* acc, double* A64, float* A32,
                                          float* dinv) {
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    A64[o * n + B] = acc[o];
    A32[o * n + B] = (float)acc[o];
  }
  dinv[B] = acc[13] > 0.0 ? (float)(1.0 / acc[13]) : 0.0f;
}

// Level 1 from the faces of level 0 (see the file head).
__global__ void k_level1(Dims f, Dims c, const double* __restrict__ tx, const double* __restrict__ txb,
                         const double* __restrict__ ty, const double* __restrict__ tz,
                         const unsigned char* __restrict__ reduced, const int* __restrict__ root,
                         const int* __restrict__ group_of, const int* __restrict__ g_off,
                         const int* __restrict__ g_mem, double* A64, float* A32, float* dinv) {
  const long long fplane = (long long)f.nx * f.ny;
  MG_STRIDE(B, c.n) {
    const int I = (int)(B % c.nx);
    const long long rr = B / c.nx;
    const int J = (int)(rr % c.ny), K = (int)(rr / c.ny);
    double acc[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = 0.0;
    for (int kk = 0; kk < 2; ++kk)
      for (int jj = 0; jj < 2; ++jj)
        for (int ii = 0; ii < 2; ++ii) {
          const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
          if (k >= f.nz || j >= f.ny || i >= f.nx) continue;
          const long long cidx = ((long long)k * f.ny + j) * f.nx + i;
          if (!reduced[cidx]) continue;
          const int gi = group_of[cidx];
          const int nmem = 1 + (gi >= 0 ? g_off[gi + 1] - g_off[gi] : 0);
          for (int mi = 0; mi < nmem; ++mi) {
            const long long m = mi == 0 ? cidx : (long long)g_mem[g_off[gi] + mi - 1];
            const int im = (int)(m % f.nx);
            const long long rm = m / f.nx;
            const int jm = (int)(rm % f.ny), km = (int)(rm / f.ny);
            for (int face = 0; face < 6; ++face) {
              double T;
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
              if (!(T > 0.0)) continue;
              if (nb < 0) {          // a Dirichlet boundary face
                acc[13] += T;
                continue;
              }
              const int rn = root[nb];
              if (rn < 0 || (long long)rn == cidx) continue;
              const int in = rn % f.nx;
              const int rrn = rn / f.nx;
              const int jn = rrn % f.ny, kn = rrn / f.ny;
              const int dK = (kn >> 1) - K, dJ = (jn >> 1) - J, dI = (in >> 1) - I;
              if (dK == 0 && dJ == 0 && dI == 0) continue;
              acc[13] += T;
              if (dK >= -1 && dK <= 1 && dJ >= -1 && dJ <= 1 && dI >= -1 && dI <= 1)
                acc[(dK + 1) * 9 + (dJ + 1) * 3 + (dI + 1)] -= T;
            }
          }
        }
    store_row(c.n, B, acc, A64, A32, dinv);
  }
}

// Level l+1 as the Galerkin sum of level l's 27-point stencil.
__global__ void k_coarsen(Dims f, Dims c, const double* __restrict__ Af, double* A64, float* A32, float* dinv) {
  MG_STRIDE(B, c.n) {
    const int I = (int)(B % c.nx);
    const long long rr = B / c.nx;
    const int J = (int)(rr % c.ny), K = (int)(rr / c.ny);
    double acc[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = 0.0;
    for (int kk = 0; kk < 2; ++kk)
      for (int jj = 0; jj < 2; ++jj)
        for (int ii = 0; ii < 2; ++ii) {
          const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
          if (k >= f.nz || j >= f.ny || i >= f.nx) continue;
          const long long cidx = ((long long)k * f.ny + j) * f.nx + i;
          for (int o = 0; o < 27; ++o) {
            const double a = Af[o * f.n + cidx];
            if (a == 0.0) continue;
            const int kn = k + o / 9 - 1, jn = j + (o / 3) % 3 - 1, in = i + o % 3 - 1;
            if (kn < 0 || kn >= f.nz || jn < 0 || jn >= f.ny || in < 0 || in >= f.nx) continue;
            acc[((kn >> 1) - K + 1) * 9 + ((jn >> 1) - J + 1) * 3 + ((in >> 1) - I + 1)] += a;
          }
        }
    store_row(c.n, B, acc, A64, A32, dinv);
  }
}

// ------------------------------------------------------------------ cycle
__global__ void k_pre(long long n, const float* __restrict__ r, const float* __restrict__ dinv, float* z,
                      const SolveScalars* sc) {
  if (solve_done(sc)) return;
  MG_STRIDE(i, n) z[i] = kOmega * (dinv[i] * r[i]);
}

// 27-point product at cell (k, j, i) of a level.
__device__ __forceinline__ float apply27(const Dims& d, const float* __restrict__ A, const float* __restrict__ z,
                                         long long c, int k, int j, int i) {
  float s = 0.0f;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int kn = k + o / 9 - 1, jn = j + (o / 3) % 3 - 1, in = i + o % 3 - 1;
    if (kn < 0 || kn >= d.nz || jn < 0 || jn >= d.ny || in < 0 || in >= d.nx) continue;
    const long long nb = c + ((long long)(o / 9 - 1) * d.ny + ((o / 3) % 3 - 1)) * d.nx + (o % 3 - 1);
    s += A[o * d.n + c] * z[nb];
  }
  return s;
}

// r_c = P^T (r - q) on level 0 (q = A' z; only reduced unknowns).
__global__ void k_restrict0(Dims f, Dims c, const float* __restrict__ r, const float* __restrict__ q,
                            const unsigned char* __restrict__ reduced, float* rc, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  MG_STRIDE(B, c.n) {
    const int I = (int)(B % c.nx);
    const long long rr = B / c.nx;
    const int J = (int)(rr % c.ny), K = (int)(rr / c.ny);
    float s = 0.0f;
    for (int kk = 0; kk < 2; ++kk)
      for (int jj = 0; jj < 2; ++jj)
        for (int ii = 0; ii < 2; ++ii) {
          const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
          if (k >= f.nz || j >= f.ny || i >= f.nx) continue;
          const long long cidx = ((long long)k * f.ny + j) * f.nx + i;
          if (reduced[cidx]) s += r[cidx] - q[cidx];
        }
    rc[B] = s;
  }
}

// r_c = P^T (r - A z) on a coarse level.
__global__ void k_resid_restrict(Dims f, Dims c, const float* __restrict__ A, const float* __restrict__ r,
                                 const float* __restrict__ z, float* rc, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  MG_STRIDE(B, c.n) {
    const int I = (int)(B % c.nx);
    const long long rr = B / c.nx;
    const int J = (int)(rr % c.ny), K = (int)(rr / c.ny);
    float s = 0.0f;
    for (int kk = 0; kk < 2; ++kk)
      for (int jj = 0; jj < 2; ++jj)
        for (int ii = 0; ii < 2; ++ii) {
          const int k = 2 * K + kk, j = 2 * J + jj, i = 2 * I + ii;
          if (k >= f.nz || j >= f.ny || i >= f.nx) continue;
          const long long cidx = ((long long)k * f.ny + j) * f.nx + i;
          s += r[cidx] - apply27(f, A, z, cidx, k, j, i);
        }
    rc[B] = s;
  }
}

// z += P z_c (on level 0 only where mask, the reduced unknowns).
__global__ void k_prolong(Dims f, Dims c, const float* __restrict__ zc, float* z,
                          const unsigned char* __restrict__ mask, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  MG_STRIDE(idx, f.n) {
    if (mask && !mask[idx]) continue;
    const int i = (int)(idx % f.nx);
    const long long rr = idx / f.nx;
    const int j = (int)(rr % f.ny), k = (int)(rr / f.ny);
    z[idx] += zc[((long long)(k >> 1) * c.ny + (j >> 1)) * c.nx + (i >> 1)];
  }
}

// zout = z + omega D^-1 (r - A z) on a coarse level.
__global__ void k_post(Dims d, const float* __restrict__ A, const float* __restrict__ dinv,
                       const float* __restrict__ r, const float* __restrict__ z, float* zout,
                       const SolveScalars* sc) {
  if (solve_done(sc)) return;
  MG_STRIDE(idx, d.n) {
    const int i = (int)(idx % d.nx);
    const long long rr = idx / d.nx;
    const int j = (int)(rr % d.ny), k = (int)(rr / d.ny);
    zout[idx] = z[idx] + kOmega * (dinv[idx] * (r[idx] - apply27(d, A, z, idx, k, j, i)));
  }
}

// z += omega D^-1 (r - q) on level 0 (q = A' z).
__global__ void k_post0(long long n, const float* __restrict__ dinv, const float* __restrict__ r,
                        const float* __restrict__ q, float* z, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  MG_STRIDE(i, n) z[i] += kOmega * (dinv[i] * (r[i] - q[i]));
}

// z = M r with the dense coarsest inverse (column-major), in FP64: the
// coarsest matrix of a 1000:1 two-fluid problem is too ill-conditioned for
// an FP32 inverse.
__global__ void k_dense(int N, const double* __restrict__ minv, const float* __restrict__ r, float* z,
                        const SolveScalars* sc) {
  if (solve_done(sc)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int jcol = 0; jcol < N; ++jcol) s += minv[(long long)jcol * N + i] * (double)r[jcol];
  z[i] = (float)s;
}

struct Level {
  Dims d;
  DevBuf A64, A32, dinv, r, z, zt;
};

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

}  // namespace
}  // namespace nfa

using namespace nfa;

struct nfa_mg_s {
  Poisson* op = nullptr;
  int L = 0;                    // levels including level 0
  Level lv[kMaxLevels];         // lv[0]: dims only
  DevBuf q0, group_of, minv;
  int ncoarse = 0;
  int built_version = -1;       // op->version the coarse operators belong to
};

namespace nfa {

nfa_status mg_setup(nfa_mg_s& mg, hipStream_t st) {
  Poisson& op = *mg.op;
  Grid& g = *op.g;
  if (!op.assembled) return fail(NFA_ERR_INVALID, "multigrid: operator not assembled");
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
                                                     C.A64.as<double>(), C.A32.as<float>(), C.dinv.as<float>());
    else
      k_coarsen<<<blocks_for(C.d.n), kBlock, 0, st>>>(mg.lv[l - 1].d, C.d, mg.lv[l - 1].A64.as<double>(),
                                                      C.A64.as<double>(), C.A32.as<float>(), C.dinv.as<float>());
    NFA_CHECK_LAUNCH();
  }
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
  // M is symmetric: its column-major and row-major layouts agree
  NFA_HIP(hipMemcpyAsync(mg.minv.p, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, st));
  NFA_HIP(hipStreamSynchronize(st));
  mg.built_version = op.version;
  return NFA_OK;
}

// One V-cycle: z = M r on the reduced unknowns of level 0 (FP32).
nfa_status mg_vcycle(nfa_mg_s& mg, const float* r0, float* z0, const SolveScalars* sc, hipStream_t st) {
  Poisson& op = *mg.op;
  Grid& g = *op.g;
  const Coeffs<float> c32 = op.c32();
  float* q0 = mg.q0.as<float>();
  const unsigned char* red = g.reduced.as<unsigned char>();
  const Dims d0 = mg.lv[0].d;
  auto apply0 = [&](float* z) {   // q0 = A' z (z's slaves take their root's value)
    launch_merge_copy<float>(g, z, st, sc);
    launch_stencil<float>(g, c32, z, nullptr, q0, nullptr, sc, ST_APPLY, st);
    launch_merge_gather<float>(g, q0, st, sc);
  };
  // downward
  k_pre<<<blocks_for(d0.n), kBlock, 0, st>>>(d0.n, r0, c32.dinv, z0, sc);
  apply0(z0);
  k_restrict0<<<blocks_for(mg.lv[1].d.n), kBlock, 0, st>>>(d0, mg.lv[1].d, r0, q0, red, mg.lv[1].r.as<float>(), sc);
  for (int l = 1; l < mg.L - 1; ++l) {
    Level& F = mg.lv[l];
    Level& C = mg.lv[l + 1];
    k_pre<<<blocks_for(F.d.n), kBlock, 0, st>>>(F.d.n, F.r.as<float>(), F.dinv.as<float>(), F.z.as<float>(), sc);
    k_resid_restrict<<<blocks_for(C.d.n), kBlock, 0, st>>>(F.d, C.d, F.A32.as<float>(), F.r.as<float>(),
                                                            F.z.as<float>(), C.r.as<float>(), sc);
  }
  Level& Z = mg.lv[mg.L - 1];
  k_dense<<<(int)((Z.d.n + 255) / 256), 256, 0, st>>>((int)Z.d.n, mg.minv.as<double>(), Z.r.as<float>(),
                                                      Z.zt.as<float>(), sc);
  // upward: each level's corrected z ends in zt
  for (int l = mg.L - 2; l >= 1; --l) {
    Level& F = mg.lv[l];
    Level& C = mg.lv[l + 1];
    k_prolong<<<blocks_for(F.d.n), kBlock, 0, st>>>(F.d, C.d, C.zt.as<float>(), F.z.as<float>(), nullptr, sc);
    k_post<<<blocks_for(F.d.n), kBlock, 0, st>>>(F.d, F.A32.as<float>(), F.dinv.as<float>(), F.r.as<float>(),
                                                 F.z.as<float>(), F.zt.as<float>(), sc);
  }
  k_prolong<<<blocks_for(d0.n), kBlock, 0, st>>>(d0, mg.lv[1].d, mg.lv[1].zt.as<float>(), z0, red, sc);
  apply0(z0);
  k_post0<<<blocks_for(d0.n), kBlock, 0, st>>>(d0.n, c32.dinv, r0, q0, z0, sc);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

nfa_status mg_precond_apply(void* mgh, Poisson& op, const float* r, float* z, const SolveScalars* sc,
                            hipStream_t st) {
  if (!mgh) return fail(NFA_ERR_INVALID, "multigrid preconditioner: no handle");
  nfa_mg_s& mg = *static_cast<nfa_mg_s*>(mgh);
  if (mg.op != &op) return fail(NFA_ERR_INVALID, "multigrid preconditioner: built for another operator");
  if (mg.built_version != op.version) return fail(NFA_ERR_INVALID, "multigrid preconditioner: not set up");
  return mg_vcycle(mg, r, z, sc, st);
}

nfa_status mg_ensure(void* mgh, Poisson& op, hipStream_t st) {
  if (!mgh) return fail(NFA_ERR_INVALID, "multigrid preconditioner: no handle");
  nfa_mg_s& mg = *static_cast<nfa_mg_s*>(mgh);
  if (mg.op != &op) return fail(NFA_ERR_INVALID, "multigrid preconditioner: built for another operator");
  return mg.built_version == op.version ? NFA_OK : mg_setup(mg, st);
}

}  // namespace nfa

extern "C" nfa_status nfa_mg_create(nfa_poisson op, nfa_mg* out) {
  if (!out) return fail(NFA_ERR_INVALID, "nfa_mg_create: out is NULL");
  *out = nullptr;
  if (!op) return fail(NFA_ERR_INVALID, "nfa_mg_create: NULL operator");
  auto* mg = new nfa_mg_s();
  mg->op = op;
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
  if ((e = mg->q0.alloc(g.n * 4)) != hipSuccess || (e = mg->group_of.alloc(g.n * 4)) != hipSuccess) return bad(e);
  for (int l = 1; l < mg->L; ++l) {
    Level& C = mg->lv[l];
    const size_t n = (size_t)C.d.n;
    if ((e = C.A64.alloc(27 * n * 8)) != hipSuccess || (e = C.A32.alloc(27 * n * 4)) != hipSuccess ||
        (e = C.dinv.alloc(n * 4)) != hipSuccess || (e = C.r.alloc(n * 4)) != hipSuccess ||
        (e = C.z.alloc(n * 4)) != hipSuccess || (e = C.zt.alloc(n * 4)) != hipSuccess)
      return bad(e);
  }
  mg->ncoarse = (int)mg->lv[mg->L - 1].d.n;
  if ((e = mg->minv.alloc((size_t)mg->ncoarse * mg->ncoarse * 8)) != hipSuccess) return bad(e);
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
  if (mg->built_version != mg->op->version)
    return fail(NFA_ERR_INVALID, "nfa_mg_apply: call nfa_mg_setup after the last assembly");
  const nfa_status e = mg_vcycle(*mg, r, z, nullptr, S(s));
  if (e != NFA_OK) return e;
  launch_merge_copy<float>(*mg->op->g, z, S(s), nullptr);
  NFA_CHECK_LAUNCH();
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
