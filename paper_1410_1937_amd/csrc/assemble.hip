// libnfa: operator handle, coefficient assembly, right-hand side, projection
// and divergence.
//
// eq. density and Density Smoothing: rho = rho_g + (rho_l - rho_g) clip(phi),
// optionally smoothed (1/4, 1/2, 1/4) along x, then y, then z (mirrored ends).
// eq. integral2: T_f = (open area_f * beta_f) / h_f with beta_f = 2/(rho_L +
// rho_R) inside and 1/rho_c on a Dirichlet boundary face (h = half width);
// Neumann faces carry T = 0.  The Jacobi inverse diagonal is that of the
// merged operator: a group's diagonal sums T over its members' faces that
// lead out of the group.  Built with -ffp-contract=off: every value here is
// bitwise the expression written.
#include <cmath>

#include <string>

#include "device_util.h"

#include "nfa_internal.h"
#include "vecops.h"

namespace nfa {
namespace {

#define GRID_STRIDE(idx, n) \
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (n); idx += (long long)gridDim.x * blockDim.x)

template <class P>
__device__ __forceinline__ double rho_of(const P* phi, long long c, double rl, double rg) {
  double h = (double)phi[c];
  h = fmin(fmax(h, 0.0), 1.0);
  return rg + (rl - rg) * h;
}

template <class P>
__global__ void k_density_x(int nx, int ny, int nz, const P* phi, double rl, double rg, int smooth,
                            double* out) {
  const long long n = (long long)nx * ny * nz;
  GRID_STRIDE(c, n) {
    const int i = (int)(c % nx);
    const double b = rho_of(phi, c, rl, rg);
    if (!smooth) { out[c] = b; continue; }
    const double a = i > 0 ? rho_of(phi, c - 1, rl, rg) : b;
    const double d = i < nx - 1 ? rho_of(phi, c + 1, rl, rg) : b;
    out[c] = (0.25 * a + 0.5 * b) + 0.25 * d;
  }
}

// smoothing along y (stride nx) or z (stride nx*ny)
__global__ void k_smooth(int nx, int ny, int nz, int axis, const double* in, double* out) {
  const long long n = (long long)nx * ny * nz;
  const long long stride = axis == 1 ? nx : (long long)nx * ny;
  GRID_STRIDE(c, n) {
    int pos, len;
    if (axis == 1) { pos = (int)((c / nx) % ny); len = ny; }
    else { pos = (int)(c / ((long long)nx * ny)); len = nz; }
    const double b = in[c];
    const double a = pos > 0 ? in[c - stride] : b;
    const double d = pos < len - 1 ? in[c + stride] : b;
    out[c] = (0.25 * a + 0.5 * b) + 0.25 * d;
  }
}

struct BC6 { int b[6]; };

// lower-face coefficients of every cell, boundary planes, Jacobi inverse of
// unmerged cells
__global__ void k_coeff(int nx, int ny, int nz, BC6 bc, const double* rho, const double* ox,
                        const double* oy, const double* oz, const double* hx, const double* hy,
                        const double* hz, const unsigned char* red, double* tx, double* txb,
                        double* ty, double* tz, double* dinv, float* tx32, float* txb32,
                        float* ty32, float* tz32, float* dinv32) {
  const long long n = (long long)nx * ny * nz;
  const long long plane = (long long)nx * ny;
  GRID_STRIDE(c, n) {
    const int i = (int)(c % nx);
    const long long r = c / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const double rc = rho[c];
    const long long fx = ((long long)k * ny + j) * (nx + 1) + i;
    const long long fy = ((long long)k * (ny + 1) + j) * nx + i;
    const long long fz = c;
    // x- face (face i)
    double txm;
    if (i > 0) txm = (ox[fx] * (2.0 / (rho[c - 1] + rc))) / hx[i];
    else txm = bc.b[0] ? (ox[fx] * (1.0 / rc)) / hx[0] : 0.0;
    // x+ face (face i+1)
    double txp;
    if (i < nx - 1) txp = (ox[fx + 1] * (2.0 / (rc + rho[c + 1]))) / hx[i + 1];
    else txp = bc.b[1] ? (ox[fx + 1] * (1.0 / rc)) / hx[nx] : 0.0;
    double tym;
    if (j > 0) tym = (oy[fy] * (2.0 / (rho[c - nx] + rc))) / hy[j];
    else tym = bc.b[2] ? (oy[fy] * (1.0 / rc)) / hy[0] : 0.0;
    double typ;
    if (j < ny - 1) typ = (oy[fy + nx] * (2.0 / (rc + rho[c + nx]))) / hy[j + 1];
    else typ = bc.b[3] ? (oy[fy + nx] * (1.0 / rc)) / hy[ny] : 0.0;
    double tzm;
    if (k > 0) tzm = (oz[fz] * (2.0 / (rho[c - plane] + rc))) / hz[k];
    else tzm = bc.b[4] ? (oz[fz] * (1.0 / rc)) / hz[0] : 0.0;
    double tzp;
    if (k < nz - 1) tzp = (oz[fz + plane] * (2.0 / (rc + rho[c + plane]))) / hz[k + 1];
    else tzp = bc.b[5] ? (oz[fz + plane] * (1.0 / rc)) / hz[nz] : 0.0;
    tx[c] = txm;
    tx32[c] = (float)txm;
    ty[fy] = tym;
    ty32[fy] = (float)tym;
    tz[fz] = tzm;
    tz32[fz] = (float)tzm;
    if (i == nx - 1) { txb[(long long)k * ny + j] = txp; txb32[(long long)k * ny + j] = (float)txp; }
    if (j == ny - 1) { ty[fy + nx] = typ; ty32[fy + nx] = (float)typ; }
    if (k == nz - 1) { tz[fz + plane] = tzp; tz32[fz + plane] = (float)tzp; }
    const double d = ((((txm + txp) + tym) + typ) + tzm) + tzp;
    const double di = (red[c] && d > 0) ? 1.0 / d : 0.0;
    dinv[c] = di;
    dinv32[c] = (float)di;
  }
}

// Jacobi diagonal of a merge group: members root, then slaves ascending;
// faces x-, x+, y-, y+, z-, z+; faces whose neighbour is in the group drop out.
__global__ void k_dinv_groups(int nx, int ny, int nz, int ng, const int* g_root, const int* g_off,
                              const int* g_mem, const double* tx, const double* txb,
                              const double* ty, const double* tz, double* dinv, float* dinv32) {
  const long long plane = (long long)nx * ny;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ng; t += gridDim.x * blockDim.x) {
    const int r = g_root[t];
    const int m0 = g_off[t], m1 = g_off[t + 1];
    double acc = 0.0;
    bool first = true;
    for (int q = -1; q < m1 - m0; ++q) {
      const long long m = q < 0 ? r : g_mem[m0 + q];
      const int i = (int)(m % nx);
      const long long rr = m / nx;
      const int j = (int)(rr % ny), k = (int)(rr / ny);
      const long long fy = ((long long)k * (ny + 1) + j) * nx + i;
      const double tv[6] = {tx[m], i < nx - 1 ? tx[m + 1] : txb[(long long)k * ny + j], ty[fy],
                            ty[fy + nx], tz[m], tz[m + plane]};
      const long long nb[6] = {i > 0 ? m - 1 : -1, i < nx - 1 ? m + 1 : -1,
                               j > 0 ? m - nx : -1, j < ny - 1 ? m + nx : -1,
                               k > 0 ? m - plane : -1, k < nz - 1 ? m + plane : -1};
      for (int f = 0; f < 6; ++f) {
        bool inside = false;
        if (nb[f] >= 0) {
          inside = nb[f] == r;
          for (int u = m0; u < m1 && !inside; ++u) inside = nb[f] == g_mem[u];
        }
        if (inside) continue;
        acc = first ? tv[f] : acc + tv[f];
        first = false;
      }
    }
    const double di = acc > 0 ? 1.0 / acc : 0.0;
    dinv[r] = di;
    dinv32[r] = (float)di;
  }
}

// b = -((D F~) + B)/dt on active cells, 0 elsewhere
// (vbx, vby, vbz: per-cell body velocity, or NULL for the uniform (vx, vy, vz))
__global__ void k_rhs(int nx, int ny, int nz, const double* ox, const double* oy, const double* oz,
                      const double* u, const double* v, const double* w, double dt, double vx,
                      double vy, double vz, const double* vbx, const double* vby, const double* vbz,
                      const unsigned char* act, double* b) {
  const long long n = (long long)nx * ny * nz;
  const long long plane = (long long)nx * ny;
  GRID_STRIDE(c, n) {
    const int i = (int)(c % nx);
    const long long r = c / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const long long fx = ((long long)k * ny + j) * (nx + 1) + i;
    const long long fy = ((long long)k * (ny + 1) + j) * nx + i;
    const long long fz = c;
    const double fxm = ox[fx] * u[fx], fxp = ox[fx + 1] * u[fx + 1];
    const double fym = oy[fy] * v[fy], fyp = oy[fy + nx] * v[fy + nx];
    const double fzm = oz[fz] * w[fz], fzp = oz[fz + plane] * w[fz + plane];
    const double div = ((fxp - fxm) + (fyp - fym)) + (fzp - fzm);
    const double sx = -(ox[fx + 1] - ox[fx]);
    const double sy = -(oy[fy + nx] - oy[fy]);
    const double sz = -(oz[fz + plane] - oz[fz]);
    const double B = vbx ? (vbx[c] * sx + vby[c] * sy) + vbz[c] * sz : (vx * sx + vy * sy) + vz * sz;
    b[c] = act[c] ? -(div + B) / dt : 0.0;
  }
}

// merged divergence (before gather): (D F + B) on active cells
__global__ void k_div(int nx, int ny, int nz, const double* ox, const double* oy, const double* oz,
                      const double* fu, const double* fv, const double* fw, double vx, double vy,
                      double vz, const unsigned char* act, double* out) {
  const long long n = (long long)nx * ny * nz;
  const long long plane = (long long)nx * ny;
  GRID_STRIDE(c, n) {
    const int i = (int)(c % nx);
    const long long r = c / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const long long fx = ((long long)k * ny + j) * (nx + 1) + i;
    const long long fy = ((long long)k * (ny + 1) + j) * nx + i;
    const long long fz = c;
    const double div = ((fu[fx + 1] - fu[fx]) + (fv[fy + nx] - fv[fy])) + (fw[fz + plane] - fw[fz]);
    const double sx = -(ox[fx + 1] - ox[fx]);
    const double sy = -(oy[fy + nx] - oy[fy]);
    const double sz = -(oz[fz + plane] - oz[fz]);
    const double B = (vx * sx + vy * sy) + vz * sz;
    out[c] = act[c] ? div + B : 0.0;
  }
}

// F = open*u - dt*(T*(p_+ - p_-)) on the three face sets
__global__ void k_project(int nx, int ny, int nz, const double* ox, const double* oy,
                          const double* oz, const double* tx, const double* txb, const double* ty,
                          const double* tz, const double* u, const double* v, const double* w,
                          const double* p, double dt, double* fu, double* fv, double* fw) {
  const long long plane = (long long)nx * ny;
  const long long nfx = (long long)nz * ny * (nx + 1);
  const long long nfy = (long long)nz * (ny + 1) * nx;
  const long long nfz = (long long)(nz + 1) * ny * nx;
  GRID_STRIDE(f, nfx + nfy + nfz) {
    if (f < nfx) {
      const int i = (int)(f % (nx + 1));
      const long long r = f / (nx + 1);
      const int j = (int)(r % ny), k = (int)(r / ny);
      const long long c = ((long long)k * ny + j) * nx + i;
      const double pm = i > 0 ? p[c - 1] : 0.0;
      const double pp = i < nx ? p[c] : 0.0;
      const double t = i < nx ? tx[c] : txb[(long long)k * ny + j];
      fu[f] = ox[f] * u[f] - dt * (t * (pp - pm));
    } else if (f < nfx + nfy) {
      const long long g = f - nfx;
      const int i = (int)(g % nx);
      const long long r = g / nx;
      const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
      const long long c = ((long long)k * ny + j) * nx + i;
      const double pm = j > 0 ? p[c - nx] : 0.0;
      const double pp = j < ny ? p[c] : 0.0;
      fv[g] = oy[g] * v[g] - dt * (ty[g] * (pp - pm));
    } else {
      const long long g = f - nfx - nfy;
      const int k = (int)(g / plane);
      const double pm = k > 0 ? p[g - plane] : 0.0;
      const double pp = k < nz ? p[g] : 0.0;
      fw[g] = oz[g] * w[g] - dt * (tz[g] * (pp - pm));
    }
  }
}

// lower-face x array (+ boundary plane) -> natural x-face layout
template <class T>
__global__ void k_export_tx(int nx, int ny, int nz, const T* tx, const T* txb, T* out) {
  const long long n = (long long)nz * ny * (nx + 1);
  GRID_STRIDE(f, n) {
    const int i = (int)(f % (nx + 1));
    const long long r = f / (nx + 1);
    out[f] = i < nx ? tx[r * nx + i] : txb[r];
  }
}

template <class T>
__global__ void k_copy(long long n, const T* a, T* b) {
  GRID_STRIDE(i, n) b[i] = a[i];
}

}  // namespace
}  // namespace nfa

using namespace nfa;

namespace nfa {
namespace {
// Every device buffer of an operator: coefficients in both precisions and the
// work vectors of the FP64 and FP32 solvers, in one fixed order.
hipError_t poisson_buffers(Poisson& op, const Grid& g, Carver& c) {
  const long long n = g.n;
  const long long nzy = (long long)g.nz * g.ny;
  hipError_t e = hipSuccess;
  DevBuf* f64[] = {&op.rho, &op.rho_tmp, &op.tx64, &op.dinv64, &op.r, &op.z, &op.p, &op.p2, &op.p3, &op.q, &op.tmp};
  for (DevBuf* b : f64)
    if ((e = c.take(*b, n * 8)) != hipSuccess) return e;
  if ((e = c.take(op.txb64, nzy * 8)) != hipSuccess || (e = c.take(op.ty64, g.nfy() * 8)) != hipSuccess ||
      (e = c.take(op.tz64, g.nfz() * 8)) != hipSuccess)
    return e;
  DevBuf* f32[] = {&op.tx32, &op.dinv32, &op.x32, &op.r32, &op.z32, &op.p32, &op.p32b, &op.p32c, &op.q32};
  for (DevBuf* b : f32)
    if ((e = c.take(*b, n * 4)) != hipSuccess) return e;
  if ((e = c.take(op.txb32, nzy * 4)) != hipSuccess || (e = c.take(op.ty32, g.nfy() * 4)) != hipSuccess ||
      (e = c.take(op.tz32, g.nfz() * 4)) != hipSuccess)
    return e;
  if ((e = c.take(op.partials, (size_t)kMaxPartials * 4 * 8)) != hipSuccess ||
      (e = c.take(op.scal, 4 * sizeof(SolveScalars))) != hipSuccess ||
      (e = c.take(op.hist, (size_t)(kHistCap + 2) * 8)) != hipSuccess)
    return e;
  return hipSuccess;
}
}  // namespace
}  // namespace nfa

extern "C" size_t nfa_poisson_workspace_bytes(nfa_grid g) {
  if (!g) return 0;
  Poisson tmp;
  Carver c;
  c.measure = true;
  (void)poisson_buffers(tmp, *g, c);
  return c.used;
}

extern "C" nfa_status nfa_poisson_create(nfa_grid g, void* workspace, size_t ws_bytes, nfa_poisson* out) {
  if (!g || !out) return fail(NFA_ERR_INVALID, "nfa_poisson_create: NULL argument");
  *out = nullptr;
  // one FP64 partial per 64x4 column tile of the stencil sweep (z chunks are
  // enlarged until the count fits)
  if ((long long)((g->nx + 63) / 64) * ((g->ny + 3) / 4) > kMaxPartials)
    return fail(NFA_ERR_INVALID, "nfa_poisson_create: nx*ny too large for the reduction buffer");
  if (workspace) {
    const size_t need = nfa_poisson_workspace_bytes(g);
    if (ws_bytes < need)
      return fail(NFA_ERR_NOMEM, "nfa_poisson_create: workspace of " + std::to_string(ws_bytes) +
                                     " bytes, the operator needs " + std::to_string(need));
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
      return fail(NFA_ERR_INVALID, "nfa_poisson_create: workspace must be 256-byte aligned");
  }
  auto* op = new nfa_poisson_s();
  op->g = g;
  auto bad = [&](hipError_t e) {
    delete op;
    return fail(NFA_ERR_HIP, std::string("nfa_poisson_create: ") + hipGetErrorString(e));
  };
  Carver c;
  c.base = static_cast<unsigned char*>(workspace);
  c.cap = ws_bytes;
  hipError_t e = poisson_buffers(*op, *g, c);
  if (e != hipSuccess) return bad(e);
  if ((e = hipHostMalloc((void**)&op->h_scal, 2 * sizeof(SolveScalars), hipHostMallocDefault)) != hipSuccess)
    return bad(e);
  for (int i = 0; i < 2; ++i)
    if ((e = hipEventCreateWithFlags(&op->ev[i], hipEventDisableTiming)) != hipSuccess) return bad(e);
  *out = op;
  return NFA_OK;
}

extern "C" void nfa_poisson_destroy(nfa_poisson op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  if (op->h_scal) (void)hipHostFree(op->h_scal);
  for (int i = 0; i < 2; ++i)
    if (op->ev[i]) (void)hipEventDestroy(op->ev[i]);
  for (auto e : op->prof_ev)
    if (e) (void)hipEventDestroy(e);
  delete op;
}

extern "C" nfa_status nfa_poisson_assemble(nfa_poisson op, const void* phi,
                                           const nfa_assemble_params* prm, nfa_stream s) {
  if (!op || !phi || !prm) return fail(NFA_ERR_INVALID, "nfa_poisson_assemble: NULL argument");
  if (prm->phi_dtype != NFA_F64 && prm->phi_dtype != NFA_F32)
    return fail(NFA_ERR_INVALID, "nfa_poisson_assemble: phi_dtype must be NFA_F64 or NFA_F32");
  if (!(prm->rho_liquid > 0) || !(prm->rho_gas > 0))
    return fail(NFA_ERR_INVALID, "nfa_poisson_assemble: densities must be positive");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const int nb = blocks_for(g.n);
  double* rho = op->rho.as<double>();
  double* tmp = op->rho_tmp.as<double>();
  if (prm->phi_dtype == NFA_F64)
    k_density_x<double><<<nb, kBlock, 0, st>>>(g.nx, g.ny, g.nz, (const double*)phi, prm->rho_liquid,
                                               prm->rho_gas, prm->smooth, rho);
  else
    k_density_x<float><<<nb, kBlock, 0, st>>>(g.nx, g.ny, g.nz, (const float*)phi, prm->rho_liquid,
                                              prm->rho_gas, prm->smooth, rho);
  if (prm->smooth) {
    k_smooth<<<nb, kBlock, 0, st>>>(g.nx, g.ny, g.nz, 1, rho, tmp);
    k_smooth<<<nb, kBlock, 0, st>>>(g.nx, g.ny, g.nz, 2, tmp, rho);
  }
  BC6 bc;
  for (int f = 0; f < 6; ++f) bc.b[f] = g.bc[f];
  k_coeff<<<nb, kBlock, 0, st>>>(g.nx, g.ny, g.nz, bc, rho, g.open_x.as<double>(),
                                 g.open_y.as<double>(), g.open_z.as<double>(), g.d_hx.as<double>(),
                                 g.d_hy.as<double>(), g.d_hz.as<double>(),
                                 g.reduced.as<unsigned char>(), op->tx64.as<double>(),
                                 op->txb64.as<double>(), op->ty64.as<double>(), op->tz64.as<double>(),
                                 op->dinv64.as<double>(), op->tx32.as<float>(), op->txb32.as<float>(),
                                 op->ty32.as<float>(), op->tz32.as<float>(), op->dinv32.as<float>());
  if (g.n_groups > 0)
    k_dinv_groups<<<blocks_for(g.n_groups), kBlock, 0, st>>>(
        g.nx, g.ny, g.nz, g.n_groups, g.g_root.as<int>(), g.g_off.as<int>(), g.g_mem.as<int>(),
        op->tx64.as<double>(), op->txb64.as<double>(), op->ty64.as<double>(), op->tz64.as<double>(),
        op->dinv64.as<double>(), op->dinv32.as<float>());
  NFA_CHECK_LAUNCH();
  op->assembled = true;
  op->version += 1;
  op->body_version = g.body_version;
  return NFA_OK;
}

extern "C" nfa_status nfa_poisson_apply(nfa_poisson op, const void* x, void* y, int dtype,
                                        nfa_stream s) {
  if (!op || !x || !y) return fail(NFA_ERR_INVALID, "nfa_poisson_apply: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_poisson_apply")) return e;
  if (x == y) return fail(NFA_ERR_INVALID, "nfa_poisson_apply: x and y must not overlap");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  if (dtype == NFA_F64) {
    const double* src = (const double*)x;
    if (g.n_slaves > 0) {
      k_copy<double><<<blocks_for(g.n), kBlock, 0, st>>>(g.n, src, op->tmp.as<double>());
      launch_merge_copy<double>(g, op->tmp.as<double>(), st, nullptr);
      src = op->tmp.as<double>();
    }
    launch_stencil<double>(g, op->c64(), src, nullptr, (double*)y, st);
    launch_merge_gather<double>(g, (double*)y, st, nullptr);
  } else if (dtype == NFA_F32) {
    const float* src = (const float*)x;
    if (g.n_slaves > 0) {
      k_copy<float><<<blocks_for(g.n), kBlock, 0, st>>>(g.n, src, op->tmp.as<float>());
      launch_merge_copy<float>(g, op->tmp.as<float>(), st, nullptr);
      src = op->tmp.as<float>();
    }
    launch_stencil<float>(g, op->c32(), src, nullptr, (float*)y, st);
    launch_merge_gather<float>(g, (float*)y, st, nullptr);
  } else {
    return fail(NFA_ERR_INVALID, "nfa_poisson_apply: dtype must be NFA_F64 or NFA_F32");
  }
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

namespace {
nfa_status rhs_impl(nfa_poisson op, const double* u, const double* v, const double* w, double dt,
                    const double* vel, const double* vbx, const double* vby, const double* vbz,
                    double* b, nfa_stream s, const char* who) {
  if (!op || !u || !v || !w || !b) return fail(NFA_ERR_INVALID, std::string(who) + ": NULL argument");
  if (!(dt > 0)) return fail(NFA_ERR_INVALID, std::string(who) + ": dt must be > 0");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const double vx = vel ? vel[0] : 0.0, vy = vel ? vel[1] : 0.0, vz = vel ? vel[2] : 0.0;
  k_rhs<<<blocks_for(g.n), kBlock, 0, st>>>(g.nx, g.ny, g.nz, g.open_x.as<double>(),
                                            g.open_y.as<double>(), g.open_z.as<double>(), u, v, w, dt,
                                            vx, vy, vz, vbx, vby, vbz, g.active.as<unsigned char>(), b);
  launch_merge_gather<double>(g, b, st, nullptr);
  if (g.all_neumann() && g.n_reduced > 0) {
    double* parts = op->partials.as<double>();
    const int np = launch_masked_sum<double>(b, g.reduced.as<unsigned char>(), g.n, parts, st);
    double* sum = parts + (size_t)kMaxPartials * 3;
    launch_sum_partials(parts, np, 1, sum, st);
    launch_sub_mean(b, g.reduced.as<unsigned char>(), g.n, sum, (double)g.n_reduced, st);
  }
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}
}  // namespace

extern "C" nfa_status nfa_poisson_rhs(nfa_poisson op, const double* u, const double* v,
                                      const double* w, double dt, const double* vel, double* b,
                                      nfa_stream s) {
  return rhs_impl(op, u, v, w, dt, vel, nullptr, nullptr, nullptr, b, s, "nfa_poisson_rhs");
}

extern "C" nfa_status nfa_poisson_rhs_cells(nfa_poisson op, const double* u, const double* v,
                                            const double* w, double dt, const double* vbx,
                                            const double* vby, const double* vbz, double* b,
                                            nfa_stream s) {
  if (!vbx || !vby || !vbz) return fail(NFA_ERR_INVALID, "nfa_poisson_rhs_cells: NULL body velocity");
  return rhs_impl(op, u, v, w, dt, nullptr, vbx, vby, vbz, b, s, "nfa_poisson_rhs_cells");
}

extern "C" nfa_status nfa_poisson_project(nfa_poisson op, const double* u, const double* v,
                                          const double* w, const double* p, double dt, double* fu,
                                          double* fv, double* fw, nfa_stream s) {
  if (!op || !u || !v || !w || !p || !fu || !fv || !fw)
    return fail(NFA_ERR_INVALID, "nfa_poisson_project: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_poisson_project")) return e;
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const double* src = p;
  if (g.n_slaves > 0) {
    k_copy<double><<<blocks_for(g.n), kBlock, 0, st>>>(g.n, p, op->tmp.as<double>());
    launch_merge_copy<double>(g, op->tmp.as<double>(), st, nullptr);
    src = op->tmp.as<double>();
  }
  k_project<<<blocks_for(g.nfx() + g.nfy() + g.nfz()), kBlock, 0, st>>>(
      g.nx, g.ny, g.nz, g.open_x.as<double>(), g.open_y.as<double>(), g.open_z.as<double>(),
      op->tx64.as<double>(), op->txb64.as<double>(), op->ty64.as<double>(), op->tz64.as<double>(), u,
      v, w, src, dt, fu, fv, fw);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_poisson_divergence(nfa_poisson op, const double* fu, const double* fv,
                                             const double* fw, const double* vel, double* div,
                                             nfa_stream s) {
  if (!op || !fu || !fv || !fw || !div) return fail(NFA_ERR_INVALID, "nfa_poisson_divergence: NULL argument");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const double vx = vel ? vel[0] : 0.0, vy = vel ? vel[1] : 0.0, vz = vel ? vel[2] : 0.0;
  k_div<<<blocks_for(g.n), kBlock, 0, st>>>(g.nx, g.ny, g.nz, g.open_x.as<double>(),
                                            g.open_y.as<double>(), g.open_z.as<double>(), fu, fv, fw,
                                            vx, vy, vz, g.active.as<unsigned char>(), div);
  launch_merge_gather<double>(g, div, st, nullptr);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_poisson_export(nfa_poisson op, int what, void* dst, nfa_stream s) {
  if (!op || !dst) return fail(NFA_ERR_INVALID, "nfa_poisson_export: NULL argument");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const DevBuf* b = nullptr;
  switch (what) {
    case NFA_EXPORT_RHO: b = &op->rho; break;
    case NFA_EXPORT_TY: b = &op->ty64; break;
    case NFA_EXPORT_TZ: b = &op->tz64; break;
    case NFA_EXPORT_DINV: b = &op->dinv64; break;
    case NFA_EXPORT_TY32: b = &op->ty32; break;
    case NFA_EXPORT_TZ32: b = &op->tz32; break;
    case NFA_EXPORT_DINV32: b = &op->dinv32; break;
    case NFA_EXPORT_TX:
      k_export_tx<double><<<blocks_for(g.nfx()), kBlock, 0, st>>>(
          g.nx, g.ny, g.nz, op->tx64.as<double>(), op->txb64.as<double>(), (double*)dst);
      NFA_CHECK_LAUNCH();
      return NFA_OK;
    case NFA_EXPORT_TX32:
      k_export_tx<float><<<blocks_for(g.nfx()), kBlock, 0, st>>>(
          g.nx, g.ny, g.nz, op->tx32.as<float>(), op->txb32.as<float>(), (float*)dst);
      NFA_CHECK_LAUNCH();
      return NFA_OK;
    default: return fail(NFA_ERR_INVALID, "nfa_poisson_export: unknown item");
  }
  NFA_HIP(hipMemcpyAsync(dst, b->p, b->bytes, hipMemcpyDeviceToDevice, st));
  return NFA_OK;
}
