// libnfa: one cycle of the second-order Runge-Kutta projection
// (Numerical Time Integration, eqs. poisson1, runge1, poisson2, runge2).
//
//   stage 1:  u~1 = u^k + dt R;  solve with rho(phi^k);  u* = u~1 - dt beta grad P*
//   stage 2:  u~2 = (u* + u^k) + dt R;  solve with rho(phi*) (body flux 2v:
//             u~2 is a sum of two fields that each carry v on the body);
//             u^{k+1} = 1/2 (u~2 - dt beta grad P)
//
// The velocity update on a face is u~ - dt (g (p+ - p-)) with g = beta_f/h_f:
// beta_f = 2/(rho_L + rho_R) inside, 1/rho_c with the half width on a
// Dirichlet boundary face (p = 0 beyond it); g = 0 on Neumann boundary faces
// and on closed faces (zero open area), which keep their provisional
// velocity.  Built with -ffp-contract=off: bitwise the expressions written.
#include <cmath>

#include "device_util.h"
#include "nfa_internal.h"
#include "vecops.h"

namespace nfa {
namespace {

#define GRID_STRIDE(idx, n) \
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (n); idx += (long long)gridDim.x * blockDim.x)

struct BCs {
  int b[6];
};

__global__ void k_velocity(int nx, int ny, int nz, BCs bc, const double* __restrict__ rho,
                           const double* __restrict__ ox, const double* __restrict__ oy,
                           const double* __restrict__ oz, const double* __restrict__ hx,
                           const double* __restrict__ hy, const double* __restrict__ hz,
                           const double* ux, const double* uy, const double* uz,
                           const double* __restrict__ p, double dt, double scale, double* vx,
                           double* vy, double* vz) {
  const long long plane = (long long)nx * ny;
  const long long nfx = (long long)nz * ny * (nx + 1);
  const long long nfy = (long long)nz * (ny + 1) * nx;
  const long long nfz = (long long)(nz + 1) * ny * nx;
  GRID_STRIDE(f, nfx + nfy + nfz) {
    double gc = 0.0, pm = 0.0, pp = 0.0, ut;
    double* out;
    long long o;
    if (f < nfx) {
      const int i = (int)(f % (nx + 1));
      const long long r = f / (nx + 1);
      const int j = (int)(r % ny), k = (int)(r / ny);
      const long long c = ((long long)k * ny + j) * nx + i;
      if (i > 0) pm = p[c - 1];
      if (i < nx) pp = p[c];
      if (ox[f] > 0) {
        if (i > 0 && i < nx) gc = (2.0 / (rho[c - 1] + rho[c])) / hx[i];
        else if (i == 0) gc = bc.b[0] ? (1.0 / rho[c]) / hx[0] : 0.0;
        else gc = bc.b[1] ? (1.0 / rho[c - 1]) / hx[nx] : 0.0;
      }
      ut = ux[f];
      out = vx;
      o = f;
    } else if (f < nfx + nfy) {
      const long long g = f - nfx;
      const int i = (int)(g % nx);
      const long long r = g / nx;
      const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
      const long long c = ((long long)k * ny + j) * nx + i;
      if (j > 0) pm = p[c - nx];
      if (j < ny) pp = p[c];
      if (oy[g] > 0) {
        if (j > 0 && j < ny) gc = (2.0 / (rho[c - nx] + rho[c])) / hy[j];
        else if (j == 0) gc = bc.b[2] ? (1.0 / rho[c]) / hy[0] : 0.0;
        else gc = bc.b[3] ? (1.0 / rho[c - nx]) / hy[ny] : 0.0;
      }
      ut = uy[g];
      out = vy;
      o = g;
    } else {
      const long long g = f - nfx - nfy;
      const int k = (int)(g / plane);
      if (k > 0) pm = p[g - plane];
      if (k < nz) pp = p[g];
      if (oz[g] > 0) {
        if (k > 0 && k < nz) gc = (2.0 / (rho[g - plane] + rho[g])) / hz[k];
        else if (k == 0) gc = bc.b[4] ? (1.0 / rho[g]) / hz[0] : 0.0;
        else gc = bc.b[5] ? (1.0 / rho[g - plane]) / hz[nz] : 0.0;
      }
      ut = uz[g];
      out = vz;
      o = g;
    }
    double u = ut - dt * (gc * (pp - pm));
    if (scale != 1.0) u = scale * u;
    out[o] = u;
  }
}

template <bool SUM>
__global__ void k_combine(long long n, const double* a, const double* b, double s,
                          const double* __restrict__ c, double* out) {
  GRID_STRIDE(i, n) {
    if (SUM) out[i] = (a[i] + b[i]) + s * c[i];
    else out[i] = a[i] + s * c[i];
  }
}

// exit plane (x-face nx) of ut: the upwind update of uk there, u_e - c (u_e - u_i)
__global__ void k_exit(int nx, long long nrow, const double* __restrict__ uk, double c, double* ut) {
  GRID_STRIDE(r, nrow) {
    const long long f = r * (nx + 1) + nx;
    const double ue = uk[f], ui = uk[f - 1];
    ut[f] = ue - c * (ue - ui);
  }
}

bool three(const void* const* v) { return v && v[0] && v[1] && v[2]; }

}  // namespace
}  // namespace nfa

using namespace nfa;

extern "C" nfa_status nfa_poisson_velocity(nfa_poisson op, const double* ut_x, const double* ut_y,
                                           const double* ut_z, const double* p, double dt,
                                           double scale, double* u_x, double* u_y, double* u_z,
                                           nfa_stream s) {
  if (!op || !ut_x || !ut_y || !ut_z || !p || !u_x || !u_y || !u_z)
    return fail(NFA_ERR_INVALID, "nfa_poisson_velocity: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_poisson_velocity")) return e;
  if (!(dt > 0) || !std::isfinite(scale))
    return fail(NFA_ERR_INVALID, "nfa_poisson_velocity: dt must be > 0 and scale finite");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const double* src = p;
  if (g.n_slaves > 0) {
    launch_copy<double>(p, op->tmp.as<double>(), g.n, st);
    launch_merge_copy<double>(g, op->tmp.as<double>(), st, nullptr);
    src = op->tmp.as<double>();
  }
  BCs bc;
  for (int f = 0; f < 6; ++f) bc.b[f] = g.bc[f];
  k_velocity<<<blocks_for(g.nfx() + g.nfy() + g.nfz()), kBlock, 0, st>>>(
      g.nx, g.ny, g.nz, bc, op->rho.as<double>(), g.open_x.as<double>(), g.open_y.as<double>(),
      g.open_z.as<double>(), g.d_hx.as<double>(), g.d_hy.as<double>(), g.d_hz.as<double>(), ut_x,
      ut_y, ut_z, src, dt, scale, u_x, u_y, u_z);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_exit_velocity(nfa_grid g, const double* uk_x, double uc, double dt,
                                        double* ut_x, nfa_stream s) {
  if (!g || !uk_x || !ut_x) return fail(NFA_ERR_INVALID, "nfa_exit_velocity: NULL argument");
  if (g->nx < 2) return fail(NFA_ERR_INVALID, "nfa_exit_velocity: needs nx >= 2");
  const double dxl = g->dx[g->nx - 1];
  if (!(dt > 0) || !(uc >= 0) || !(uc * dt <= dxl))
    return fail(NFA_ERR_INVALID, "nfa_exit_velocity: needs dt > 0 and 0 <= uc dt <= width of the last cell");
  const long long nrow = (long long)g->ny * g->nz;
  k_exit<<<blocks_for(nrow), kBlock, 0, S(s)>>>(g->nx, nrow, uk_x, (uc * dt) / dxl, ut_x);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_faces_combine(long long n, const double* a, const double* b, double s,
                                        const double* c, double* out, nfa_stream st) {
  if (n < 0 || (n > 0 && (!a || !c || !out))) return fail(NFA_ERR_INVALID, "nfa_faces_combine: bad argument");
  if (n == 0) return NFA_OK;
  if (b)
    k_combine<true><<<blocks_for(n), kBlock, 0, S(st)>>>(n, a, b, s, c, out);
  else
    k_combine<false><<<blocks_for(n), kBlock, 0, S(st)>>>(n, a, nullptr, s, c, out);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_rk2_cycle(nfa_poisson op, const void* phi_k, const void* phi_star,
                                    const nfa_rk2_params* prm, const double* const* uk,
                                    const double* const* R, double* const* ut, double* const* ustar,
                                    double* pstar, double* p, double* const* unext,
                                    const nfa_solve_opts* opts, nfa_stream s, nfa_solve_info* info) {
  if (!op || !phi_k || !phi_star || !prm || !pstar || !p || !opts || !info)
    return fail(NFA_ERR_INVALID, "nfa_rk2_cycle: NULL argument");
  if (!three((const void* const*)uk) || !three((const void* const*)R) ||
      !three((const void* const*)ut) || !three((const void* const*)ustar) ||
      !three((const void* const*)unext))
    return fail(NFA_ERR_INVALID, "nfa_rk2_cycle: every face-array triple needs three pointers");
  if (!(prm->dt > 0)) return fail(NFA_ERR_INVALID, "nfa_rk2_cycle: dt must be > 0");
  Grid& g = *op->g;
  const long long nf[3] = {g.nfx(), g.nfy(), g.nfz()};
  const double dt = prm->dt;
  double* b = op->tmp.as<double>();
  nfa_status worst = NFA_OK;
  auto track = [&](nfa_status e) {
    if (e > worst) worst = e;
    return e;
  };
  nfa_status e;
  // stage 1 (eqs. poisson1, runge1)
  if ((e = nfa_poisson_assemble(op, phi_k, &prm->rho, s)) != NFA_OK) return e;
  for (int d = 0; d < 3; ++d)
    if ((e = nfa_faces_combine(nf[d], uk[d], nullptr, dt, R[d], ut[d], s)) != NFA_OK) return e;
  if ((e = nfa_poisson_rhs(op, ut[0], ut[1], ut[2], dt, prm->body_vel, b, s)) != NFA_OK) return e;
  if ((e = track(nfa_poisson_solve(op, b, pstar, opts, s, &info[0]))) < 0) return e;
  if ((e = nfa_poisson_velocity(op, ut[0], ut[1], ut[2], pstar, dt, 1.0, ustar[0], ustar[1], ustar[2], s)) !=
      NFA_OK)
    return e;
  // stage 2 (eqs. poisson2, runge2)
  if ((e = nfa_poisson_assemble(op, phi_star, &prm->rho, s)) != NFA_OK) return e;
  for (int d = 0; d < 3; ++d)
    if ((e = nfa_faces_combine(nf[d], ustar[d], uk[d], dt, R[d], ut[d], s)) != NFA_OK) return e;
  const double vel2[3] = {2.0 * prm->body_vel[0], 2.0 * prm->body_vel[1], 2.0 * prm->body_vel[2]};
  if ((e = nfa_poisson_rhs(op, ut[0], ut[1], ut[2], dt, vel2, b, s)) != NFA_OK) return e;
  if ((e = track(nfa_poisson_solve(op, b, p, opts, s, &info[1]))) < 0) return e;
  if ((e = nfa_poisson_velocity(op, ut[0], ut[1], ut[2], p, dt, 0.5, unext[0], unext[1], unext[2], s)) !=
      NFA_OK)
    return e;
  NFA_HIP(hipStreamSynchronize(S(s)));
  return worst;
}
