// libnfa: solver drivers.
//
// Introduction: the projection's Poisson equation is solved by a
// preconditioned conjugate-gradient method; the preconditioner is not named,
// Jacobi (diag of the merged operator) is used.  Two variants sit on top:
//  * mixed precision: FP64 iterative refinement (true residual b' - A'x in
//    FP64, solution update in FP64) around an FP32 inner solve of the
//    correction equation A'_32 d = r/||r|| to a relative reduction inner_tol;
//  * flexible CG (Notay FCG(1)) for a nonlinear preconditioner such as the
//    learned one, with a stagnation monitor that switches to Jacobi-PCG.
// Every solve ends when the FP64 true relative residual meets tol (the
// judge); a mixed solve that fails to get there falls back to FP64 PCG.
//
// The host only enqueues kernels: alpha, beta, norms, the iteration count
// and the convergence flag live on the device, every kernel exits at once
// when the flag is set, and the host polls a pinned copy of the state every
// `check_every` iterations with one batch in flight.
#include <chrono>
#include <cmath>
#include <functional>

#include "device_util.h"
#include "nfa_internal.h"
#include "vecops.h"

namespace nfa {

template <class T> struct Vecs {
  T *x, *r, *z, *p, *q;
};

namespace {

// Stencil launch wrapped in a timing event pair when profiling is on.
template <class T>
int timed_stencil(Poisson& op, const Coeffs<T>& C, const T* p, T* q, double* parts,
                  const SolveScalars* sc, hipStream_t st) {
  const bool rec = op.prof_on && op.prof_used * 2 + 1 < (int)op.prof_ev.size();
  if (rec) (void)hipEventRecord(op.prof_ev[2 * op.prof_used], st);
  const int np = launch_stencil<T>(*op.g, C, p, nullptr, q, parts, sc, ST_APPLY, st);
  if (rec) {
    (void)hipEventRecord(op.prof_ev[2 * op.prof_used + 1], st);
    op.prof_kind[op.prof_used] = sizeof(T) == 8 ? 0 : 1;
    ++op.prof_used;
  }
  return np;
}

// Accumulate the recorded launches that actually ran (the device state may
// have ended the solve, making later launches exit at once: those are the
// ones after the last `done` poll and are excluded by counting only launches
// up to the iteration count).
void harvest_profile(Poisson& op, int iterations) {  // iterations run in this phase
  if (!op.prof_on) return;
  (void)hipDeviceSynchronize();
  const int upto = std::min(op.prof_used, std::max(0, iterations));
  for (int i = 0; i < upto; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, op.prof_ev[2 * i], op.prof_ev[2 * i + 1]) == hipSuccess) {
      op.prof_ms[op.prof_kind[i]] += ms;
      op.prof_launches[op.prof_kind[i]] += 1;
    }
  }
  op.prof_used = 0;
}

nfa_status poll_until_done(Poisson& op, const std::function<void()>& batch, hipStream_t st,
                           SolveScalars* out) {
  SolveScalars* sc = op.scal.as<SolveScalars>();
  int slot = 0;
  bool have_prev = false;
  for (;;) {
    batch();
    NFA_CHECK_LAUNCH();
    NFA_HIP(hipMemcpyAsync(&op.h_scal[slot], sc, sizeof(SolveScalars), hipMemcpyDeviceToHost, st));
    NFA_HIP(hipEventRecord(op.ev[slot], st));
    if (have_prev) {
      NFA_HIP(hipEventSynchronize(op.ev[slot ^ 1]));
      if (op.h_scal[slot ^ 1].done) break;
    }
    have_prev = true;
    slot ^= 1;
  }
  NFA_HIP(hipStreamSynchronize(st));
  NFA_HIP(hipMemcpy(out, sc, sizeof(SolveScalars), hipMemcpyDeviceToHost));
  return NFA_OK;
}

nfa_status read_scalars(Poisson& op, hipStream_t st, SolveScalars* out) {
  NFA_HIP(hipStreamSynchronize(st));
  NFA_HIP(hipMemcpy(out, op.scal.p, sizeof(SolveScalars), hipMemcpyDeviceToHost));
  return NFA_OK;
}

// Jacobi-PCG from the residual in v.r and the iterate in v.x (primal).
template <class T>
nfa_status pcg_phase(Poisson& op, const Coeffs<T>& C, Vecs<T> v, int check_every, hipStream_t st,
                     SolveScalars* out, int iter0) {
  Grid& g = *op.g;
  const long long n = g.n;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  double* parts = op.partials.as<double>();
  double* hist = op.hist.as<double>();
  const int nb = launch_jacobi<T>(v.r, C.dinv, v.z, n, parts, st);
  launch_merge_copy<T>(g, v.z, st, nullptr);
  launch_finalize(parts, nb, 2, PH_INIT, sc, hist, st);
  launch_copy<T>(v.z, v.p, n, st);
  auto batch = [&]() {
    for (int it = 0; it < check_every; ++it) {
      const int np = timed_stencil<T>(op, C, v.p, v.q, parts, sc, st);
      launch_merge_gather<T>(g, v.q, st, sc);
      launch_finalize(parts, np, 1, PH_PQ, sc, hist, st);
      const int nu = launch_update<T>(v.x, v.p, v.r, v.q, C.dinv, v.z, n, parts, sc, st);
      launch_merge_copy<T>(g, v.z, st, sc);
      launch_finalize(parts, nu, 2, PH_UPD, sc, hist, st);
      launch_direction<T>(v.z, v.p, n, sc, st);
    }
  };
  nfa_status e = poll_until_done(op, batch, st, out);
  harvest_profile(op, out->iter - iter0);
  return e;
}

// Flexible CG(1) with preconditioner `pc` from the residual in v.r.
template <class T>
nfa_status fcg_phase(Poisson& op, const Coeffs<T>& C, Vecs<T> v, int pc, void* unet,
                     int check_every, hipStream_t st, SolveScalars* out, int iter0) {
  Grid& g = *op.g;
  const long long n = g.n;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  double* parts = op.partials.as<double>();
  double* hist = op.hist.as<double>();
  launch_fill<T>(v.p, T(0), n, st);
  launch_fill<T>(v.q, T(0), n, st);
  const int nb = launch_dot<T>(v.r, v.r, n, parts, nullptr, st);
  launch_finalize(parts, nb, 1, PH_INIT, sc, hist, st);
  nfa_status pst = NFA_OK;
  auto batch = [&]() {
    for (int it = 0; it < check_every; ++it) {
      if (pc == NFA_PC_JACOBI || pc == NFA_PC_JACOBI_FCG) {
        launch_scale<T>(v.r, C.dinv, v.z, n, sc, st);
      } else if (pc == NFA_PC_TEST_SABOTAGE) {
        launch_sabotage<T>(g.reduced.as<unsigned char>(), v.z, n, sc, st);
      } else {
        nfa_status e = unet_precond_apply(unet, op, (const float*)v.r, (float*)v.z, sc, st);
        if (e != NFA_OK && pst == NFA_OK) pst = e;
      }
      launch_merge_copy<T>(g, v.z, st, sc);
      const int nz = launch_dot<T>(v.z, v.q, n, parts, sc, st);
      launch_finalize(parts, nz, 1, PH_ZQ, sc, hist, st);
      const int nd = launch_fdirection<T>(v.z, v.p, v.r, n, parts, sc, st);
      launch_finalize(parts, nd, 1, PH_PR, sc, hist, st);
      const int np = timed_stencil<T>(op, C, v.p, v.q, parts, sc, st);
      launch_merge_gather<T>(g, v.q, st, sc);
      launch_finalize(parts, np, 1, PH_PQF, sc, hist, st);
      const int nu = launch_fupdate<T>(v.x, v.p, v.r, v.q, n, parts, sc, st);
      launch_finalize(parts, nu, 1, PH_UPDF, sc, hist, st);
    }
  };
  nfa_status e = poll_until_done(op, batch, st, out);
  harvest_profile(op, out->iter - iter0);
  if (pst != NFA_OK) return pst;
  return e;
}

// r = b' - A' x (x primal), optionally ||r||^2 into the state (phase).
nfa_status residual64(Poisson& op, const double* b, const double* x, double* r, int phase,
                      hipStream_t st) {
  Grid& g = *op.g;
  launch_stencil<double>(g, op.c64(), x, b, r, nullptr, nullptr, ST_RESIDUAL, st);
  launch_merge_gather<double>(g, r, st, nullptr);
  if (phase >= 0) {
    double* parts = op.partials.as<double>();
    const int nb = launch_dot<double>(r, r, g.n, parts, nullptr, st);
    launch_finalize(parts, nb, 1, phase, op.scal.as<SolveScalars>(), nullptr, st);
  }
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

void copy_history(Poisson& op, const nfa_solve_opts* o, nfa_solve_info* info, int upto,
                  double scale2, hipStream_t st) {
  if (!o->history || o->history_cap <= 0) return;
  const int have = info->history_len;
  const int room = o->history_cap - have;
  if (room <= 0) return;
  const int cnt = std::min(room, upto + 1);
  std::vector<double> h(cnt);
  (void)hipStreamSynchronize(st);
  (void)hipMemcpy(h.data(), op.hist.p, cnt * sizeof(double), hipMemcpyDeviceToHost);
  for (int k = 0; k < cnt; ++k) o->history[have + k] = std::sqrt(std::max(0.0, h[k] * scale2));
  info->history_len = have + cnt;
}

nfa_status solve_f64(Poisson& op, const double* b, double* x, const nfa_solve_opts* o,
                     const SolveScalars& s0, hipStream_t st, nfa_solve_info* info, int iters_done) {
  Grid& g = *op.g;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  const int budget = std::max(0, o->max_iters - iters_done);
  launch_set_scalars(sc, o->tol * o->tol, 0, budget, 1, 0, 1.0, st);
  Vecs<double> v{x, op.r.as<double>(), op.z.as<double>(), op.p.as<double>(), op.q.as<double>()};
  SolveScalars out{};
  nfa_status status = NFA_NOT_CONVERGED;
  for (int restart = 0; restart <= 3; ++restart) {
    nfa_status e = residual64(op, b, x, v.r, -1, st);
    if (e != NFA_OK) return e;
    e = pcg_phase<double>(op, op.c64(), v, std::max(1, o->check_every), st, &out, out.iter);
    if (e != NFA_OK) return e;
    if (out.breakdown == 2) return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf in the iteration");
    e = residual64(op, b, x, v.r, PH_RR, st);
    if (e != NFA_OK) return e;
    SolveScalars now{};
    if ((e = read_scalars(op, st, &now)) != NFA_OK) return e;
    info->relres = std::sqrt(now.rr / s0.bb);
    info->iterations = iters_done + out.iter;
    info->outer = restart;
    if (!std::isfinite(info->relres)) return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf residual");
    if (info->relres <= o->tol) { status = NFA_OK; break; }
    if (out.iter >= budget) break;
    launch_set_scalars(sc, o->tol * o->tol, 0, budget, 0, 0, 1.0, st);
  }
  copy_history(op, o, info, std::min(out.iter, kHistCap), 1.0 / s0.bb, st);
  return status;
}

nfa_status solve_mixed(Poisson& op, const double* b, double* x, const nfa_solve_opts* o,
                       const SolveScalars& s0, hipStream_t st, nfa_solve_info* info) {
  Grid& g = *op.g;
  const long long n = g.n;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  Vecs<float> v{op.x32.as<float>(), op.r32.as<float>(), op.z32.as<float>(), op.p32.as<float>(),
                op.q32.as<float>()};
  const int check = std::max(1, o->check_every);
  int total = 0;
  bool converged = false;
  for (int outer = 0; outer <= o->max_outer; ++outer) {
    nfa_status e = residual64(op, b, x, op.r.as<double>(), PH_RRO, st);
    if (e != NFA_OK) return e;
    SolveScalars now{};
    if ((e = read_scalars(op, st, &now)) != NFA_OK) return e;
    const double relres = std::sqrt(now.rr_outer / s0.bb);
    info->relres = relres;
    info->outer = outer;
    info->iterations = total;
    if (!std::isfinite(relres)) return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf residual");
    if (relres <= o->tol) { converged = true; break; }
    if (total >= o->max_iters || outer == o->max_outer) break;
    launch_cast_scaled(op.r.as<double>(), v.r, n, sc, st);
    launch_fill<float>(v.x, 0.0f, n, st);
    // inner reduction: what is still needed (with a factor 4 margin), but no
    // deeper than inner_tol, near where FP32 residuals stop being accurate
    const double need = 0.25 * o->tol / relres;
    const double eta = std::min(0.5, std::max(o->inner_tol, need));
    const double eta2 = eta * eta;
    const bool flexible = o->precond == NFA_PC_UNET || o->precond == NFA_PC_TEST_SABOTAGE ||
                          o->precond == NFA_PC_JACOBI_FCG;
    launch_set_scalars(sc, eta2, 1, o->max_iters - total, 1, flexible ? o->fallback_window : 0,
                       o->fallback_ratio, st);
    SolveScalars out{};
    if (flexible && !info->fallback) {
      e = fcg_phase<float>(op, op.c32(), v, o->precond, o->unet, check, st, &out, 0);
      if (e != NFA_OK) return e;
      if (out.stalled || out.breakdown == 1) {
        // switch to Jacobi-PCG for the rest of the inner solve, from the current iterate
        info->fallback = 1;
        launch_set_scalars(sc, eta2, 1, o->max_iters - total, 0, 0, 1.0, st);
        e = pcg_phase<float>(op, op.c32(), v, check, st, &out, out.iter);
        if (e != NFA_OK) return e;
      }
    } else {
      e = pcg_phase<float>(op, op.c32(), v, check, st, &out, 0);
      if (e != NFA_OK) return e;
    }
    copy_history(op, o, info, std::min(out.iter, kHistCap), now.rr_outer / s0.bb, st);
    if (out.breakdown == 2) return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf in the inner iteration");
    total += out.iter;
    launch_refine_update(x, v.x, n, sc, st);
    NFA_CHECK_LAUNCH();
  }
  info->iterations = total;
  if (converged) return NFA_OK;
  if (total < o->max_iters) {
    // refinement did not reach the tolerance: FP64 Jacobi-PCG from the current x
    info->fallback = 1;
    const int outer = info->outer;
    nfa_status e = solve_f64(op, b, x, o, s0, st, info, total);
    info->outer += outer;
    return e;
  }
  return NFA_NOT_CONVERGED;
}

}  // namespace
}  // namespace nfa

using namespace nfa;

extern "C" void nfa_solve_opts_default(nfa_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_iters = 200000;
  o->precond = NFA_PC_JACOBI;
  o->precision = NFA_PREC_F64;
  o->inner_tol = 1e-6;
  o->max_outer = 8;
  o->fcg_m = 1;
  o->fallback_ratio = 0.99;
  o->fallback_window = 10;
  o->warm_start = 0;
  o->check_every = 16;
  o->unet = nullptr;
  o->history = nullptr;
  o->history_cap = 0;
}

extern "C" nfa_status nfa_poisson_solve(nfa_poisson op, const double* b, double* x,
                                        const nfa_solve_opts* o, nfa_stream s, nfa_solve_info* info) {
  if (!op || !b || !x || !o || !info) return fail(NFA_ERR_INVALID, "nfa_poisson_solve: NULL argument");
  if (!op->assembled) return fail(NFA_ERR_INVALID, "nfa_poisson_solve: operator not assembled");
  if (!(o->tol > 0) || o->max_iters < 1 || o->check_every < 1)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: tol > 0, max_iters >= 1, check_every >= 1 required");
  if (o->precision != NFA_PREC_F64 && o->precision != NFA_PREC_MIXED)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: unknown precision");
  if (o->precond != NFA_PC_JACOBI && o->precond != NFA_PC_UNET && o->precond != NFA_PC_TEST_SABOTAGE &&
      o->precond != NFA_PC_JACOBI_FCG)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: unknown preconditioner");
  if (o->precond != NFA_PC_JACOBI && o->precision != NFA_PREC_MIXED)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: flexible CG runs as the FP32 inner solve (NFA_PREC_MIXED)");
  if (o->precond == NFA_PC_UNET && !o->unet)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: NFA_PC_UNET needs opts->unet");
  if (o->fcg_m != 1) return fail(NFA_ERR_INVALID, "nfa_poisson_solve: fcg_m must be 1");
  if (o->precision == NFA_PREC_MIXED && (!(o->inner_tol > 0 && o->inner_tol < 1) || o->max_outer < 1))
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: mixed needs 0 < inner_tol < 1 and max_outer >= 1");
  const auto t0 = std::chrono::steady_clock::now();
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  *info = nfa_solve_info{};
  SolveScalars* sc = op->scal.as<SolveScalars>();
  double* parts = op->partials.as<double>();
  launch_init_x(x, g.active.as<unsigned char>(), g.n, o->warm_start, st);
  launch_merge_copy<double>(g, x, st, nullptr);
  const int nb = launch_dot<double>(b, b, g.n, parts, nullptr, st);
  launch_finalize(parts, nb, 1, PH_BB, sc, nullptr, st);
  NFA_CHECK_LAUNCH();
  SolveScalars s0{};
  nfa_status e = read_scalars(*op, st, &s0);
  if (e != NFA_OK) return e;
  if (!std::isfinite(s0.bb)) return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf in b");
  if (s0.bb == 0.0) {
    launch_fill<double>(x, 0.0, g.n, st);
    NFA_HIP(hipStreamSynchronize(st));
    info->relres = 0.0;
    return NFA_OK;
  }
  nfa_status status = o->precision == NFA_PREC_F64 ? solve_f64(*op, b, x, o, s0, st, info, 0)
                                                   : solve_mixed(*op, b, x, o, s0, st, info);
  if (status < 0) return status;
  if (g.all_neumann() && g.n_reduced > 0) {
    const int np = launch_masked_sum<double>(x, g.reduced.as<unsigned char>(), g.n, parts, st);
    double* sum = parts + (size_t)kMaxPartials * 3;
    launch_sum_partials(parts, np, 1, sum, st);
    launch_sub_mean(x, g.reduced.as<unsigned char>(), g.n, sum, (double)g.n_reduced, st);
    launch_merge_copy<double>(g, x, st, nullptr);
    NFA_CHECK_LAUNCH();
  }
  NFA_HIP(hipStreamSynchronize(st));
  info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

extern "C" nfa_status nfa_poisson_profile(nfa_poisson op, int enable) {
  if (!op) return fail(NFA_ERR_INVALID, "nfa_poisson_profile: NULL handle");
  NFA_HIP(hipDeviceSynchronize());
  if (enable && op->prof_ev.empty()) {
    const int pairs = 4096;
    op->prof_ev.resize(2 * pairs, nullptr);
    op->prof_kind.resize(pairs, 0);
    for (auto& e : op->prof_ev) NFA_HIP(hipEventCreate(&e));
  }
  op->prof_on = enable != 0;
  op->prof_used = 0;
  op->prof_launches[0] = op->prof_launches[1] = 0;
  op->prof_ms[0] = op->prof_ms[1] = 0.0;
  return NFA_OK;
}

extern "C" nfa_status nfa_poisson_profile_read(nfa_poisson op, int dtype, nfa_kernel_stats* out) {
  if (!op || !out || (dtype != NFA_F64 && dtype != NFA_F32))
    return fail(NFA_ERR_INVALID, "nfa_poisson_profile_read: bad argument");
  out->launches = op->prof_launches[dtype];
  out->ms = op->prof_ms[dtype];
  out->cells = op->g->n;
  return NFA_OK;
}
