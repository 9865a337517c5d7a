// libnfa: solver drivers.
//
// Introduction: the projection's Poisson equation is solved by a
// preconditioned conjugate-gradient method; the preconditioner is not named,
// Jacobi (diag of the merged operator) is used.  Two variants sit on top:
//  * mixed precision: the CG recurrence (operator, preconditioner, vector
//    updates) runs in FP32; the solution is accumulated in FP64 and the true
//    residual b' - A'x is recomputed in FP64 and replaces the FP32 one each
//    time the recursive residual has dropped by `replace_drop` (iterative
//    refinement without restarting the Krylov recurrence);
//  * flexible CG (Notay FCG(1)) for a nonlinear preconditioner such as the
//    learned one, with a stagnation monitor that switches to Jacobi-PCG.
// Every solve ends when the FP64 true relative residual meets tol.
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

template <class T> struct CG {
  T* x;
  T* r;
  T* z;
  T* q;
  T* p[3];      // directions: flexible CG alternates p[0], p[1]; Jacobi-PCG rotates all three
  Coeffs<T> C;
  bool vec;
};

namespace {

inline double sq(double a) { return a * a; }

// Sweep A wrapped in a timing event pair when profiling is on.
template <class T>
int timed_cg_a(Poisson& op, CG<T>& B, int j, bool flex, int xm, hipStream_t st) {
  const bool rec = prof_begin(op, st);
  const T* pold = flex ? B.p[j & 1] : B.p[j % 3];
  const T* pold2 = flex ? nullptr : B.p[(j + 2) % 3];
  T* pnew = flex ? B.p[(j + 1) & 1] : B.p[(j + 1) % 3];
  const int np = launch_cg_a<T>(*op.g, B.C, B.z, pold, pold2, pnew, B.x, B.r, B.q, op.partials.as<double>(),
                                op.scal.as<SolveScalars>(), flex, xm, B.vec, st);
  const int kind = sizeof(T) == 8 ? (xm == 2 ? kProfF64X2 : 0) : (flex ? kProfF32Flex : (xm == 2 ? kProfF32X2 : 1));
  prof_end(op, rec, kind, st);
  return np;
}

// Accumulate the recorded launches of the first `ran` iterations enqueued
// since the last harvest (later ones saw the solver state say done and
// exited at once).
void harvest_profile(Poisson& op, int ran) {
  if (!op.prof_on) return;
  (void)hipDeviceSynchronize();
  for (int i = 0; i < op.prof_used; ++i) {
    if (op.prof_seq[i] >= ran) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, op.prof_ev[2 * i], op.prof_ev[2 * i + 1]) == hipSuccess) {
      op.prof_ms[op.prof_kind[i]] += ms;
      op.prof_launches[op.prof_kind[i]] += 1;
    }
  }
  op.prof_used = 0;
  op.prof_iter = 0;
}

nfa_status read_scalars(Poisson& op, hipStream_t st, SolveScalars* out) {
  NFA_HIP(hipStreamSynchronize(st));
  NFA_HIP(hipMemcpy(out, op.scal.p, sizeof(SolveScalars), hipMemcpyDeviceToHost));
  return NFA_OK;
}

// r = b' - A' x (x primal), ||r||^2 into the state (phase) when phase >= 0.
nfa_status residual64(Poisson& op, const double* b, const double* x, double* r, int phase,
                      hipStream_t st) {
  Grid& g = *op.g;
  launch_stencil<double>(g, op.c64(), x, b, r, st);
  launch_merge_gather<double>(g, r, st, nullptr);
  if (phase >= 0) {
    double* parts = op.partials.as<double>();
    const int nb = launch_dot<double>(r, r, g.n, parts, nullptr, st);
    launch_finalize(parts, nb, 1, phase, op.scal.as<SolveScalars>(), nullptr, st);
  }
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

// One iteration of PCG (pc == Jacobi) or flexible CG (any other pc).
template <class T>
void enqueue_iter(Poisson& op, CG<T>& B, int j, int pc, void* unet, nfa_status* pst, hipStream_t st) {
  Grid& g = *op.g;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  double* parts = op.partials.as<double>();
  double* hist = op.hist.as<double>();
  const bool flex = pc != NFA_PC_JACOBI;
  if (flex) {
    int nzq = 0;   // partials of z.q written by the preconditioner itself
    if (pc == NFA_PC_JACOBI_FCG) {
      launch_scale<T>(B.r, B.C.dinv, B.z, g.n, sc, st);
    } else if (pc == NFA_PC_TEST_SABOTAGE) {
      launch_sabotage<T>(g.reduced.as<unsigned char>(), B.z, g.n, sc, st);
    } else if (pc == NFA_PC_MG) {
      const nfa_status e = mg_precond_apply(unet, op, (const float*)B.r, (float*)B.z, (const float*)B.q, parts, &nzq,
                                            sc, st);
      if (e != NFA_OK && *pst == NFA_OK) *pst = e;
    } else {
      const bool rec = prof_begin(op, st);
      const nfa_status e = unet_precond_apply(unet, op, (const float*)B.r, (float*)B.z, sc, st);
      prof_end(op, rec, kProfUnet, st);
      if (e != NFA_OK && *pst == NFA_OK) *pst = e;
    }
    if (nzq > 0) {
      // z.q summed by the cycle (slaves' q is 0, so their z does not enter
      // it): its finalize and the slaves' copy of z share a launch
      launch_finalize_merge<T>(g, false, B.z, parts, nzq, 1, PH_ZQ, sc, hist, st);
    } else {
      launch_merge_copy<T>(g, B.z, st, sc);
      nzq = launch_dot<T>(B.z, B.q, g.n, parts, sc, st);
      launch_finalize(parts, nzq, 1, PH_ZQ, sc, hist, st);
    }
  }
  // Jacobi-PCG: iterations 0, 2, 4 ... of a phase leave x alone, the odd ones
  // apply the two owed steps
  const int xm = flex ? 1 : ((j & 1) ? 2 : 0);
  const int na = timed_cg_a<T>(op, B, j, flex, xm, st);
  launch_finalize_merge<T>(g, true, B.q, parts, na, flex ? 2 : 1, flex ? PH_PQF : (xm == 0 ? PH_PQ_SKIP : PH_PQ),
                           sc, hist, st);
  const int nb = launch_cg_b<T>(g, B.r, B.q, B.C.dinv, B.z, parts, sc, flex, B.vec, st);
  if (flex)
    launch_finalize(parts, nb, 1, PH_UPDF, sc, hist, st);
  else
    launch_finalize_merge<T>(g, false, B.z, parts, nb, 2, PH_UPD, sc, hist, st);
  ++op.prof_iter;
}

// Start (fresh) or continue (after a residual replacement) the recurrence
// from the residual in B.r.
template <class T>
void begin_phase(Poisson& op, CG<T>& B, int pc, bool fresh, hipStream_t st) {
  Grid& g = *op.g;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  double* parts = op.partials.as<double>();
  double* hist = op.hist.as<double>();
  const bool flex = pc != NFA_PC_JACOBI;
  if (fresh) {
    launch_fill<T>(B.p[0], T(0), g.n, st);
    if (flex) launch_fill<T>(B.q, T(0), g.n, st);
  }
  if (flex) {
    const int nb = launch_dot<T>(B.r, B.r, g.n, parts, nullptr, st);
    launch_finalize(parts, nb, 1, fresh ? PH_INIT : PH_RELIABLE_F, sc, hist, st);
  } else {
    const int nb = launch_jacobi<T>(B.r, B.C.dinv, B.z, g.n, parts, st);
    launch_merge_copy<T>(g, B.z, st, nullptr);
    launch_finalize(parts, nb, 2, fresh ? PH_INIT : PH_RELIABLE, sc, hist, st);
  }
}

void copy_history(Poisson& op, const nfa_solve_opts* o, nfa_solve_info* info, int upto,
                  double inv_norm2, hipStream_t st) {
  if (!o->history || o->history_cap <= 0) return;
  const int cnt = std::min(o->history_cap, std::min(upto, kHistCap) + 1);
  std::vector<double> h(cnt);
  (void)hipStreamSynchronize(st);
  (void)hipMemcpy(h.data(), op.hist.p, cnt * sizeof(double), hipMemcpyDeviceToHost);
  for (int k = 0; k < cnt; ++k) o->history[k] = std::sqrt(std::max(0.0, h[k] * inv_norm2));
  info->history_len = cnt;
}

// CG with FP64 residual replacement.  T = double: plain FP64 Jacobi-PCG, the
// true residual checked when the recursion converges.  T = float: the
// iteration runs in FP32 on the scaled residual; whenever the recursive
// residual has dropped by `delta` (or the recursion ends) the FP32 solution
// increment is folded into the FP64 solution, the FP64 true residual
// b' - A'x is recomputed and replaces the FP32 one, and CG goes
// on with the same search direction.
template <class T>
nfa_status cg_solve(Poisson& op, const double* b, double* x64, const nfa_solve_opts* o,
                    const SolveScalars& s0, hipStream_t st, nfa_solve_info* info) {
  constexpr bool mixed = sizeof(T) == 4;
  Grid& g = *op.g;
  SolveScalars* sc = op.scal.as<SolveScalars>();
  const double bnorm = std::sqrt(s0.bb);
  const double scale = mixed ? std::ldexp(1.0, -std::ilogb(bnorm)) : 1.0;   // exact power of two
  CG<T> B;
  if constexpr (mixed) {
    B = CG<T>{op.x32.as<float>(), op.r32.as<float>(), op.z32.as<float>(), op.q32.as<float>(),
              {op.p32.as<float>(), op.p32b.as<float>(), op.p32c.as<float>()}, op.c32(), false};
  } else {
    B = CG<T>{x64, op.r.as<double>(), op.z.as<double>(), op.q.as<double>(),
              {op.p.as<double>(), op.p2.as<double>(), op.p3.as<double>()}, op.c64(), false};
  }
  const void* ptrs[] = {B.x, B.r, B.z, B.q, B.p[0], B.p[1], B.p[2], B.C.tx, B.C.ty, B.C.tz, B.C.dinv};
  B.vec = cg_vectorizable<T>(g, ptrs, 11);
  int pc = o->precond;
  const double delta = mixed ? o->replace_drop : 0.0;
  double* r64 = op.r.as<double>();
  // the multigrid-preconditioned recursion falls by ~10x every two or three
  // iterations: polled less often, an FP32 phase would run far past the
  // replacement point and below its own accuracy
  const int check = pc == NFA_PC_MG ? std::min(std::max(1, o->check_every), 2) : std::max(1, o->check_every);

  op.prof_used = 0;
  op.prof_iter = 0;
  nfa_status e = residual64(op, b, x64, r64, PH_RRO, st);
  if (e != NFA_OK) return e;
  SolveScalars S{};
  if ((e = read_scalars(op, st, &S)) != NFA_OK) return e;
  double relres = std::sqrt(S.rr_outer / s0.bb);
  info->relres = relres;
  if (!std::isfinite(relres)) return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf residual");
  if (relres <= o->tol) return NFA_OK;
  if (mixed) {
    launch_cast(g, r64, op.r32.as<float>(), scale, st);
    launch_fill<float>(op.x32.as<float>(), 0.0f, g.n, st);
  }
  // the FP32 recursion aims a little below tol so that its rounding cannot
  // stop it just above the FP64 tolerance
  const double tol2 = sq((mixed ? 0.7 : 1.0) * o->tol * bnorm * scale);
  const bool flex0 = pc != NFA_PC_JACOBI;
  launch_set_scalars(sc, tol2, 1, o->max_iters, 1,
                     flex0 ? o->fallback_window : 0, o->fallback_ratio, st);
  begin_phase<T>(op, B, pc, true, st);
  int iter_phase = 0, j = 0, last_harvest = 0, last_update_iter = -1, stuck = 0;
  double rr_ref = sq(relres * bnorm * scale);
  nfa_status pst = NFA_OK, status = NFA_NOT_CONVERGED;
  int slot = 0;
  bool have_prev = false;
  for (;;) {
    void* handle = pc == NFA_PC_MG ? o->mg : o->unet;
    for (int it = 0; it < check; ++it, ++j) enqueue_iter<T>(op, B, j, pc, handle, &pst, st);
    NFA_CHECK_LAUNCH();
    if (pst != NFA_OK) return pst;
    NFA_HIP(hipMemcpyAsync(&op.h_scal[slot], sc, sizeof(SolveScalars), hipMemcpyDeviceToHost, st));
    NFA_HIP(hipEventRecord(op.ev[slot], st));
    bool act = false;
    if (have_prev) {
      NFA_HIP(hipEventSynchronize(op.ev[slot ^ 1]));
      const SolveScalars& snap = op.h_scal[slot ^ 1];
      act = snap.done || (delta > 0 && snap.rr <= sq(delta) * rr_ref);
    }
    if (!act) {
      have_prev = true;
      slot ^= 1;
      continue;
    }
    // ---- residual replacement (FP64 true residual)
    if ((e = read_scalars(op, st, &S)) != NFA_OK) return e;
    harvest_profile(op, S.iter - last_harvest);
    last_harvest = S.iter;
    // J iterations of this phase are complete; the step on their last
    // direction (and in Jacobi-PCG possibly the one before) is still owed
    const int J = S.iter - iter_phase;
    if (pc == NFA_PC_JACOBI) launch_cg_fixup<T>(g, B.x, B.p[J % 3], B.p[(J + 2) % 3], sc, st);
    else launch_cg_fixup<T>(g, B.x, B.p[J & 1], nullptr, sc, st);
    if (mixed) launch_fold(g, x64, op.x32.as<float>(), 1.0 / scale, st);
    if ((e = residual64(op, b, x64, r64, PH_RRO, st)) != NFA_OK) return e;
    SolveScalars S2{};
    if ((e = read_scalars(op, st, &S2)) != NFA_OK) return e;
    relres = std::sqrt(S2.rr_outer / s0.bb);
    info->relres = relres;
    info->iterations = S.iter;
    info->outer += 1;
    if (S.breakdown == 2 || !std::isfinite(relres))
      return fail(NFA_ERR_NUMERIC, "nfa_poisson_solve: NaN/Inf in the iteration");
    if (relres <= o->tol) { status = NFA_OK; break; }
    if (S.iter >= o->max_iters) break;
    if (S.iter == last_update_iter && ++stuck >= 3) break;   // no progress possible
    if (S.iter != last_update_iter) stuck = 0;
    last_update_iter = S.iter;
    if (mixed) launch_cast(g, r64, op.r32.as<float>(), scale, st);
    const bool fresh = S.breakdown == 1 || S.stalled;
    if (S.stalled && pc != NFA_PC_JACOBI) {
      // the flexible preconditioner stopped paying: Jacobi-PCG from here on
      pc = NFA_PC_JACOBI;
      info->fallback = 1;
    }
    launch_set_scalars(sc, tol2, 1, o->max_iters, 0,
                       pc != NFA_PC_JACOBI ? o->fallback_window : 0, o->fallback_ratio, st);
    begin_phase<T>(op, B, pc, fresh, st);
    if (fresh) {
      iter_phase = S.iter;
      j = 0;
    } else {
      j = J;
    }
    rr_ref = sq(relres * bnorm * scale);
    have_prev = false;
    slot = 0;
  }
  copy_history(op, o, info, info->iterations, 1.0 / sq(bnorm * scale), st);
  return status;
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
  o->replace_drop = 0.1;
  o->fcg_m = 1;
  o->fallback_ratio = 0.99;
  o->fallback_window = 10;
  o->warm_start = 0;
  o->check_every = 16;
  o->unet = nullptr;
  o->history = nullptr;
  o->history_cap = 0;
  o->mg = nullptr;
}

extern "C" nfa_status nfa_poisson_solve(nfa_poisson op, const double* b, double* x,
                                        const nfa_solve_opts* o, nfa_stream s, nfa_solve_info* info) {
  if (!op || !b || !x || !o || !info) return fail(NFA_ERR_INVALID, "nfa_poisson_solve: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_poisson_solve")) return e;
  if (!(o->tol > 0) || o->max_iters < 1 || o->check_every < 1)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: tol > 0, max_iters >= 1, check_every >= 1 required");
  if (o->precision != NFA_PREC_F64 && o->precision != NFA_PREC_MIXED)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: unknown precision");
  if (o->precond != NFA_PC_JACOBI && o->precond != NFA_PC_UNET && o->precond != NFA_PC_TEST_SABOTAGE &&
      o->precond != NFA_PC_JACOBI_FCG && o->precond != NFA_PC_MG)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: unknown preconditioner");
  if (o->precond != NFA_PC_JACOBI && o->precision != NFA_PREC_MIXED)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: flexible CG runs as the FP32 inner solve (NFA_PREC_MIXED)");
  if (o->precond == NFA_PC_UNET && !o->unet)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: NFA_PC_UNET needs opts->unet");
  if (o->precond == NFA_PC_MG && !o->mg)
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: NFA_PC_MG needs opts->mg");
  if (o->fcg_m != 1) return fail(NFA_ERR_INVALID, "nfa_poisson_solve: fcg_m must be 1");
  if (o->precision == NFA_PREC_MIXED && !(o->replace_drop > 0 && o->replace_drop < 1))
    return fail(NFA_ERR_INVALID, "nfa_poisson_solve: mixed needs 0 < replace_drop < 1");
  const auto t0 = std::chrono::steady_clock::now();
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  if (o->precond == NFA_PC_MG) {
    const nfa_status me = mg_ensure(o->mg, *op, st);   // rebuild after a new assembly
    if (me != NFA_OK) return me;
  }
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
  nfa_status status = o->precision == NFA_PREC_F64 ? cg_solve<double>(*op, b, x, o, s0, st, info)
                                                   : cg_solve<float>(*op, b, x, o, s0, st, info);
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
    op->prof_seq.resize(pairs, 0);
    for (auto& e : op->prof_ev) NFA_HIP(hipEventCreate(&e));
  }
  op->prof_on = enable != 0;
  op->prof_used = 0;
  op->prof_iter = 0;
  for (int k = 0; k < kProfKinds; ++k) {
    op->prof_launches[k] = 0;
    op->prof_ms[k] = 0.0;
  }
  return NFA_OK;
}

extern "C" nfa_status nfa_poisson_profile_read(nfa_poisson op, int dtype, nfa_kernel_stats* out) {
  if (!op || !out || dtype < 0 || dtype >= kProfKinds)
    return fail(NFA_ERR_INVALID, "nfa_poisson_profile_read: bad argument");
  out->launches = op->prof_launches[dtype];
  out->ms = op->prof_ms[dtype];
  out->cells = op->g->n;
  return NFA_OK;
}

extern "C" nfa_status nfa_poisson_residual(nfa_poisson op, const double* b, const double* x, double* r,
                                           double* rr, nfa_stream s) {
  if (!op || !b || !x || !r) return fail(NFA_ERR_INVALID, "nfa_poisson_residual: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_poisson_residual")) return e;
  if (x == r) return fail(NFA_ERR_INVALID, "nfa_poisson_residual: r must not alias x");
  Grid& g = *op->g;
  const hipStream_t st = S(s);
  const double* src = x;
  if (g.n_slaves > 0) {
    launch_copy<double>(x, op->tmp.as<double>(), g.n, st);
    launch_merge_copy<double>(g, op->tmp.as<double>(), st, nullptr);
    src = op->tmp.as<double>();
  }
  nfa_status e = residual64(*op, b, src, r, rr ? PH_RR : -1, st);
  if (e != NFA_OK) return e;
  if (rr) {
    SolveScalars now{};
    if ((e = read_scalars(*op, st, &now)) != NFA_OK) return e;
    *rr = now.rr;
  }
  return NFA_OK;
}
