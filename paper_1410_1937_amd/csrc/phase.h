// Solver-state transitions applied after each reduction by the finalize
// kernels.  Header-only: device functions do not link across files here.
#pragma once

#include <hip/hip_runtime.h>

#include "nfa_internal.h"
#include "vecops.h"

namespace nfa {

// Stagnation test on the squared-residual history: mean reduction factor of
// ||r|| per iteration over the last `window` iterations above `ratio`.
__device__ __forceinline__ bool stalled_now(const SolveScalars* sc, const double* hist) {
  const int w = sc->window;
  if (!hist || w <= 0 || sc->iter < 2 * w || sc->iter > sc->max_iter || sc->iter > kHistCap)
    return false;
  const double a = hist[sc->iter], b = hist[sc->iter - w];
  if (!(b > 0.0)) return false;
  const double rate = pow(a / b, 0.5 / w);
  return !(rate <= sc->ratio);
}

// Advance the solver state from the summed reduction values (thread 0 of
// one workgroup).
__device__ __forceinline__ void apply_phase(int phase, int ncomp, const double* val, SolveScalars* sc, double* hist) {
  switch (phase) {
  case PH_BB:
    sc->bb = val[0];
    break;
  case PH_RR:
    sc->rr = val[0];
    break;
  case PH_RRO:
    sc->rr_outer = val[0];
    break;
  case PH_INIT:
    // ncomp 2: (r.z, r.r) for PCG; ncomp 1: (r.r) for FCG
    if (ncomp == 2) { sc->rz = val[0]; sc->rr = val[1]; }
    else { sc->rr = val[0]; }
    sc->pq = 0.0;
    sc->beta = 0.0;
    sc->rz_prev = sc->rz;
    sc->alpha_pend = 0.0;
    sc->alpha_pend2 = 0.0;
    sc->done = 0;
    sc->breakdown = 0;
    sc->stalled = 0;
    if (!isfinite(sc->rr) || (ncomp == 2 && !isfinite(sc->rz))) { sc->breakdown = 2; sc->done = 1; }
    else if (sc->rr <= sc->tol2) sc->done = 1;
    if (hist && sc->iter <= sc->max_iter && sc->iter <= kHistCap) hist[sc->iter] = sc->rr;
    break;
  case PH_PQ:
    // Jacobi-PCG, after a sweep A that applied every owed x update
    sc->pq = val[0];
    sc->alpha_pend2 = 0.0;
    if (!(val[0] > 0.0) || !isfinite(val[0])) {
      sc->breakdown = isfinite(val[0]) ? 1 : 2;
      sc->done = 1;
      sc->alpha_pend = 0.0;
    } else {
      sc->alpha = sc->rz / val[0];
    }
    break;
  case PH_PQ_SKIP:
    // Jacobi-PCG, after a sweep A that left x alone: the step owed on the
    // old direction moves one place back (the next sweep A applies both);
    // on a breakdown it stays owed on the old direction alone
    sc->pq = val[0];
    if (!(val[0] > 0.0) || !isfinite(val[0])) {
      sc->breakdown = isfinite(val[0]) ? 1 : 2;
      sc->done = 1;
      sc->alpha_pend2 = 0.0;
    } else {
      sc->alpha_pend2 = sc->alpha_pend;
      sc->alpha = sc->rz / val[0];
    }
    break;
  case PH_UPD: {
    const double rzn = val[0], rr = val[1];
    sc->beta = rzn / sc->rz;
    sc->rz_prev = sc->rz;
    sc->rz = rzn;
    sc->rr = rr;
    sc->alpha_pend = sc->alpha;
    sc->iter += 1;
    if (hist && sc->iter <= sc->max_iter && sc->iter <= kHistCap) hist[sc->iter] = rr;
    if (!isfinite(rr) || !isfinite(rzn)) { sc->breakdown = 2; sc->done = 1; }
    else if (rr <= sc->tol2) sc->done = 1;
    else if (sc->iter >= sc->max_iter) sc->done = 1;
    else if (stalled_now(sc, hist)) { sc->stalled = 1; sc->done = 1; }
    break;
  }
  case PH_ZQ:   // flexible CG: beta = -(z.q_prev)/(p_prev.q_prev), 0 on the first step
    sc->zq = val[0];
    sc->beta = (sc->pq > 0.0 && isfinite(val[0])) ? -val[0] / sc->pq : 0.0;
    break;
  case PH_PR:
    sc->pr = val[0];
    break;
  case PH_PQF:   // (p.q, p.r) from the flexible sweep A
    sc->pq = val[0];
    sc->pr = val[1];
    if (!(val[0] > 0.0) || !isfinite(val[0]) || !isfinite(val[1])) {
      sc->breakdown = isfinite(val[0]) && isfinite(val[1]) ? 1 : 2;
      sc->done = 1;
      sc->alpha_pend = 0.0;
      sc->alpha_pend2 = 0.0;
    } else {
      sc->alpha = val[1] / val[0];
    }
    break;
  case PH_RELIABLE:
    // residual replaced: (r.z, r.r) of the true residual.  CG continues with
    // the same p: the next direction is z + beta p with beta = r.z / (r.z of
    // the step before the last update), the recursion's own beta with the
    // replaced residual in its numerator.  (Dividing by the last r.z, which
    // the replaced residual nearly equals, gives beta ~ 1: a direction no
    // longer conjugate to p, which cost the FP32 solve 30-60 % more
    // iterations.)
    sc->beta = val[0] / sc->rz_prev;
    sc->rz = val[0];
    sc->rr = val[1];
    sc->alpha_pend = 0.0;
    sc->alpha_pend2 = 0.0;
    sc->done = 0;
    sc->breakdown = 0;
    sc->stalled = 0;
    if (!isfinite(val[0]) || !isfinite(val[1])) { sc->breakdown = 2; sc->done = 1; }
    else if (val[1] <= sc->tol2) sc->done = 1;
    break;
  case PH_RELIABLE_F:  // flexible CG: residual replaced, (r.r)
    sc->rr = val[0];
    sc->alpha_pend = 0.0;
    sc->alpha_pend2 = 0.0;
    sc->done = 0;
    sc->breakdown = 0;
    sc->stalled = 0;
    if (!isfinite(val[0])) { sc->breakdown = 2; sc->done = 1; }
    else if (val[0] <= sc->tol2) sc->done = 1;
    break;
  case PH_UPDF: {
    const double rr = val[0];
    sc->rr = rr;
    sc->alpha_pend = sc->alpha;
    sc->iter += 1;
    if (hist && sc->iter <= sc->max_iter && sc->iter <= kHistCap) hist[sc->iter] = rr;
    if (!isfinite(rr)) { sc->breakdown = 2; sc->done = 1; }
    else if (rr <= sc->tol2) sc->done = 1;
    else if (sc->iter >= sc->max_iter) sc->done = 1;
    else if (stalled_now(sc, hist)) { sc->stalled = 1; sc->done = 1; }
    break;
  }
  default:
    break;
}
}


}  // namespace nfa
