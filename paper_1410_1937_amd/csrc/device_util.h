// Device helpers shared by the libnfa kernels: wave64 / block reductions in
// a fixed order (results are bitwise reproducible run to run), XCD-aware
// block remapping, and the solver-state early exit.
#pragma once

#include <hip/hip_runtime.h>

#include "nfa_internal.h"

namespace nfa {

// Sum over the 64 lanes of a wavefront by butterfly shuffles (fixed order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Block sum of a double; the result is valid in thread 0.  `lds` must hold
// at least blockDim/64 doubles.  Every thread of the block must call it.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int nthreads = blockDim.x * blockDim.y;
  v = wave_sum(v);
  const int lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0) {
    const int nw = (nthreads + 63) >> 6;
    for (int w = 0; w < nw; ++w) r += lds[w];
  }
  return r;
}

// Consecutive workgroup ids land on different XCDs (round robin over 8).
// Remap so that each XCD works on a contiguous range of logical tiles and
// neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int per = nb >> 3;
  const int full = per << 3;
  if (b >= full) return b;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ bool solve_done(const SolveScalars* sc) {
  return sc != nullptr && sc->done != 0;
}

}  // namespace nfa
