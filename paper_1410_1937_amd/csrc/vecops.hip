// libnfa: vector kernels of the Krylov solvers and fixed-order reductions.
//
// Every reduction writes one partial per workgroup (fixed grid, fixed
// element-to-thread map) and a single workgroup sums the partials in index
// order, so dot products are bitwise reproducible run to run; there are no
// floating-point atomics.  FP32 vectors accumulate their products in FP64.
// Solver scalars (alpha, beta, norms, iteration count, convergence flag) stay
// on the device (SolveScalars) so that iterations need no host round trip.
#include <algorithm>
#include <cmath>

#include "device_util.h"
#include "nfa_internal.h"
#include "vecops.h"
#include "phase.h"

namespace nfa {
namespace {

#define GRID_STRIDE(idx, n) \
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (n); idx += (long long)gridDim.x * blockDim.x)

constexpr int kVecBlocks = 2048;

inline int vec_blocks(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b > kVecBlocks) b = kVecBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_dot(long long n, const T* __restrict__ a,
                                                const T* __restrict__ b, double* partials,
                                                const SolveScalars* sc) {
  if (solve_done(sc)) return;
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += (double)a[i] * (double)b[i];
  const double t = block_sum(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_masked_sum(long long n, const T* __restrict__ a,
                                                       const unsigned char* __restrict__ m,
                                                       double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += m[i] ? (double)a[i] : 0.0;
  const double t = block_sum(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void k_sub_mean(long long n, double* b, const unsigned char* __restrict__ m,
                           const double* sum, double count) {
  const double mean = *sum / count;
  GRID_STRIDE(i, n) if (m[i]) b[i] = b[i] - mean;
}

// out[c] = sum_i partials[c*kMaxPartials + i], fixed order
__global__ __launch_bounds__(1024) void k_sum_partials(const double* partials, int n, int ncomp,
                                                        double* out) {
  __shared__ double lds[1024 / 64];
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += partials[(size_t)c * kMaxPartials + i];
    const double t = block_sum(acc, lds);
    if (threadIdx.x == 0) out[c] = t;
    __syncthreads();
  }
}

// Finalize a reduction and advance the solver state; run by one workgroup of
// 1024 threads (every thread of that workgroup must call it).
__device__ __forceinline__ void finalize_block(const double* partials, int n, int ncomp, int phase,
                                               SolveScalars* sc, double* hist) {
  if (phase != PH_BB && phase != PH_RR && phase != PH_RRO && phase != PH_INIT && phase != PH_RELIABLE &&
      phase != PH_RELIABLE_F && sc->done)
    return;
  __shared__ double lds[2][1024 / 64];
  __shared__ double val[4];
  // both components' partials in one pass (their loads in flight together)
  double acc0 = 0.0, acc1 = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    acc0 += partials[i];
    if (ncomp > 1) acc1 += partials[(size_t)kMaxPartials + i];
  }
  const double t0 = block_sum(acc0, lds[0]);
  const double t1 = ncomp > 1 ? block_sum(acc1, lds[1]) : 0.0;
  if (threadIdx.x == 0) {
    val[0] = t0;
    val[1] = t1;
    apply_phase(phase, ncomp, val, sc, hist);
  }
}

__global__ __launch_bounds__(1024) void k_finalize(const double* partials, int n, int ncomp, int phase,
                                                    SolveScalars* sc, double* hist) {
  finalize_block(partials, n, ncomp, phase, sc, hist);
}

// Workgroup 0 finalizes a reduction; the others apply a merge operation the
// reduction does not depend on (the dots of the merged system need neither
// the gathered q nor the copied z: slaves carry r = 0 and p equal to their
// root's).  GATHER: v[root] += v[slaves] in ascending member order, slaves
// set to 0.  Otherwise: v[slave] = v[root].  Both are idempotent, so the
// merge part runs whatever the solver state says (no read of the flag the
// finalizing workgroup may be writing).
template <class T, bool GATHER>
__global__ __launch_bounds__(1024) void k_finalize_merge(const double* partials, int n, int ncomp,
                                                          int phase, SolveScalars* sc, double* hist,
                                                          int cnt, const int* __restrict__ ia,
                                                          const int* __restrict__ ib,
                                                          const int* __restrict__ ic, T* v) {
  if (blockIdx.x == 0) {
    finalize_block(partials, n, ncomp, phase, sc, hist);
    return;
  }
  const int stride = (gridDim.x - 1) * blockDim.x;
  for (int t = (blockIdx.x - 1) * blockDim.x + threadIdx.x; t < cnt; t += stride) {
    if (GATHER) {
      // the members' values are loaded together (groups have at most a few
      // dozen members; the first 16 in one round), then added in order
      const int r = ia[t], m0 = ib[t], m1 = ib[t + 1];
      T acc = v[r];
      T mv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) mv[k] = m0 + k < m1 ? v[ic[m0 + k]] : T(0);
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (m0 + k < m1) acc = acc + mv[k];
      for (int m = m0 + 16; m < m1; ++m) acc = acc + v[ic[m]];
      for (int m = m0; m < m1; ++m) v[ic[m]] = T(0);
      v[r] = acc;
    } else {
      v[ia[t]] = v[ib[t]];
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_jacobi(long long n, const T* __restrict__ r,
                                                   const T* __restrict__ dinv, T* __restrict__ z,
                                                   double* partials) {
  __shared__ double lds[2 * kBlock / 64];
  double rz = 0.0, rr = 0.0;
  GRID_STRIDE(i, n) {
    const T ri = r[i];
    const T zi = dinv[i] * ri;
    z[i] = zi;
    rz += (double)ri * (double)zi;
    rr += (double)ri * (double)ri;
  }
  const double t0 = block_sum(rz, lds);
  const double t1 = block_sum(rr, lds + kBlock / 64);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = t0;
    partials[kMaxPartials + blockIdx.x] = t1;
  }
}

// preconditioner z = dinv r (no reduction), early exit with the solver state
template <class T>
__global__ void k_scale(long long n, const T* __restrict__ r, const T* __restrict__ dinv,
                        T* __restrict__ z, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  GRID_STRIDE(i, n) z[i] = dinv[i] * r[i];
}

// test hook: a fixed field unrelated to r (stands in for a broken preconditioner)
template <class T>
__global__ void k_sabotage(long long n, const unsigned char* __restrict__ red, T* __restrict__ z,
                           const SolveScalars* sc) {
  if (solve_done(sc)) return;
  GRID_STRIDE(i, n) {
    unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ull + (unsigned long long)sc->iter;
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    z[i] = red[i] ? (T)(1e-6 * u) : T(0);
  }
}

template <class T>
__global__ void k_copy(long long n, const T* __restrict__ a, T* __restrict__ b) {
  GRID_STRIDE(i, n) b[i] = a[i];
}

template <class T>
__global__ void k_fill(long long n, T* a, T v) {
  GRID_STRIDE(i, n) a[i] = v;
}

__global__ void k_init_x(long long n, double* x, const unsigned char* act, int warm) {
  GRID_STRIDE(i, n) x[i] = (warm && act[i]) ? x[i] : 0.0;
}

// tol_mode 0: tol2 = t * bb; 1: tol2 = t (absolute)
__global__ void k_set_scalars(SolveScalars* sc, double t, int tol_mode, int max_iter, int reset_iter,
                              int window, double ratio) {
  sc->tol2 = tol_mode == 0 ? t * sc->bb : t;
  sc->window = window;
  sc->ratio = ratio;
  sc->max_iter = max_iter;
  sc->done = 0;
  sc->breakdown = 0;
  sc->stalled = 0;
  if (reset_iter) sc->iter = 0;
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <class T> int launch_masked_sum(const T* a, const unsigned char* mask, long long n,
                                         double* partials, hipStream_t s) {
  const int nb = vec_blocks(n);
  k_masked_sum<T><<<nb, kBlock, 0, s>>>(n, a, mask, partials);
  return nb;
}
template int launch_masked_sum<double>(const double*, const unsigned char*, long long, double*, hipStream_t);
template int launch_masked_sum<float>(const float*, const unsigned char*, long long, double*, hipStream_t);

void launch_sub_mean(double* b, const unsigned char* mask, long long n, const double* sum,
                     double count, hipStream_t s) {
  k_sub_mean<<<vec_blocks(n), kBlock, 0, s>>>(n, b, mask, sum, count);
}

void launch_sum_partials(const double* partials, int n, int ncomp, double* out, hipStream_t s) {
  k_sum_partials<<<1, 1024, 0, s>>>(partials, n, ncomp, out);
}

void launch_finalize(const double* partials, int n, int ncomp, int phase, SolveScalars* sc,
                     double* hist, hipStream_t s) {
  k_finalize<<<1, 1024, 0, s>>>(partials, n, ncomp, phase, sc, hist);
}

template <class T>
void launch_finalize_merge(const Grid& g, bool gather, T* v, const double* partials, int n, int ncomp,
                           int phase, SolveScalars* sc, double* hist, hipStream_t s) {
  const int cnt = gather ? g.n_groups : g.n_slaves;
  if (cnt == 0) {
    k_finalize<<<1, 1024, 0, s>>>(partials, n, ncomp, phase, sc, hist);
    return;
  }
  const int mb = std::min(64, (cnt + 1023) / 1024);
  if (gather)
    k_finalize_merge<T, true><<<1 + mb, 1024, 0, s>>>(partials, n, ncomp, phase, sc, hist, cnt,
                                                      g.g_root.as<int>(), g.g_off.as<int>(),
                                                      g.g_mem.as<int>(), v);
  else
    k_finalize_merge<T, false><<<1 + mb, 1024, 0, s>>>(partials, n, ncomp, phase, sc, hist, cnt,
                                                       g.s_cell.as<int>(), g.s_root.as<int>(), nullptr, v);
}
template void launch_finalize_merge<double>(const Grid&, bool, double*, const double*, int, int, int,
                                            SolveScalars*, double*, hipStream_t);
template void launch_finalize_merge<float>(const Grid&, bool, float*, const double*, int, int, int,
                                           SolveScalars*, double*, hipStream_t);

template <class T> int launch_dot(const T* a, const T* b, long long n, double* partials,
                                  const SolveScalars* sc, hipStream_t s) {
  const int nb = vec_blocks(n);
  k_dot<T><<<nb, kBlock, 0, s>>>(n, a, b, partials, sc);
  return nb;
}
template int launch_dot<double>(const double*, const double*, long long, double*, const SolveScalars*, hipStream_t);
template int launch_dot<float>(const float*, const float*, long long, double*, const SolveScalars*, hipStream_t);

template <class T> int launch_jacobi(const T* r, const T* dinv, T* z, long long n, double* partials,
                                     hipStream_t s) {
  const int nb = vec_blocks(n);
  k_jacobi<T><<<nb, kBlock, 0, s>>>(n, r, dinv, z, partials);
  return nb;
}
template int launch_jacobi<double>(const double*, const double*, double*, long long, double*, hipStream_t);
template int launch_jacobi<float>(const float*, const float*, float*, long long, double*, hipStream_t);

template <class T> void launch_scale(const T* r, const T* dinv, T* z, long long n, const SolveScalars* sc,
                                     hipStream_t s) {
  k_scale<T><<<vec_blocks(n), kBlock, 0, s>>>(n, r, dinv, z, sc);
}
template void launch_scale<double>(const double*, const double*, double*, long long, const SolveScalars*, hipStream_t);
template void launch_scale<float>(const float*, const float*, float*, long long, const SolveScalars*, hipStream_t);

template <class T> void launch_sabotage(const unsigned char* red, T* z, long long n, const SolveScalars* sc,
                                        hipStream_t s) {
  k_sabotage<T><<<vec_blocks(n), kBlock, 0, s>>>(n, red, z, sc);
}
template void launch_sabotage<double>(const unsigned char*, double*, long long, const SolveScalars*, hipStream_t);
template void launch_sabotage<float>(const unsigned char*, float*, long long, const SolveScalars*, hipStream_t);

template <class T> void launch_copy(const T* a, T* b, long long n, hipStream_t s) {
  k_copy<T><<<vec_blocks(n), kBlock, 0, s>>>(n, a, b);
}
template void launch_copy<double>(const double*, double*, long long, hipStream_t);
template void launch_copy<float>(const float*, float*, long long, hipStream_t);

template <class T> void launch_fill(T* a, T v, long long n, hipStream_t s) {
  k_fill<T><<<vec_blocks(n), kBlock, 0, s>>>(n, a, v);
}
template void launch_fill<double>(double*, double, long long, hipStream_t);
template void launch_fill<float>(float*, float, long long, hipStream_t);

void launch_init_x(double* x, const unsigned char* act, long long n, int warm, hipStream_t s) {
  k_init_x<<<vec_blocks(n), kBlock, 0, s>>>(n, x, act, warm);
}
void launch_set_scalars(SolveScalars* sc, double t, int tol_mode, int max_iter, int reset_iter,
                        int window, double ratio, hipStream_t s) {
  k_set_scalars<<<1, 1, 0, s>>>(sc, t, tol_mode, max_iter, reset_iter, window, ratio);
}

}  // namespace nfa

namespace {
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;
constexpr long long kChunk = 256LL * kCopyUnroll;   // 16-byte words per workgroup (16 KB)

// Both streaming kernels give each workgroup one contiguous 16 KB chunk, and
// each XCD a contiguous range of chunks (workgroups are dealt to the XCDs
// round robin).  Measured at 1 GiB on MI355X, that order moves 6.0 TB/s
// (copy, read + written) and 6.4 TB/s (writes only), against 5.1 and 4.4
// TB/s for a grid-stride loop over the whole array.
__device__ __forceinline__ long long stream_chunk(int per) {
  return (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// dst = src in 16-byte words: kCopyUnroll non-temporal loads in flight per lane
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     long long n, int per) {
  const long long i = stream_chunk(per) * kChunk + threadIdx.x;
  if (i + (kCopyUnroll - 1) * 256 < n) {
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * 256);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * 256);
  } else {
    for (int u = 0; u < kCopyUnroll; ++u)
      if (i + u * 256 < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i + u * 256), dst + i + u * 256);
  }
}

// dst = v in every 16-byte word, plain stores (the form the convolutions'
// outputs use)
__global__ __launch_bounds__(256) void k_stream_fill(u32x4* __restrict__ dst, unsigned v, long long n, int per) {
  const long long i = stream_chunk(per) * kChunk + threadIdx.x;
  const u32x4 w = {v, v, v, v};
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u)
    if (i + u * 256 < n) dst[i + u * 256] = w;
}

// chunks per XCD for n words
int stream_per(long long n) { return (int)(((n + kChunk - 1) / kChunk + 7) / 8); }
}  // namespace

extern "C" nfa_status nfa_stream_copy(void* dst, const void* src, size_t bytes, nfa_stream s) {
  using namespace nfa;
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0)
    return fail(NFA_ERR_INVALID, "nfa_stream_copy: pointers and size must be multiples of 16 bytes");
  if (bytes == 0) return NFA_OK;
  if (dst == nullptr || src == nullptr) return fail(NFA_ERR_INVALID, "nfa_stream_copy: null pointer");
  const long long n = (long long)(bytes / 16);
  const int per = stream_per(n);
  k_stream_copy<<<8 * per, 256, 0, S(s)>>>(reinterpret_cast<const u32x4*>(src), reinterpret_cast<u32x4*>(dst), n, per);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

extern "C" nfa_status nfa_stream_fill(void* dst, unsigned value, size_t bytes, nfa_stream s) {
  using namespace nfa;
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return fail(NFA_ERR_INVALID, "nfa_stream_fill: pointer and size must be multiples of 16 bytes");
  if (bytes == 0) return NFA_OK;
  if (dst == nullptr) return fail(NFA_ERR_INVALID, "nfa_stream_fill: null pointer");
  const long long n = (long long)(bytes / 16);
  const int per = stream_per(n);
  k_stream_fill<<<8 * per, 256, 0, S(s)>>>(reinterpret_cast<u32x4*>(dst), value, n, per);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}
