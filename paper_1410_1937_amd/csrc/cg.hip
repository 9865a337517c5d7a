// libnfa: fused conjugate-gradient sweeps.
//
// One CG iteration is two streaming sweeps over the grid:
//   sweep A:  p  = z + beta p_old            (new search direction)
//             q  = A p                        (flux-form 7-point operator)
//             x += alpha_prev p_old           (update deferred from the
//                                              previous iteration)
//             partials p.q (and p.r for flexible CG)
//             (Jacobi-PCG defers further: every other sweep A leaves x
//             alone, and the next one applies both owed steps,
//             x = (x + alpha_(k-2) p_(k-2)) + alpha_(k-1) p_(k-1), bitwise
//             the two updates one after the other; p is kept in three
//             buffers for it)
//   sweep B:  z -= alpha D^-1 q               partials r.z, r.r
//             (Jacobi-PCG carries the preconditioned residual z = D^-1 r as
//             its state: r = z / D^-1 where D^-1 > 0 and 0 elsewhere is
//             formed for the partials only, so r is neither read nor written;
//             flexible CG: r -= alpha q, partial r.r, and the preconditioner
//             runs as its own pass)
// so the direction update and the x update cost no extra pass: Jacobi-PCG
// moves 100 B/cell per iteration in FP64 (sweep A 56 or 80, 68 on average,
// + 32), 50 B/cell in FP32 (28 or 40, 34 on average, + 16), against 128 / 64
// B for the textbook three-pass form.  p is double-buffered in flexible CG and
// triple-buffered in Jacobi-PCG (the neighbours of a cell must see the old
// direction).
//
// Launch shape of sweep A: a workgroup is a tile of WX wavefronts across x
// by AY rows in y (WX * AY = 16 wavefronts).  Each lane owns V consecutive x
// cells (one 16-byte vector: V = 2 doubles or 4 floats) and marches up a
// contiguous range of z-planes keeping the new direction of planes k-1, k,
// k+1 and the coefficient of face k in registers.  Per plane, the tile's new
// direction and its lower y-face coefficients are exchanged through LDS
// (double-buffered, one barrier per plane): y-neighbours inside the tile and
// x-neighbours across wavefront edges come from LDS, x-neighbours inside a
// wavefront from shuffles, and only the tile's outer rows and columns read
// their neighbours through the caches.  The grid is persistent (one
// workgroup per resident slot) and the (column tile, plane) work is split
// into equal contiguous ranges, so no workgroup waits on a partly filled
// last round; workgroup ids are remapped so that each XCD owns a contiguous
// block of y-adjacent column tiles (shared L2 halos).
// The operator sum keeps the order x-, x+, y-, y+, z-, z+ (FP contraction is
// off), so q is bitwise the value of the plain sweep.
#include "device_util.h"
#include "nfa_internal.h"
#include "sweep_tile.h"
#include "vecops.h"

#include <map>
#include <mutex>
#include <tuple>

namespace nfa {
namespace {

using namespace tile;

// Where the non-temporal hint pays was measured per sweep and precision on the
// 512 x 256 x 192 grid (sweep A: loads and stores in FP32, stores only in
// FP64; sweep B: loads in FP32, loads and stores in FP64).
template <class T> struct StreamHints {
  static constexpr bool a_load = sizeof(T) == 4, a_store = true;
  static constexpr bool b_load = true, b_store = sizeof(T) == 8;
};

// new direction z + beta p_old of V cells
template <class T, int V>
__device__ __forceinline__ Pack<T, V> dir(const T* z, const T* po, long long c, T beta) {
  const Pack<T, V> a = ld<T, V>(z + c), b = ld<T, V>(po + c);
  Pack<T, V> r;
#pragma unroll
  for (int e = 0; e < V; ++e) r.v[e] = a.v[e] + beta * b.v[e];
  return r;
}

// XM: the x update of this sweep: 0 none (the step on p_old stays owed), 1
// x += alpha_pend p_old, 2 x = (x + alpha_pend2 p_old2) + alpha_pend p_old
template <class T, int V, int WX, bool FLEX, int XM>
__global__ __launch_bounds__(AX* kTileWaves) void k_cg_a(
    int nx, int ny, int nz, int tiles_x, long long ncol, long long per_block,
    const T* __restrict__ z, const T* __restrict__ pold, const T* __restrict__ pold2, T* __restrict__ pnew,
    T* __restrict__ x,
    const T* __restrict__ r, const T* __restrict__ tx, const T* __restrict__ txb,
    const T* __restrict__ ty, const T* __restrict__ tz, T* __restrict__ q,
    double* __restrict__ partials, const SolveScalars* __restrict__ sc) {
  constexpr int AY = kTileWaves / WX;
  constexpr int TW = WX * AX;  // vectors per tile row
  if (solve_done(sc)) return;
  __shared__ Pack<T, V> shp[2][AY][TW];  // new direction of the current plane
  __shared__ Pack<T, V> sht[2][AY][TW];  // lower y-face coefficient of the current plane
  __shared__ double lds[2 * kTileWaves];
  const T beta = (T)sc->beta;
  const T apend = (T)sc->alpha_pend;
  const T apend2 = (T)sc->alpha_pend2;
  const int lane = threadIdx.x;
  const int wx = threadIdx.y % WX, row = threadIdx.y / WX;
  const int col = wx * AX + lane;
  const long long plane = (long long)nx * ny;
  const long long yplane = (long long)(ny + 1) * nx;
  double acc_pq = 0.0, acc_pr = 0.0;
  const long long L = xcd_remap(blockIdx.x, gridDim.x);
  long long u = L * per_block;
  const long long uend = min(ncol * nz, u + per_block);
  // every wavefront of the workgroup walks the same (tile, plane) sequence,
  // so the barrier below is reached the same number of times by all
  while (u < uend) {
    const long long ct = u / nz;
    const int k0 = (int)(u - ct * nz);
    const int k1 = (int)min((long long)nz, k0 + (uend - u));
    u += k1 - k0;
    const int bx = (int)(ct % tiles_x);
    const int by = (int)(ct / tiles_x);
    const int j = by * AY + row;
    const int i0 = (bx * TW + col) * V;
    const bool live = j < ny && i0 < nx;
    long long c = (long long)k0 * plane + (long long)j * nx + i0;
    long long yi = ((long long)k0 * (ny + 1) + j) * nx + i0;
    const bool lbdy = i0 == 0, rbdy = i0 + V >= nx;
    const bool ledge = lane == 0 && !lbdy, redge = lane == AX - 1 && !rbdy;
    const bool lglob = ledge && wx == 0, rglob = redge && wx == WX - 1;
    const bool ylo = j > 0, yhi = j < ny - 1;
    const bool yin_lo = ylo && row > 0, yin_hi = yhi && row < AY - 1;
    Pack<T, V> pm = zero<T, V>(), pc = zero<T, V>(), poc = zero<T, V>(), tzc = zero<T, V>();
    if (live) {
      if (k0 > 0) pm = dir<T, V>(z, pold, c - plane, beta);
      poc = ld<T, V>(pold + c);
      const Pack<T, V> zc = ld<T, V>(z + c);
#pragma unroll
      for (int e = 0; e < V; ++e) pc.v[e] = zc.v[e] + beta * poc.v[e];
      tzc = ld<T, V>(tz + c);
    }
    for (int k = k0; k < k1; ++k, c += plane, yi += yplane) {
      Pack<T, V> pp = zero<T, V>(), pop = zero<T, V>(), tzp = zero<T, V>();
      Pack<T, V> txv = zero<T, V>(), tym = zero<T, V>(), typ = zero<T, V>();
      Pack<T, V> pym = zero<T, V>(), pyp = zero<T, V>();
      T left = T(0), right = T(0), txr = T(0);
      if (live) {
        if (k + 1 < nz) {
          pop = ld_stream<StreamHints<T>::a_load, T, V>(pold + c + plane);
          const Pack<T, V> zp = ld_stream<StreamHints<T>::a_load, T, V>(z + c + plane);
#pragma unroll
          for (int e = 0; e < V; ++e) pp.v[e] = zp.v[e] + beta * pop.v[e];
        }
        tzp = ld_stream<StreamHints<T>::a_load, T, V>(tz + c + plane);
        txv = ld_stream<StreamHints<T>::a_load, T, V>(tx + c);
        tym = ld_stream<StreamHints<T>::a_load, T, V>(ty + yi);
        if (!yin_hi) typ = ld<T, V>(ty + yi + nx);
        if (ylo && row == 0) pym = dir<T, V>(z, pold, c - nx, beta);
        if (yhi && row == AY - 1) pyp = dir<T, V>(z, pold, c + nx, beta);
        if (lglob) left = z[c - 1] + beta * pold[c - 1];
        if (rglob) right = z[c + V] + beta * pold[c + V];
        if (redge) txr = tx[c + V];
        else if (rbdy) txr = txb[(long long)k * ny + j];
      }
      const int b = k & 1;
      shp[b][row][col] = pc;
      sht[b][row][col] = tym;
      __syncthreads();
      if (live) {
        if (yin_lo) pym = shp[b][row - 1][col];
        if (yin_hi) {
          pyp = shp[b][row + 1][col];
          typ = sht[b][row + 1][col];
        }
        if (ledge && wx > 0) left = shp[b][row][col - 1].v[V - 1];
        if (redge && wx < WX - 1) right = shp[b][row][col + 1].v[0];
      }
      // neighbours inside the wavefront (all lanes take part)
      const T sl = __shfl_up(pc.v[V - 1], 1, AX);
      const T sr = __shfl_down(pc.v[0], 1, AX);
      const T st0 = __shfl_down(txv.v[0], 1, AX);
      if (!lbdy && !ledge) left = sl;
      if (!rbdy && !redge) {
        right = sr;
        txr = st0;
      }
      if (live) {
        Pack<T, V> qv;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const T p0 = pc.v[e];
          const T pxm = e == 0 ? left : pc.v[e - 1];
          const T pxp = e == V - 1 ? right : pc.v[e + 1];
          const T txm = txv.v[e];
          const T txp = e == V - 1 ? txr : txv.v[e + 1];
          T s = txm * (p0 - pxm);
          s = s + txp * (p0 - pxp);
          s = s + tym.v[e] * (p0 - pym.v[e]);
          s = s + typ.v[e] * (p0 - pyp.v[e]);
          s = s + tzc.v[e] * (p0 - pm.v[e]);
          s = s + tzp.v[e] * (p0 - pp.v[e]);
          qv.v[e] = s;
          acc_pq += (double)p0 * (double)s;
        }
        st_stream<StreamHints<T>::a_store, T, V>(q + c, qv);
        st_stream<StreamHints<T>::a_store, T, V>(pnew + c, pc);
        if constexpr (XM == 1) {
          Pack<T, V> xv = ld_stream<StreamHints<T>::a_load, T, V>(x + c);
#pragma unroll
          for (int e = 0; e < V; ++e) xv.v[e] = xv.v[e] + apend * poc.v[e];
          st_stream<StreamHints<T>::a_store, T, V>(x + c, xv);
        } else if constexpr (XM == 2) {
          Pack<T, V> xv = ld_stream<StreamHints<T>::a_load, T, V>(x + c);
          const Pack<T, V> p2 = ld_stream<StreamHints<T>::a_load, T, V>(pold2 + c);
#pragma unroll
          for (int e = 0; e < V; ++e) xv.v[e] = (xv.v[e] + apend2 * p2.v[e]) + apend * poc.v[e];
          st_stream<StreamHints<T>::a_store, T, V>(x + c, xv);
        }
        if (FLEX) {
          const Pack<T, V> rv = ld_stream<StreamHints<T>::a_load, T, V>(r + c);
#pragma unroll
          for (int e = 0; e < V; ++e) acc_pr += (double)pc.v[e] * (double)rv.v[e];
        }
      }
      pm = pc;
      pc = pp;
      poc = pop;
      tzc = tzp;
    }
  }
  const double t0 = block_sum(acc_pq, lds);
  if (FLEX) {
    const double t1 = block_sum(acc_pr, lds + kTileWaves);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[kMaxPartials + blockIdx.x] = t1;
  }
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[blockIdx.x] = t0;
}

constexpr int kCgbBlocks = 2048;

// Jacobi-PCG sweep B: z -= alpha (D^-1 q); partials r.z = sum z^2 / D^-1 and
// r.r = sum (z / D^-1)^2 over the cells with D^-1 > 0 (slaves and inactive
// cells have D^-1 = 0: their z is left as it is and overwritten by the merge
// copy that follows), r formed in FP64
template <class T, int V>
__global__ __launch_bounds__(kBlock) void k_cg_bz(long long nvec, T* __restrict__ z, const T* __restrict__ q,
                                                  const T* __restrict__ dinv, double* __restrict__ partials,
                                                  const SolveScalars* __restrict__ sc) {
  if (solve_done(sc)) return;
  __shared__ double lds[2 * kBlock / 64];
  const T alpha = (T)sc->alpha;
  double rz = 0.0, rr = 0.0;
  for (long long iv = blockIdx.x * (long long)blockDim.x + threadIdx.x; iv < nvec;
       iv += (long long)gridDim.x * blockDim.x) {
    const long long c = iv * V;
    Pack<T, V> zv = ld_stream<StreamHints<T>::b_load, T, V>(z + c);
    const Pack<T, V> qv = ld_stream<StreamHints<T>::b_load, T, V>(q + c);
    const Pack<T, V> dv = ld_stream<StreamHints<T>::b_load, T, V>(dinv + c);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      zv.v[e] = zv.v[e] - alpha * (dv.v[e] * qv.v[e]);
      if (dv.v[e] > T(0)) {
        const double rd = (double)zv.v[e] / (double)dv.v[e];
        rz += rd * (double)zv.v[e];
        rr += rd * rd;
      }
    }
    st_stream<StreamHints<T>::b_store, T, V>(z + c, zv);
  }
  const double t0 = block_sum(rz, lds);
  const double t1 = block_sum(rr, lds + kBlock / 64);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = t0;
    partials[kMaxPartials + blockIdx.x] = t1;
  }
}

// flexible CG sweep B: r -= alpha q; partial r.r (the preconditioner runs as
// its own pass)
template <class T, int V>
__global__ __launch_bounds__(kBlock) void k_cg_b(long long nvec, T* __restrict__ r, const T* __restrict__ q,
                                                 double* __restrict__ partials, const SolveScalars* __restrict__ sc) {
  if (solve_done(sc)) return;
  __shared__ double lds[kBlock / 64];
  const T alpha = (T)sc->alpha;
  double rr = 0.0;
  for (long long iv = blockIdx.x * (long long)blockDim.x + threadIdx.x; iv < nvec;
       iv += (long long)gridDim.x * blockDim.x) {
    const long long c = iv * V;
    Pack<T, V> rv = ld_stream<StreamHints<T>::b_load, T, V>(r + c);
    const Pack<T, V> qv = ld_stream<StreamHints<T>::b_load, T, V>(q + c);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      rv.v[e] = rv.v[e] - alpha * qv.v[e];
      rr += (double)rv.v[e] * (double)rv.v[e];
    }
    st_stream<StreamHints<T>::b_store, T, V>(r + c, rv);
  }
  const double t = block_sum(rr, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// the x updates still owed when the iteration stopped: x += alpha_pend p, or
// with p2 (Jacobi-PCG) x = (x + alpha_pend2 p2) + alpha_pend p, the order of
// sweep A's two-step update.  p2 is not read when nothing is owed on it: a
// phase stopped before its second iteration has never written that buffer.
template <class T>
__global__ void k_cg_fixup(long long n, T* __restrict__ x, const T* __restrict__ p, const T* __restrict__ p2,
                           const SolveScalars* __restrict__ sc) {
  const T a = (T)sc->alpha_pend;
  const T a2 = (T)sc->alpha_pend2;
  const bool two = p2 && a2 != T(0);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = two ? (x[i] + a2 * p2[i]) + a * p[i] : x[i] + a * p[i];
}

// x64 += x32 * inv_scale; x32 = 0
__global__ void k_fold(long long n, double* __restrict__ x, float* __restrict__ d, double inv_scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    x[i] = x[i] + (double)d[i] * inv_scale;
    d[i] = 0.0f;
  }
}

// r32 = float(r64 * scale)
__global__ void k_cast(long long n, const double* __restrict__ r, float* __restrict__ r32, double scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    r32[i] = (float)(r[i] * scale);
}

inline int vblocks(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (int)std::max(1LL, std::min(b, (long long)kCgbBlocks));
}

}  // namespace

template <class T>
bool cg_vectorizable(const Grid& g, const void* const* ptrs, int nptr) {
  constexpr int V = tile::vec_width<T>();
  if (g.nx % V != 0) return false;
  for (int i = 0; i < nptr; ++i)
    if (reinterpret_cast<uintptr_t>(ptrs[i]) % 16 != 0) return false;
  return true;
}

int resident_blocks(const void* fn, int threads) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  const int nb = std::min(kMaxPartials, per_cu * cus);
  cache[fn] = nb;
  return nb;
}

// sweep A; returns the number of workgroup partials per component
template <class T>
int launch_cg_a(const Grid& g, const Coeffs<T>& C, const T* z, const T* pold, const T* pold2, T* pnew,
                T* x, const T* r, T* q, double* partials, const SolveScalars* sc, bool flex, int xm,
                bool vec, hipStream_t s) {
  const int V = vec ? tile::vec_width<T>() : 1;
  const int wx = tile_wx<T>(g, V);
  const int ay = kTileWaves / wx;
  const int tiles_x = (g.nx + AX * wx * V - 1) / (AX * wx * V);
  const long long ncol = (long long)tiles_x * ((g.ny + ay - 1) / ay);
  dim3 blk(AX, kTileWaves);
  int nb = 0;
#define CGA(VV, WW, FF, XX)                                                                      \
  do {                                                                                           \
    const void* fn = reinterpret_cast<const void*>(&k_cg_a<T, VV, WW, FF, XX>);                  \
    nb = resident_blocks(fn, AX * kTileWaves);                                                   \
    const long long per = (ncol * g.nz + nb - 1) / nb;                                           \
    k_cg_a<T, VV, WW, FF, XX><<<nb, blk, 0, s>>>(g.nx, g.ny, g.nz, tiles_x, ncol, per, z, pold, pold2, \
                                                 pnew, x, r, C.tx, C.txb, C.ty, C.tz, q, partials, sc); \
  } while (0)
#define CGA_X(VV, WW)                                 \
  do {                                                \
    if (flex) CGA(VV, WW, true, 1);                   \
    else if (xm == 2) CGA(VV, WW, false, 2);          \
    else CGA(VV, WW, false, 0);                       \
  } while (0)
  // flexible CG updates x every sweep; Jacobi-PCG every other one (xm 0 / 2)
  if (vec) {
    if (wx == 4) CGA_X(tile::vec_width<T>(), 4);
    else if (wx == 2) CGA_X(tile::vec_width<T>(), 2);
    else CGA_X(tile::vec_width<T>(), 1);
  } else {
    CGA_X(1, 1);
  }
#undef CGA_X
#undef CGA
  return nb;
}

// sweep B; returns the number of workgroup partials per component
template <class T>
int launch_cg_b(const Grid& g, T* r, const T* q, const T* dinv, T* z, double* partials,
                const SolveScalars* sc, bool flex, bool vec, hipStream_t s) {
  constexpr int VW = tile::vec_width<T>();
  const long long nv = vec ? g.n / VW : g.n;
  const int nb = vblocks(nv);
#define CGB(VV) k_cg_b<T, VV><<<nb, kBlock, 0, s>>>(nv, r, q, partials, sc)
#define CGBZ(VV) k_cg_bz<T, VV><<<nb, kBlock, 0, s>>>(nv, z, q, dinv, partials, sc)
  if (vec) {
    if (flex) CGB(VW);
    else CGBZ(VW);
  } else {
    if (flex) CGB(1);
    else CGBZ(1);
  }
#undef CGBZ
#undef CGB
  return nb;
}

template <class T>
void launch_cg_fixup(const Grid& g, T* x, const T* p, const T* p2, const SolveScalars* sc, hipStream_t s) {
  k_cg_fixup<T><<<vblocks(g.n), kBlock, 0, s>>>(g.n, x, p, p2, sc);
}
void launch_fold(const Grid& g, double* x, float* d, double inv_scale, hipStream_t s) {
  k_fold<<<vblocks(g.n), kBlock, 0, s>>>(g.n, x, d, inv_scale);
}
void launch_cast(const Grid& g, const double* r, float* r32, double scale, hipStream_t s) {
  k_cast<<<vblocks(g.n), kBlock, 0, s>>>(g.n, r, r32, scale);
}

template bool cg_vectorizable<double>(const Grid&, const void* const*, int);
template bool cg_vectorizable<float>(const Grid&, const void* const*, int);
template int launch_cg_a<double>(const Grid&, const Coeffs<double>&, const double*, const double*, const double*,
                                 double*, double*, const double*, double*, double*, const SolveScalars*, bool,
                                 int, bool, hipStream_t);
template int launch_cg_a<float>(const Grid&, const Coeffs<float>&, const float*, const float*, const float*,
                                float*, float*, const float*, float*, double*, const SolveScalars*, bool, int,
                                bool, hipStream_t);
template int launch_cg_b<double>(const Grid&, double*, const double*, const double*, double*, double*,
                                 const SolveScalars*, bool, bool, hipStream_t);
template int launch_cg_b<float>(const Grid&, float*, const float*, const float*, float*, double*,
                                const SolveScalars*, bool, bool, hipStream_t);
template void launch_cg_fixup<double>(const Grid&, double*, const double*, const double*, const SolveScalars*,
                                      hipStream_t);
template void launch_cg_fixup<float>(const Grid&, float*, const float*, const float*, const SolveScalars*,
                                     hipStream_t);

}  // namespace nfa
