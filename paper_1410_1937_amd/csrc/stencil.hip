// libnfa: the flux-form 7-point operator sweep and the merge kernels.
//
// (A p)_c = sum_f T_f (p_c - p_nb(f)) over the faces x-, x+, y-, y+, z-, z+
// in that order (eq. integral2, left side; eq. pois), p_nb = 0 beyond the
// domain (a Neumann face has T = 0).  Built with -ffp-contract=off so the
// FP64 sweep is bitwise the sum written above.
//
// Layout: cells (nz, ny, nx) x fastest.  tx holds the lower x-face of every
// cell plus a (nz, ny) plane for the +x boundary; ty and tz use the natural
// face layouts (nz, ny+1, nx) and (nz+1, ny, nx).
//
// Launch shape: the tile of the CG sweep A (16 wavefronts, WX across x by
// 16 / WX rows in y, V cells per lane in one 16-byte vector) marching up a
// contiguous range of z-planes on a persistent grid.  Per plane the tile's p
// and lower y-face coefficients are exchanged through LDS (one barrier per
// plane, double-buffered); x-neighbours inside a wavefront come from
// shuffles, and only the tile's outer rows and columns read neighbours
// through the caches.  p(k-1), p(k) and the z-face coefficient T_z(k) stay in
// registers, so every plane of p and of the coefficients is fetched once.
#include "device_util.h"
#include "nfa_internal.h"
#include "sweep_tile.h"

namespace nfa {
namespace {

using namespace tile;

// q = A p (b == nullptr) or q = b - A p (RES, FP64 only: b and q double).
// Non-temporal loads: the FP32 streams and the right-hand side b (measured
// on the 512 x 256 x 192 grid: the residual 230.7 -> 226.6 us with b alone,
// 238.6 us with every FP64 stream).
template <class T, int V, int WX, bool RES>
__global__ __launch_bounds__(AX* kTileWaves) void k_stencil(
    int nx, int ny, int nz, int tiles_x, long long ncol, long long per_block,
    const T* __restrict__ p, const T* __restrict__ tx, const T* __restrict__ txb,
    const T* __restrict__ ty, const T* __restrict__ tz, const double* __restrict__ b,
    T* __restrict__ q) {
  constexpr int AY = kTileWaves / WX;
  constexpr int TW = WX * AX;  // vectors per tile row
  constexpr bool NT_LOAD = sizeof(T) == 4;
  __shared__ Pack<T, V> shp[2][AY][TW];  // p of the current plane
  __shared__ Pack<T, V> sht[2][AY][TW];  // lower y-face coefficient of the current plane
  const int lane = threadIdx.x;
  const int wx = threadIdx.y % WX, row = threadIdx.y / WX;
  const int col = wx * AX + lane;
  const long long plane = (long long)nx * ny;
  const long long yplane = (long long)(ny + 1) * nx;
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
    Pack<T, V> pm = zero<T, V>(), pc = zero<T, V>(), tzc = zero<T, V>();
    if (live) {
      if (k0 > 0) pm = ld<T, V>(p + c - plane);
      pc = ld<T, V>(p + c);
      tzc = ld<T, V>(tz + c);
    }
    for (int k = k0; k < k1; ++k, c += plane, yi += yplane) {
      Pack<T, V> pp = zero<T, V>(), tzp = zero<T, V>(), txv = zero<T, V>();
      Pack<T, V> tym = zero<T, V>(), typ = zero<T, V>(), pym = zero<T, V>(), pyp = zero<T, V>();
      Pack<double, V> bv;
      T left = T(0), right = T(0), txr = T(0);
      if (live) {
        if (k + 1 < nz) pp = ld_stream<NT_LOAD, T, V>(p + c + plane);
        tzp = ld_stream<NT_LOAD, T, V>(tz + c + plane);
        txv = ld_stream<NT_LOAD, T, V>(tx + c);
        tym = ld_stream<NT_LOAD, T, V>(ty + yi);
        if (!yin_hi) typ = ld<T, V>(ty + yi + nx);
        if (ylo && row == 0) pym = ld<T, V>(p + c - nx);
        if (yhi && row == AY - 1) pyp = ld<T, V>(p + c + nx);
        if (lglob) left = p[c - 1];
        if (rglob) right = p[c + V];
        if (redge) txr = tx[c + V];
        else if (rbdy) txr = txb[(long long)k * ny + j];
        if constexpr (RES) bv = ld_stream<true, double, V>(b + c);
      }
      const int bb = k & 1;
      shp[bb][row][col] = pc;
      sht[bb][row][col] = tym;
      __syncthreads();
      if (live) {
        if (yin_lo) pym = shp[bb][row - 1][col];
        if (yin_hi) {
          pyp = shp[bb][row + 1][col];
          typ = sht[bb][row + 1][col];
        }
        if (ledge && wx > 0) left = shp[bb][row][col - 1].v[V - 1];
        if (redge && wx < WX - 1) right = shp[bb][row][col + 1].v[0];
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
          if constexpr (RES) qv.v[e] = (T)(bv.v[e] - (double)s);
          else qv.v[e] = s;
        }
        st_stream<true, T, V>(q + c, qv);
      }
      pm = pc;
      pc = pp;
      tzc = tzp;
    }
  }
}

template <class T>
__global__ void k_merge_copy(int ns, const int* __restrict__ s_cell, const int* __restrict__ s_root,
                             T* v, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ns; t += gridDim.x * blockDim.x)
    v[s_cell[t]] = v[s_root[t]];
}

// root value + slaves (ascending), slaves -> 0
template <class T>
__global__ void k_merge_gather(int ng, const int* __restrict__ g_root, const int* __restrict__ g_off,
                               const int* __restrict__ g_mem, T* v, const SolveScalars* sc) {
  if (solve_done(sc)) return;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ng; t += gridDim.x * blockDim.x) {
    const int r = g_root[t];
    T acc = v[r];
    for (int m = g_off[t]; m < g_off[t + 1]; ++m) {
      const int cm = g_mem[m];
      acc = acc + v[cm];
      v[cm] = T(0);
    }
    v[r] = acc;
  }
}

}  // namespace

template <class T>
void launch_stencil(const Grid& g, const Coeffs<T>& c, const T* p, const double* b, T* q, hipStream_t s) {
  using namespace tile;
  constexpr int VW = vec_width<T>();
  const auto al = [](const void* a) { return reinterpret_cast<uintptr_t>(a) % 16 == 0; };
  const bool vec = g.nx % VW == 0 && al(p) && al(q) && al(c.tx) && al(c.ty) && al(c.tz) && (!b || al(b));
  const int V = vec ? VW : 1;
  const int wx = tile_wx<T>(g, V);
  const int ay = kTileWaves / wx;
  const int tiles_x = (g.nx + AX * wx * V - 1) / (AX * wx * V);
  const long long ncol = (long long)tiles_x * ((g.ny + ay - 1) / ay);
  const dim3 blk(AX, kTileWaves);
#define STL(VV, WW, RR)                                                                           \
  do {                                                                                            \
    const void* fn = reinterpret_cast<const void*>(&k_stencil<T, VV, WW, RR>);                   \
    const int nb = resident_blocks(fn, AX * kTileWaves);                                          \
    const long long per = (ncol * g.nz + nb - 1) / nb;                                            \
    k_stencil<T, VV, WW, RR><<<nb, blk, 0, s>>>(g.nx, g.ny, g.nz, tiles_x, ncol, per, p, c.tx,    \
                                                c.txb, c.ty, c.tz, b, q);                         \
  } while (0)
#define STL_R(VV, WW)                 \
  do {                                \
    if constexpr (sizeof(T) == 8) {   \
      if (b) {                        \
        STL(VV, WW, true);            \
        break;                        \
      }                               \
    }                                 \
    STL(VV, WW, false);               \
  } while (0)
  if (!vec) STL_R(1, 1);
  else if (wx == 4) STL_R(VW, 4);
  else if (wx == 2) STL_R(VW, 2);
  else STL_R(VW, 1);
#undef STL_R
#undef STL
}

template <class T> void launch_merge_copy(const Grid& g, T* v, hipStream_t s, const SolveScalars* sc) {
  if (g.n_slaves == 0) return;
  k_merge_copy<T><<<blocks_for(g.n_slaves), kBlock, 0, s>>>(g.n_slaves, g.s_cell.as<int>(),
                                                            g.s_root.as<int>(), v, sc);
}

template <class T> void launch_merge_gather(const Grid& g, T* v, hipStream_t s, const SolveScalars* sc) {
  if (g.n_groups == 0) return;
  k_merge_gather<T><<<blocks_for(g.n_groups), kBlock, 0, s>>>(g.n_groups, g.g_root.as<int>(),
                                                              g.g_off.as<int>(), g.g_mem.as<int>(), v, sc);
}

template void launch_stencil<double>(const Grid&, const Coeffs<double>&, const double*, const double*,
                                     double*, hipStream_t);
template void launch_stencil<float>(const Grid&, const Coeffs<float>&, const float*, const double*,
                                    float*, hipStream_t);
template void launch_merge_copy<double>(const Grid&, double*, hipStream_t, const SolveScalars*);
template void launch_merge_copy<float>(const Grid&, float*, hipStream_t, const SolveScalars*);
template void launch_merge_gather<double>(const Grid&, double*, hipStream_t, const SolveScalars*);
template void launch_merge_gather<float>(const Grid&, float*, hipStream_t, const SolveScalars*);

}  // namespace nfa
