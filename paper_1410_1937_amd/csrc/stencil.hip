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
// Launch shape: a workgroup is a 64 x 4 tile of (i, j) columns that marches
// up a chunk of z-planes, carrying p(k-1), p(k) and T_z(k) in registers so
// that each plane of p and of the coefficients is fetched once; x- and
// y-neighbours of the plane being swept are re-read through the vector L1 /
// L2 (the 64-wide row of a wavefront is one coalesced 512 B (FP64) line
// set).  Workgroup ids are remapped so that consecutive tiles run on the same
// XCD and share its L2 for the y halos.
#include "device_util.h"
#include "nfa_internal.h"

namespace nfa {
namespace {

constexpr int TX = 64, TY = 4;

template <class T, bool DOT>
__global__ __launch_bounds__(TX* TY) void k_stencil(int nx, int ny, int nz, int kchunk, int tiles_x,
                                                    int tiles_y, const T* __restrict__ p,
                                                    const T* __restrict__ tx,
                                                    const T* __restrict__ txb,
                                                    const T* __restrict__ ty,
                                                    const T* __restrict__ tz,
                                                    const double* __restrict__ b,
                                                    T* __restrict__ q,
                                                    double* __restrict__ partials,
                                                    const SolveScalars* __restrict__ sc) {
  if (solve_done(sc)) return;
  __shared__ double lds[TX * TY / 64];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = blk % tiles_x;
  const int rest = blk / tiles_x;
  const int by = rest % tiles_y;
  const int bz = rest / tiles_y;
  const int i = bx * TX + threadIdx.x;
  const int j = by * TY + threadIdx.y;
  const int k0 = bz * kchunk;
  const int k1 = min(nz, k0 + kchunk);
  double acc = 0.0;
  if (i < nx && j < ny && k0 < nz) {
    const long long plane = (long long)nx * ny;
    long long c = (long long)k0 * plane + (long long)j * nx + i;
    long long yi = ((long long)k0 * (ny + 1) + j) * nx + i;
    const long long yplane = (long long)(ny + 1) * nx;
    T pzm = k0 > 0 ? p[c - plane] : T(0);
    T pc = p[c];
    T tzm = tz[c];
    const bool xlo = i > 0, xhi = i < nx - 1, ylo = j > 0, yhi = j < ny - 1;
    for (int k = k0; k < k1; ++k, c += plane, yi += yplane) {
      const T pzp = (k + 1 < nz) ? p[c + plane] : T(0);
      const T tzp = tz[c + plane];
      const T pxm = xlo ? p[c - 1] : T(0);
      const T pxp = xhi ? p[c + 1] : T(0);
      const T pym = ylo ? p[c - nx] : T(0);
      const T pyp = yhi ? p[c + nx] : T(0);
      const T txm = tx[c];
      const T txp = xhi ? tx[c + 1] : txb[(long long)k * ny + j];
      const T tym = ty[yi];
      const T typ = ty[yi + nx];
      T s = txm * (pc - pxm);
      s = s + txp * (pc - pxp);
      s = s + tym * (pc - pym);
      s = s + typ * (pc - pyp);
      s = s + tzm * (pc - pzm);
      s = s + tzp * (pc - pzp);
      if (b) {
        q[c] = (T)(b[c] - (double)s);
      } else {
        q[c] = s;
        if (DOT) acc += (double)pc * (double)s;
      }
      pzm = pc;
      pc = pzp;
      tzm = tzp;
    }
  }
  if (DOT) {
    const double t = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[blockIdx.x] = t;
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
int launch_stencil(const Grid& g, const Coeffs<T>& c, const T* p, const double* b, T* q,
                   double* partials, const SolveScalars* sc, int mode, hipStream_t s) {
  const int tiles_x = (g.nx + TX - 1) / TX;
  const int tiles_y = (g.ny + TY - 1) / TY;
  int kchunk = 16;
  long long nb;
  for (;;) {
    const long long tz = (g.nz + kchunk - 1) / kchunk;
    nb = (long long)tiles_x * tiles_y * tz;
    if (nb <= kMaxPartials || kchunk >= g.nz) break;
    kchunk *= 2;
  }
  dim3 blk(TX, TY);
  const bool dot = partials != nullptr && mode == ST_APPLY;
  if (dot && nb > kMaxPartials) return -1;   // excluded when the operator is created
  const double* bb = mode == ST_RESIDUAL ? b : nullptr;
  if (dot)
    k_stencil<T, true><<<(int)nb, blk, 0, s>>>(g.nx, g.ny, g.nz, kchunk, tiles_x, tiles_y, p, c.tx,
                                               c.txb, c.ty, c.tz, nullptr, q, partials, sc);
  else
    k_stencil<T, false><<<(int)nb, blk, 0, s>>>(g.nx, g.ny, g.nz, kchunk, tiles_x, tiles_y, p, c.tx,
                                                c.txb, c.ty, c.tz, bb, q, nullptr, sc);
  return dot ? (int)nb : 0;
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

template int launch_stencil<double>(const Grid&, const Coeffs<double>&, const double*, const double*,
                                    double*, double*, const SolveScalars*, int, hipStream_t);
template int launch_stencil<float>(const Grid&, const Coeffs<float>&, const float*, const double*,
                                   float*, double*, const SolveScalars*, int, hipStream_t);
template void launch_merge_copy<double>(const Grid&, double*, hipStream_t, const SolveScalars*);
template void launch_merge_copy<float>(const Grid&, float*, hipStream_t, const SolveScalars*);
template void launch_merge_gather<double>(const Grid&, double*, hipStream_t, const SolveScalars*);
template void launch_merge_gather<float>(const Grid&, float*, hipStream_t, const SolveScalars*);

}  // namespace nfa
