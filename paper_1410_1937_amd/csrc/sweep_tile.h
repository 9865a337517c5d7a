// Pieces shared by the tiled 7-point sweeps (cg.hip: the CG sweep A;
// stencil.hip: q = A p and r = b - A x): 16-byte vectors of V cells per
// lane, streaming loads and stores with the non-temporal hint, the tile
// shape and the persistent-grid size.
//
// Tile: a workgroup of kTileWaves wavefronts holds WX wavefronts across x by
// kTileWaves / WX rows in y; each lane owns V consecutive x cells.  The tile
// marches up a contiguous range of z-planes and exchanges the current plane
// through LDS, so the only neighbour values read through the caches are the
// tile's outer rows and columns.
#pragma once

#include <hip/hip_runtime.h>

#include "nfa_internal.h"

namespace nfa {
namespace tile {

constexpr int AX = 64;          // lanes of a wavefront along x
constexpr int kTileWaves = 16;  // wavefronts per workgroup

template <class T, int V> struct alignas(sizeof(T) * V) Pack {
  T v[V];
};

template <class T, int V> __device__ __forceinline__ Pack<T, V> ld(const T* p) {
  return *reinterpret_cast<const Pack<T, V>*>(p);
}
template <class T, int V> __device__ __forceinline__ void st(T* p, const Pack<T, V>& a) {
  *reinterpret_cast<Pack<T, V>*>(p) = a;
}
// Streaming accesses (each element touched once per sweep) may carry the
// non-temporal hint; neighbour and halo reads always use ordinary loads.
template <bool NT, class T, int V> __device__ __forceinline__ Pack<T, V> ld_stream(const T* p) {
  Pack<T, V> r;
  if constexpr (!NT) {
    r = ld<T, V>(p);
  } else if constexpr (V == 1) {
    r.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T vt __attribute__((ext_vector_type(V)));
    const vt a = __builtin_nontemporal_load(reinterpret_cast<const vt*>(p));
#pragma unroll
    for (int e = 0; e < V; ++e) r.v[e] = a[e];
  }
  return r;
}
template <bool NT, class T, int V> __device__ __forceinline__ void st_stream(T* p, const Pack<T, V>& a) {
  if constexpr (!NT) {
    st<T, V>(p, a);
  } else if constexpr (V == 1) {
    __builtin_nontemporal_store(a.v[0], p);
  } else {
    typedef T vt __attribute__((ext_vector_type(V)));
    vt b;
#pragma unroll
    for (int e = 0; e < V; ++e) b[e] = a.v[e];
    __builtin_nontemporal_store(b, reinterpret_cast<vt*>(p));
  }
}
template <class T, int V> __device__ __forceinline__ Pack<T, V> zero() {
  Pack<T, V> a;
#pragma unroll
  for (int e = 0; e < V; ++e) a.v[e] = T(0);
  return a;
}

template <class T> constexpr int vec_width() { return 16 / (int)sizeof(T); }

// Tile width in wavefronts: the widest of 4, 2, 1 whose tile width divides
// nx (FP64, where a row of 2-double vectors spans several wavefronts); FP32
// uses one wavefront across and 16 rows.
template <class T> inline int tile_wx(const Grid& g, int V) {
  if (sizeof(T) != 8 || V == 1) return 1;
  for (int wx : {4, 2}) {
    if (g.nx % (wx * AX * V) == 0) return wx;
  }
  return 1;
}

}  // namespace tile

// resident workgroups of a kernel on the whole device (cached per kernel),
// capped at kMaxPartials
int resident_blocks(const void* fn, int threads);

}  // namespace nfa
