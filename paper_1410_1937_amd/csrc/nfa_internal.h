// Internal declarations of libnfa (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nfa.h"

namespace nfa {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
nfa_status fail(nfa_status st, const std::string& msg);

#define NFA_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::nfa::fail(NFA_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define NFA_CHECK_LAUNCH() NFA_HIP(hipGetLastError())

inline hipStream_t S(nfa_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------- device buffers
// A device buffer of a handle: either a slice of a caller-owned workspace
// (borrowed) or memory the library allocated when the handle was created or
// its body set (owned); never allocated on the solve/apply path.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) { o.p = nullptr; o.bytes = 0; o.owned = false; }
  ~DevBuf() { release(); }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = false;
  }
  hipError_t alloc(size_t b) {
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) {
      bytes = b;
      owned = true;
    }
    return e;
  }
  void borrow(void* q, size_t b) {
    release();
    p = q;
    bytes = b;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Lays a handle's buffers out in one caller-owned workspace as 256-byte
// aligned slices, or allocates each (no workspace), or only adds up the bytes
// a workspace needs (measure).
struct Carver {
  unsigned char* base = nullptr;
  size_t cap = 0, used = 0;
  bool measure = false;
  hipError_t take(DevBuf& b, size_t bytes) {
    const size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    if (measure) return hipSuccess;
    if (!base) return b.alloc(bytes);
    if (used > cap) return hipErrorOutOfMemory;
    b.borrow(base + off, bytes);
    return hipSuccess;
  }
};

// ------------------------------------------------------------ launch
constexpr int kBlock = 256;
constexpr int kMaxPartials = 32768;    // block partials of one reduction (per component)
constexpr int kHistCap = 1 << 20;      // per-iteration residual history entries
inline int blocks_for(long long n, int per_block = kBlock, int cap = 65535 * 4) {
  long long b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<int>(b);
}

// ----------------------------------------------------------- grid data
struct Grid {
  int nx = 0, ny = 0, nz = 0;
  long long n = 0;          // cells
  int bc[6] = {0, 0, 0, 0, 0, 0};
  std::vector<double> xf, yf, zf;     // host face coordinates
  std::vector<double> dx, dy, dz;     // host widths
  std::vector<double> hx, hy, hz;     // host face distances (n+1 each)
  // device 1-D metrics
  DevBuf d_dx, d_dy, d_dz, d_hx, d_hy, d_hz;
  DevBuf d_gx, d_gy, d_gz;            // centre-to-centre spans of the normal stencil (n each)
  DevBuf d_xf, d_yf, d_zf;            // face coordinates (n+1 each)
  // body (always present: "no body" = all open)
  bool has_body = false;
  DevBuf frac_x, frac_y, frac_z;      // face fractions (double)
  DevBuf vfrac;                       // cell fraction (double)
  DevBuf open_x, open_y, open_z;      // open face areas a_f * Area_f (double)
  DevBuf active;                      // uint8 per cell
  DevBuf reduced;                     // uint8 per cell: 1 on the cell that carries an unknown
  DevBuf root;                        // int32 per cell: root cell (-1 inactive)
  // merge groups: roots, CSR offsets into members (slaves only, ascending)
  int n_groups = 0, n_slaves = 0;
  long long n_active = 0, n_reduced = 0;
  DevBuf g_root, g_off, g_mem;        // int32
  DevBuf s_cell, s_root;              // int32: slave list and its root
  // rows whose merged row differs from the cell-wise 7-point row (roots and
  // unknowns next to a slave), ascending; host copies of the slave list
  DevBuf fix_rows;                    // int32
  std::vector<int> h_fix, h_scell, h_sroot;
  int body_version = 0;               // incremented by every body set-up
  bool all_neumann() const { return !(bc[0] | bc[1] | bc[2] | bc[3] | bc[4] | bc[5]); }
  long long nfx() const { return (long long)nz * ny * (nx + 1); }
  long long nfy() const { return (long long)nz * (ny + 1) * nx; }
  long long nfz() const { return (long long)(nz + 1) * ny * nx; }
};

// Device-side scalars of an iterative solve (one cache line each group).
struct SolveScalars {
  double rz, pq, rr, bb, alpha, beta, tol2, pr, zq, rr_outer;
  double alpha_pend; // x += alpha_pend p_(k-1) still owed by the fused sweep
  double alpha_pend2; // x += alpha_pend2 p_(k-2) also owed (Jacobi-PCG: after a sweep A that skipped x)
  double rz_prev;    // r.z before the last update: the denominator of beta
  double ratio;      // stagnation threshold (mean reduction per iteration)
  int iter, done, breakdown, stalled, max_iter, window;
};

// Operator coefficients in one precision (lower-face layout, see stencil).
template <class T> struct Coeffs {
  T* tx = nullptr;    // nz*ny*nx   lower x-face of each cell
  T* txb = nullptr;   // nz*ny      +x boundary face
  T* ty = nullptr;    // nz*(ny+1)*nx natural y-face layout
  T* tz = nullptr;    // (nz+1)*ny*nx natural z-face layout
  T* dinv = nullptr;  // nz*ny*nx   Jacobi inverse diagonal of the merged operator
};

// Everything an operator owns: coefficients in both precisions and the
// work vectors of the FP64 and FP32 solvers.
struct Poisson {
  Grid* g = nullptr;
  bool assembled = false;
  int version = 0;                              // incremented by every assembly
  int body_version = -1;                        // the grid's body version at the last assembly
  DevBuf rho, rho_tmp;                          // double cells
  DevBuf tx64, txb64, ty64, tz64, dinv64;       // FP64 coefficients
  DevBuf tx32, txb32, ty32, tz32, dinv32;       // FP32 coefficients
  DevBuf r, z, p, p2, p3, q, tmp;               // double work vectors (p in three buffers)
  DevBuf x32, r32, z32, p32, p32b, p32c, q32;   // float work vectors
  DevBuf partials;                              // double block partials
  DevBuf scal;                                  // SolveScalars (device)
  DevBuf hist;                                  // double per-iteration ||r||^2 (kHistCap)
  SolveScalars* h_scal = nullptr;               // pinned host mirror (2 slots)
  hipEvent_t ev[2] = {nullptr, nullptr};
  // optional timing of selected launches inside solves (HIP events), by
  // kind: 0 / 1 the Jacobi-PCG sweep A that leaves x alone in FP64 / FP32,
  // 6 / 7 the one that applies the two owed x steps, 2 / 3 the multigrid
  // cycle's fused level-0 down / up sweep (FP32), 4 the flexible FP32 sweep A,
  // 5 one whole application of the learned preconditioner
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;              // 2 per recorded launch
  std::vector<int> prof_kind;                   // kind per recorded launch
  std::vector<int> prof_seq;                    // iteration (since the last harvest) per recorded launch
  int prof_used = 0;
  int prof_iter = 0;                            // iterations enqueued since the last harvest
  long long prof_launches[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double prof_ms[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  Coeffs<double> c64() const {
    return {tx64.as<double>(), txb64.as<double>(), ty64.as<double>(), tz64.as<double>(), dinv64.as<double>()};
  }
  Coeffs<float> c32() const {
    return {tx32.as<float>(), txb32.as<float>(), ty32.as<float>(), tz32.as<float>(), dinv32.as<float>()};
  }
};

constexpr int kProfMgDown = 2, kProfMgUp = 3, kProfF32Flex = 4, kProfUnet = 5, kProfF64X2 = 6, kProfF32X2 = 7,
              kProfKinds = 8;

// The operator holds coefficients of its grid's current body: assembled, and
// no nfa_grid_set_body since (a new body changes the apertures, the active
// set and the merge groups that the coefficients and D^-1 were formed from).
inline nfa_status require_assembled(const Poisson& op, const char* who) {
  if (!op.assembled) return fail(NFA_ERR_INVALID, std::string(who) + ": operator not assembled");
  if (op.body_version != op.g->body_version)
    return fail(NFA_ERR_INVALID, std::string(who) + ": the grid's body was set after the last assembly; assemble again");
  return NFA_OK;
}

// Open / close the timing of one launch on st when profiling is on.
inline bool prof_begin(Poisson& op, hipStream_t st) {
  const bool rec = op.prof_on && op.prof_used * 2 + 1 < (int)op.prof_ev.size();
  if (rec) (void)hipEventRecord(op.prof_ev[2 * op.prof_used], st);
  return rec;
}
inline void prof_end(Poisson& op, bool rec, int kind, hipStream_t st) {
  if (!rec) return;
  (void)hipEventRecord(op.prof_ev[2 * op.prof_used + 1], st);
  op.prof_kind[op.prof_used] = kind;
  op.prof_seq[op.prof_used] = op.prof_iter;
  ++op.prof_used;
}

// ---------------------------------------------------------------- kernels
// Stencil sweep (stencil.hip): q = A p, or q = b - A p when b is given
// (FP64 only: a FP32 sweep ignores b).
template <class T>
void launch_stencil(const Grid& g, const Coeffs<T>& c, const T* p, const double* b, T* q, hipStream_t s);

// Merge kernels (stencil.hip): slaves copy their root (primal vectors);
// roots add their slaves, slaves -> 0 (dual vectors).
template <class T> void launch_merge_copy(const Grid& g, T* v, hipStream_t s, const SolveScalars* sc);
template <class T> void launch_merge_gather(const Grid& g, T* v, hipStream_t s, const SolveScalars* sc);

// The learned preconditioner inside flexible CG (unet.hip): z = M(r) on FP32
// cell arrays, exits at once when the solver state says done.
nfa_status unet_precond_apply(void* unet, Poisson& op, const float* r, float* z,
                              const SolveScalars* sc, hipStream_t s);

// Fixed-order sum of `n` partials of `ncomp` components (stride kMaxPartials)
// into out[0..ncomp) (solver.hip).
void launch_sum_partials(const double* partials, int n, int ncomp, double* out, hipStream_t s);

}  // namespace nfa

struct nfa_grid_s : nfa::Grid {};

namespace nfa {
// Multigrid preconditioner (multigrid.hip): one V-cycle z = M r in FP32, and
// a (re)build of the hierarchy when the operator has been reassembled.  With
// q and partials given, the cycle also writes the block partial sums of
// z.q (z before the slaves copy their roots) and returns their count in *np
// (0: not summed, the caller sums them).
nfa_status mg_precond_apply(void* mg, Poisson& op, const float* r, float* z, const float* q, double* partials,
                            int* np, const SolveScalars* sc, hipStream_t s);
nfa_status mg_ensure(void* mg, Poisson& op, hipStream_t s);
}  // namespace nfa
struct nfa_poisson_s : nfa::Poisson {};
