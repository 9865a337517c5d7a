// libnfa: learned preconditioner (3-D U-Net) for flexible CG.
//
// Forward convolutions are implicit GEMMs on the BF16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), tiled for LDS: a workgroup of
// four wavefronts computes a brick of 16 x 4 x 4 output positions from the
// brick's input halo (18 x 6 x 6 positions) staged once in LDS, channels in
// groups of at most 32, so every one of the 27 taps reads its B fragments
// (8 consecutive channels of one position per lane, one 16-byte LDS read)
// from LDS.  A wavefront owns a 2 x 2 (y, z) block of 16-position x-rows and
// all output channels: each A (weight) fragment, read through the L1 from a
// packed per-lane layout, feeds four MFMAs.  The epilogues fuse what the
// network does next to each convolution: bias, ReLU and the BF16 storage
// rounding; the 2 x 2 x 2 average pool (the wavefront's 2 x 2 rows are summed
// in registers, x pairs by a lane shuffle); and the 1 x 1 x 1 head projected
// onto the outputs of the first encoder and of the last decoder convolution.
// The first convolution forms its input features from r and log(1/rho) while
// staging them.  At inference nothing of full resolution is stored but the
// head's partial sum: the 16-channel activation a0 stays in registers.
//
// Training keeps every activation; the data gradient runs the earlier
// direct-gather MFMA kernel on the flipped, transposed weights and the weight
// gradient is an MFMA GEMM over positions with per-workgroup partials summed
// in a fixed order.  Activations are stored as BF16 (round to nearest even),
// exactly where the CPU oracle rounds.
#include <cmath>
#include <cstring>
#include <random>
#include <type_traits>
#include <vector>

#include "../../include/nfa_unet.h"
#include "device_util.h"
#include "nfa_internal.h"
#include "sweep_tile.h"
#include "vecops.h"

namespace nfa {
namespace {

typedef unsigned short bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double kL0 = -3.5, kL1 = 3.4;   // log(1/rho) normalisation

// f(std::integral_constant<int, I>) for I = B .. E-1, in order
template <int B, int E, class F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
constexpr int kMaxLevels = 6;
constexpr int kWgradBlocks = 64;

__device__ __forceinline__ bf16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }

union Frag {
  uint4 u;
  bf16x8 v;
  bf16_t h[8];
};

__device__ __forceinline__ void tap_offset(int t, int& dz, int& dy, int& dx) {
  dz = t / 9 - 1;
  dy = (t / 3) % 3 - 1;
  dx = t % 3 - 1;
}

#define GRID_STRIDE(idx, n) \
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (n); idx += (long long)gridDim.x * blockDim.x)

// ------------------------------------------------------------ features
__global__ void k_ell(long long n, const double* __restrict__ rho, bf16_t* __restrict__ ell) {
  GRID_STRIDE(c, n) ell[c] = f2bf((float)((log(1.0 / rho[c]) - kL0) / kL1));
}

// ------------------------------------------------------------ conv (MFMA)
// out[p][co] = act(bias[co] + sum_{t,ci} in'[p + off_t][ci] W[t][ci][co]) (* mask>0)
// in' = in, or bf16(in + up(in2)) when UPADD (in2 at half resolution).
template <int CIN, int COUT, bool UPADD>
__global__ __launch_bounds__(256) void k_conv(int D, int H, int W, const bf16_t* __restrict__ in,
                                              const bf16_t* __restrict__ in2,
                                              const uint4* __restrict__ frag,
                                              const float* __restrict__ bias, int relu,
                                              const bf16_t* __restrict__ mask,
                                              bf16_t* __restrict__ out,
                                              const SolveScalars* __restrict__ sc) {
  if (solve_done(sc)) return;
  constexpr int K = 27 * CIN;
  constexpr int KS = (K + 31) / 32;
  constexpr int MT = COUT / 16;
  const int lane = threadIdx.x & 63;
  const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int segs = (W + 15) / 16;
  if (wave >= (long long)D * H * segs) return;   // uniform per wavefront
  const int seg = (int)(wave % segs);
  const long long rest = wave / segs;
  const int y = (int)(rest % H), z = (int)(rest / H);
  const int n = lane & 15, kq = lane >> 4;
  const int x = seg * 16 + n;
  const bool xok = x < W;
  const int H2 = H >> 1, W2 = W >> 1;
  f32x4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < KS; ++ks) {
    Frag b;
    b.u = make_uint4(0u, 0u, 0u, 0u);
    const int kb = ks * 32 + kq * 8;
    if constexpr (CIN >= 8) {
      const int t = kb / CIN, ci0 = kb % CIN;
      if (t < 27 && xok) {
        int dz, dy, dx;
        tap_offset(t, dz, dy, dx);
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        if (zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W) {
          const long long p = ((long long)zz * H + yy) * W + xx;
          b.u = *reinterpret_cast<const uint4*>(in + p * CIN + ci0);
          if constexpr (UPADD) {
            const long long q = ((long long)(zz >> 1) * H2 + (yy >> 1)) * W2 + (xx >> 1);
            Frag c;
            c.u = *reinterpret_cast<const uint4*>(in2 + q * CIN + ci0);
#pragma unroll
            for (int j = 0; j < 8; ++j) b.h[j] = f2bf(bf2f(b.h[j]) + bf2f(c.h[j]));
          }
        }
      }
    } else {
      static_assert(CIN == 2, "input channels: 2 or a multiple of 8");
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int t = kb / 2 + qq;
        if (t < 27 && xok) {
          int dz, dy, dx;
          tap_offset(t, dz, dy, dx);
          const int zz = z + dz, yy = y + dy, xx = x + dx;
          if (zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W) {
            const long long p = ((long long)zz * H + yy) * W + xx;
            const unsigned v = *reinterpret_cast<const unsigned*>(in + p * 2);
            b.h[2 * qq] = (bf16_t)(v & 0xFFFFu);
            b.h[2 * qq + 1] = (bf16_t)(v >> 16);
          }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      Frag a;
      a.u = frag[((long long)ks * MT + m) * 64 + lane];
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[m], 0, 0, 0);
    }
  }
  if (!xok) return;
  const long long p = ((long long)z * H + y) * W + x;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    bf16_t h[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ch = m * 16 + kq * 4 + i;
      float v = acc[m][i];
      if (bias) v += bias[ch];
      if (relu) v = fmaxf(v, 0.f);
      if (mask && !(bf2f(mask[p * COUT + ch]) > 0.f)) v = 0.f;
      h[i] = f2bf(v);
    }
    uint2 w;
    w.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
    w.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
    *reinterpret_cast<uint2*>(out + p * COUT + m * 16 + kq * 4) = w;
  }
}

// ------------------------------------------------------------ tiled conv (MFMA)
// out[p][co] = bf16(relu(bias[co] + sum_{t,ci} in'[p + off_t][ci] W[t][ci][co]))
// on bricks of kTX x kTY x kTZ positions; in' = in, bf16(in + up(in2)) when
// UPADD, or the features [bf16(r/s), ell] when FEAT (then CIN = 2).
// A workgroup's brick is kTX x 4 SUB x 4 SUB positions; each wavefront takes
// SUB x SUB blocks of 2 x 2 (y, z) rows one after the other from one staged halo.
constexpr int kTX = 16, kHX = kTX + 2;
template <int SUB> struct Brick {
  static constexpr int TY = 4 * SUB, TZ = 4 * SUB, HY = TY + 2, HZ = TZ + 2, HALO = kHX * HY * HZ;
};

struct TconvArgs {
  int D, H, W;             // grid of the convolution's level
  int nbx, nby, nb, per;   // bricks along x and y, in all, per XCD range
  const bf16_t* in;        // [n][CIN] (not FEAT)
  const bf16_t* in2;       // UPADD: [n/8][CIN], the coarser level
  const float* r;          // FEAT, head: residual, float cells
  const bf16_t* ell;       // FEAT: normalised log(1/rho)
  const double* rr;        // FEAT, head: ||r||^2 over the unknowns
  double nred;             // FEAT, head: number of unknowns
  bf16_t* x0;              // FEAT: features out [n][2], or null
  const uint4* frag;       // A fragments (k_pack_tile)
  const float* bias;       // [COUT]
  bf16_t* out;             // [n][COUT], or null
  bf16_t* pooled;          // [n/8][COUT] (2 x 2 x 2 average), or null
  float* z;                // head on this layer's output (16 channels): z = dinv (x0[.,0] + (b + w . out)), or null
  const float* wproj;      // [COUT] head weights (BF16 values)
  const float* pbias;      // head bias b
  const float* dinv;       // head: FP32 D^-1 of the operator
  const SolveScalars* sc;
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// two floats rounded to BF16 (nearest even; v_cvt_pk_bf16_f32), packed low/high
__device__ __forceinline__ unsigned pack_bf2(float lo, float hi) {
  bf16x2 v;
  v.x = (__bf16)lo;
  v.y = (__bf16)hi;
  return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ float lo_bf(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_bf(unsigned w) { return __uint_as_float(w & 0xFFFF0000u); }
// bf16(a + b) for the two BF16 values packed in each of a and b
__device__ __forceinline__ unsigned add_bf2(unsigned a, unsigned b) {
  return pack_bf2(lo_bf(a) + lo_bf(b), hi_bf(a) + hi_bf(b));
}

// offset in staged positions of tap t from the centre (rows of kHX, planes of HY rows)
template <int HY> __host__ __device__ constexpr int tap_halo(int t) {
  return ((t / 9 - 1) * HY + ((t / 3) % 3 - 1)) * kHX + (t % 3 - 1);
}

// Staged position stride in bytes.  Measured on gfx950 for 16-byte reads of
// sixteen consecutive positions (one fragment row): strides of 32 or 96
// bytes run without bank conflicts at 170-200 B/clk per CU, 48, 64 and 80
// bytes conflict (115-120 B/clk).  16 channels are stored unpadded (32
// bytes); 32 channels keep 80 bytes, since 96 would cost the 32 -> 16
// decoder a resident workgroup per CU (LDS) and that was measured slower.
template <int CG> constexpr int lds_stride() { return CG == 2 ? 4 : CG == 16 ? 32 : CG * 2 + 16; }

template <int CIN, int COUT, bool UPADD, bool FEAT, int SUB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_tconv(const TconvArgs a) {
  if (solve_done(a.sc)) return;
  constexpr int kTY = Brick<SUB>::TY, kTZ = Brick<SUB>::TZ, kHY = Brick<SUB>::HY, kHZ = Brick<SUB>::HZ;
  constexpr int kHalo = Brick<SUB>::HALO, HY = kHY;
  static_assert(!FEAT || CIN == 2, "features have two channels");
  static_assert(FEAT || CIN % 16 == 0, "input channels: 2 (features) or a multiple of 16");
  constexpr int CG = CIN < 32 ? CIN : 32;          // channels per staged group
  constexpr int NG = CIN / CG;
  constexpr int KC = (27 * CIN + 31) / 32;         // K chunks of 32
  constexpr int KCG = NG > 1 ? 27 : KC;            // chunks per group
  constexpr int MT = COUT / 16;
  constexpr int ST = lds_stride<CG>();
  static_assert(SUB == 1 || NG == 1, "several blocks per wavefront need a single staged group");
  // staged rows: kHX positions, or for the features the kFX loaded ones
  // (position x0b - 1 + hx at kFO + hx)
  constexpr int kFX = 24, kFO = 3, RS = FEAT ? kFX : kHX, XO = FEAT ? kFO : 0;
  __shared__ __align__(16) unsigned char lds[FEAT ? kHY * kHZ * kFX * 4 : kHalo * ST];
  // the first encoder's A fragments (2 KB) sit in LDS: its wavefronts take
  // four blocks per brick, each reloading them
  __shared__ __align__(16) uint4 afr[FEAT ? KC * MT * 64 : 1];
  // bricks in contiguous ranges per XCD (workgroups are dealt to the XCDs
  // round robin), so that neighbouring bricks share an L2
  const int b = (int)(blockIdx.x & 7) * a.per + (int)(blockIdx.x >> 3);
  if (b >= a.nb) return;
  const int bx = b % a.nbx, brest = b / a.nbx;
  const int x0b = bx * kTX, y0b = (brest % a.nby) * kTY, z0b = (brest / a.nby) * kTZ;
  const int D = a.D, H = a.H, W = a.W;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 15, kq = lane >> 4;

  // loads that depend on nothing staged, issued first: this lane's biases and
  // head weights, the residual scale, the first chunk's A fragments
  float bi[MT][4], wp[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bi[m][i] = a.bias[m * 16 + 4 * kq + i];
      wp[m][i] = a.z ? a.wproj[m * 16 + 4 * kq + i] : 0.f;
    }
  const float pb = a.z ? a.pbias[0] : 0.f;
  const double rr = (FEAT || a.z) ? *a.rr : 0.0;
  const uint4* fr = a.frag + lane;
  Frag An[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) An[m].u = fr[m * 64];
  if constexpr (FEAT) {
    for (int e = threadIdx.x; e < KC * MT * 64; e += 256) afr[e] = a.frag[e];
  }
  auto load_a = [&](int idx) -> uint4 {
    if constexpr (FEAT) return afr[idx * 64 + lane];
    else return fr[idx * 64];
  };


  // ---- staging of channel group g's halo
  auto stage = [&](auto gg) {
    constexpr int g = decltype(gg)::value;
    // ---- stage the halo of channel group g
    if constexpr (FEAT) {
      // one thread per (halo row, 4 aligned x positions): a row holds the
      // kFX = 24 positions x0b - 4 .. x0b + 19 as loaded (6 quads; W is a
      // multiple of 4, so a quad is wholly inside the grid or wholly outside,
      // and outside it is zero), each quad one 16-byte LDS write; the taps
      // read x0b - 1 .. x0b + 16 of it.  Element indices fit in 32 bits.
      const double ms = rr / a.nred;
      const double inv = ms > 0 ? 1.0 / sqrt(ms) : 1.0;
      constexpr int NQ = kHY * kHZ * 6;             // (row, quad) pairs
      constexpr int NIT = (NQ + 255) / 256;
      float4 rv[NIT];
      uint2 ev[NIT];
      unsigned p0[NIT];
      bool ok[NIT];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int tq = tid + it * 256;
        const int quad = tq % 6, row = tq / 6;
        const int hy = row % kHY, hz = row / kHY;
        const int gy = y0b - 1 + hy, gz = z0b - 1 + hz, gx0 = x0b - 4 + 4 * quad;
        ok[it] = ((it + 1) * 256 <= NQ || tq < NQ) && gx0 >= 0 && gx0 < W && (unsigned)gy < (unsigned)H &&
                 (unsigned)gz < (unsigned)D;
        p0[it] = ok[it] ? (unsigned)(gz * H + gy) * (unsigned)W + (unsigned)gx0 : 0u;
        rv[it] = make_float4(0.f, 0.f, 0.f, 0.f);
        ev[it] = make_uint2(0u, 0u);
        if (ok[it]) {
          rv[it] = *reinterpret_cast<const float4*>(a.r + p0[it]);
          ev[it] = *reinterpret_cast<const uint2*>(a.ell + p0[it]);
        }
      }
      // [bf16(r/s), ell] per position: r/s formed in FP64 and rounded to FP32,
      // then to BF16 (nearest even, packed hardware rounding); a position
      // outside the grid loaded zeros and stays zero
      uint4 fv[NIT];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const unsigned lo = pack_bf2((float)((double)rv[it].x * inv), (float)((double)rv[it].y * inv));
        const unsigned hi = pack_bf2((float)((double)rv[it].z * inv), (float)((double)rv[it].w * inv));
        fv[it] = make_uint4((lo & 0xFFFFu) | (ev[it].x << 16), (lo >> 16) | (ev[it].x & 0xFFFF0000u),
                            (hi & 0xFFFFu) | (ev[it].y << 16), (hi >> 16) | (ev[it].y & 0xFFFF0000u));
        const int tq = tid + it * 256;
        if ((it + 1) * 256 <= NQ || tq < NQ) *reinterpret_cast<uint4*>(lds + tq * 16) = fv[it];
      }
      if (a.x0) {
        // the features of the brick's own positions, for the backward pass
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
          const int tq = tid + it * 256;
          const int quad = tq % 6, row = tq / 6;
          const int hy = row % kHY, hz = row / kHY;
          const unsigned v[4] = {fv[it].x, fv[it].y, fv[it].z, fv[it].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int hx = 4 * quad - 3 + i;
            if (ok[it] && hx >= 1 && hx <= kTX && hy >= 1 && hy <= kTY && hz >= 1 && hz <= kTZ)
              reinterpret_cast<unsigned*>(a.x0)[p0[it] + i] = v[i];
          }
        }
      }
    } else {
      // 16-byte chunks of the halo, row by row: a row is kHX positions of CG
      // channels; element indices fit in 32 bits at every level
      constexpr int CPP = CG / 8;                  // chunks per position
      constexpr int RCH = kHX * CPP;               // chunks per halo row
      constexpr int NE = kHY * kHZ * RCH;
      constexpr int NIT = (NE + 255) / 256;
      constexpr int BATCH = UPADD ? 6 : NIT;       // loads in flight per thread (registers)
      const int H2 = H >> 1, W2 = W >> 1;
#pragma unroll
      for (int it0 = 0; it0 < NIT; it0 += BATCH) {
        uint4 v[BATCH];
        uint4 c[UPADD ? BATCH : 1];
        int lo[BATCH];
#pragma unroll
        for (int ib = 0; ib < BATCH; ++ib) {
          const int e = tid + (it0 + ib) * 256;
          const int row = e / RCH, rc = e - row * RCH;
          const int hx = rc / CPP, c8 = rc - hx * CPP;
          const int hy = row % kHY, hz = row / kHY;
          const int gx = x0b - 1 + hx, gy = y0b - 1 + hy, gz = z0b - 1 + hz;
          const bool ok = it0 + ib < NIT && e < NE && (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H &&
                          (unsigned)gz < (unsigned)D;
          lo[ib] = (it0 + ib < NIT && e < NE) ? (row * kHX + hx) * ST + c8 * 16 : -1;
          v[ib] = make_uint4(0u, 0u, 0u, 0u);
          if (ok) {
            const unsigned pe = ((unsigned)(gz * H + gy) * (unsigned)W + (unsigned)gx) * CIN + g * CG + c8 * 8;
            v[ib] = *reinterpret_cast<const uint4*>(a.in + pe);
          }
          if constexpr (UPADD) {
            c[ib] = make_uint4(0u, 0u, 0u, 0u);
            if (ok) {
              const unsigned qe =
                  ((unsigned)((gz >> 1) * H2 + (gy >> 1)) * (unsigned)W2 + (unsigned)(gx >> 1)) * CIN + g * CG + c8 * 8;
              c[ib] = *reinterpret_cast<const uint4*>(a.in2 + qe);
            }
          }
        }
#pragma unroll
        for (int ib = 0; ib < BATCH; ++ib) {
          if (lo[ib] >= 0) {
            uint4 w = v[ib];
            if constexpr (UPADD) {
              w.x = add_bf2(w.x, c[ib].x);
              w.y = add_bf2(w.y, c[ib].y);
              w.z = add_bf2(w.z, c[ib].z);
              w.w = add_bf2(w.w, c[ib].w);
            }
            *reinterpret_cast<uint4*>(lds + lo[ib]) = w;
          }
        }
      }
    }
  };

  // features: the staged offsets of this lane's taps 16 kc + 4 kq + i (the
  // padding taps beyond 26 read tap 26; A is zero there)
  int foff[FEAT ? KC : 1][4];
  if constexpr (FEAT) {
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = 16 * kc + 4 * kq + i < 27 ? 16 * kc + 4 * kq + i : 26;
        foff[kc][i] = (t / 9 - 1) * (kHY * RS) + ((t / 3) % 3 - 1) * RS + (t % 3 - 1);
      }
  }

  // ---- one block of 2 x 2 (y, z) rows of 16 positions per wavefront: (yw, zw)
  // its offset in the brick; acc accumulates over the channel groups
  int yw = 0, zw = 0, hb[4];
  f32x4 acc[MT][4];
  long long hp = -1;       // head: output position of this lane, its residual and D^-1
  float hr = 0.f, hd = 0.f;
  auto set_block = [&](int s) {
    yw = 2 * (wv & 1) + 4 * (s % SUB);
    zw = 2 * (wv >> 1) + 4 * (s / SUB);
    // staged index of this lane's output position in each of the four rows
#pragma unroll
    for (int j = 0; j < 4; ++j) hb[j] = ((zw + (j >> 1) + 1) * kHY + (yw + (j & 1) + 1)) * RS + (n + 1 + XO);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  };
  auto compute = [&](auto gg) {
    constexpr int g = decltype(gg)::value;
    // ---- K chunks of this group, unrolled so that every tap offset is an
    // immediate; A from the packed fragments (the next chunk's loads in
    // flight while this chunk multiplies), B from LDS
    int bj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bj[j] = hb[j] * ST;
    auto load_b = [&](auto kcc, Frag (&B)[4]) {
      constexpr int kc = decltype(kcc)::value;
      if constexpr (FEAT) {
        // lane's 8 K values: taps 16 kc + 4 kq + i (i < 4), two channels each
        const unsigned* l32 = reinterpret_cast<const unsigned*>(lds);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          B[j].u = make_uint4(l32[hb[j] + foff[kc][0]], l32[hb[j] + foff[kc][1]], l32[hb[j] + foff[kc][2]],
                              l32[hb[j] + foff[kc][3]]);
      } else if constexpr (CG == 16) {
        // a chunk holds two taps of 16 channels: lanes kq < 2 the even one
        constexpr int t0 = 2 * kc, t1 = 2 * kc + 1 < 27 ? 2 * kc + 1 : 26;
        const int sel = (kq >> 1) ? (tap_halo<HY>(t1) - tap_halo<HY>(t0)) * ST : 0;
        const int lo = (kq & 1) * 16 + sel + tap_halo<HY>(t0) * ST;
#pragma unroll
        for (int j = 0; j < 4; ++j) B[j].u = *reinterpret_cast<const uint4*>(lds + bj[j] + lo);
      } else {
        // a chunk is one tap of the group's 32 channels
        constexpr int t = kc - (kc / KCG) * KCG;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          B[j].u = *reinterpret_cast<const uint4*>(lds + bj[j] + kq * 16 + tap_halo<HY>(t) * ST);
      }
    };
    Frag Bn[4];
    static_for<0, KC>([&](auto kcc) {
      constexpr int kc = decltype(kcc)::value;
      if constexpr (kc >= g * KCG && kc < (g + 1) * KCG) {
        if constexpr (kc == g * KCG) load_b(kcc, Bn);
        Frag A[MT], B[4];
#pragma unroll
        for (int m = 0; m < MT; ++m) A[m] = An[m];
#pragma unroll
        for (int j = 0; j < 4; ++j) B[j] = Bn[j];
        if constexpr (kc + 1 < KC) {
#pragma unroll
          for (int m = 0; m < MT; ++m) An[m].u = load_a((kc + 1) * MT + m);
        }
        if constexpr (kc + 1 < (g + 1) * KCG && kc + 1 < KC) load_b(std::integral_constant<int, kc + 1>{}, Bn);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m].v, B[j].v, acc[m][j], 0, 0, 0);
      }
    });
  };
  auto finish = [&]() {
  // ---- epilogue: lane holds channels m*16 + 4 kq + i of position n in row j;
  // bias, ReLU, the BF16 storage rounding (packed words kept for the stores)
  unsigned pk[MT][4][2];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      pk[m][j][0] = pack_bf2(fmaxf(acc[m][j][0] + bi[m][0], 0.f), fmaxf(acc[m][j][1] + bi[m][1], 0.f));
      pk[m][j][1] = pack_bf2(fmaxf(acc[m][j][2] + bi[m][2], 0.f), fmaxf(acc[m][j][3] + bi[m][3], 0.f));
      acc[m][j][0] = lo_bf(pk[m][j][0]);
      acc[m][j][1] = hi_bf(pk[m][j][0]);
      acc[m][j][2] = lo_bf(pk[m][j][1]);
      acc[m][j][3] = hi_bf(pk[m][j][1]);
    }
  const int x = x0b + n;
  if (a.out) {
    // element offsets in 32 bits (the grid is bounded so that they fit): the
    // block's first row, then rows of W and planes of H W positions
    const unsigned e0 = ((unsigned)((z0b + zw) * H + y0b + yw) * (unsigned)W + (unsigned)x) * COUT + 4 * kq;
    const unsigned ey = (unsigned)W * COUT, ez = (unsigned)(H * W) * COUT;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int y = y0b + yw + (j & 1), z = z0b + zw + (j >> 1);
      if (x < W && y < H && z < D) {
        const unsigned e = e0 + (j & 1) * ey + (j >> 1) * ez;
#pragma unroll
        for (int m = 0; m < MT; ++m)
          *reinterpret_cast<uint2*>(a.out + e + m * 16) = make_uint2(pk[m][j][0], pk[m][j][1]);
      }
    }
  }
  if (a.pooled) {
    // the wavefront's four rows are one 2 x 2 (y, z) block; x pairs are lanes n, n^1
    const int y = y0b + yw, z = z0b + zw;
    const bool ok = (n & 1) == 0 && x < W && y < H && z < D;
    const unsigned q = (unsigned)((z >> 1) * (H >> 1) + (y >> 1)) * (unsigned)(W >> 1) + (unsigned)(x >> 1);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float t = (acc[m][0][i] + acc[m][1][i]) + (acc[m][2][i] + acc[m][3][i]);
        t += __shfl_xor(t, 1);
        v[i] = t * 0.125f;
      }
      if (ok)
        *reinterpret_cast<uint2*>(a.pooled + q * COUT + m * 16 + 4 * kq) =
            make_uint2(pack_bf2(v[0], v[1]), pack_bf2(v[2], v[3]));
    }
  }
  if (a.z) {
    // the 1 x 1 x 1 head: x0[.,0] is the BF16 scaled residual formed exactly as
    // the first encoder's staging forms it
    const double ms = rr / a.nred;
    const double inv = ms > 0 ? 1.0 / sqrt(ms) : 1.0;
    // w . out of row j summed over the lane quarters; quarter kq then
    // finishes row kq, so all 64 lanes form one output each
    float tk = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float t = 0.f;
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) t += wp[m][i] * acc[m][j][i];
      t += __shfl_xor(t, 16);
      t += __shfl_xor(t, 32);
      if (kq == j) tk = t;
    }
    if (hp >= 0) {
      const float x00 = __uint_as_float((unsigned)f2bf((float)((double)hr * inv)) << 16);
      a.z[hp] = hd * ((x00 + pb) + tk);
    }
  }
  };

  if constexpr (SUB == 1) {
    set_block(0);
    if (a.z) {
      // the head's inputs at this lane's output position (row kq of the
      // block), fetched before the staging so that their latency is hidden
      const int x = x0b + n, y = y0b + yw + (kq & 1), z = z0b + zw + (kq >> 1);
      if (x < W && y < H && z < D) {
        hp = ((long long)z * H + y) * W + x;
        hr = a.r[hp];
        hd = a.dinv[hp];
      }
    }
    static_for<0, NG>([&](auto gg) {
      if constexpr (decltype(gg)::value > 0) __syncthreads();
      stage(gg);
      __syncthreads();
      compute(gg);
    });
    finish();
  } else {
    stage(std::integral_constant<int, 0>{});
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < SUB * SUB; ++s) {
      if (s > 0) {
#pragma unroll
        for (int m = 0; m < MT; ++m) An[m].u = load_a(m);
      }
      set_block(s);
      compute(std::integral_constant<int, 0>{});
      finish();
    }
  }
}

// ------------------------------------------------------------ persistent, pipelined form
// The same convolution for 16 input channels without skip addition or head
// (the encoder 16 -> COUT, pooled output optional) on a persistent grid: each
// workgroup walks a strided run of bricks inside its XCD's range.  Its A
// fragments sit in LDS for the whole run.  Each brick's halo is loaded into
// registers while the previous brick multiplies (only LDS reads in the
// multiply loop, so the in-order vector memory counter never makes them wait
// for the halo loads), then written to LDS between two barriers.  Bitwise the
// result of k_tconv.  Measured at 25M cells: the 16 -> 32 encoder 165 -> 123
// us; the 16 -> 16 decoder with its skip sum and head gained nothing in this
// form (the skip sums of every halo copy dominate it) and runs on the
// z-marching form below, which stages a third fewer of them.
template <int COUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_tconv_pipe(const TconvArgs a) {
  constexpr bool UPADD = false;
  if (solve_done(a.sc)) return;
  constexpr int CIN = 16, CG = 16;
  constexpr int KC = (27 * CIN + 31) / 32;         // 14 chunks: two taps of 16 channels each
  constexpr int MT = COUT / 16;
  constexpr int ST = lds_stride<CG>();
  constexpr int kTY = Brick<1>::TY, kTZ = Brick<1>::TZ, kHY = Brick<1>::HY, kHZ = Brick<1>::HZ;
  constexpr int kHalo = Brick<1>::HALO, HY = kHY;
  constexpr int CPP = CG / 8;                      // 16-byte chunks per staged position
  constexpr int RCH = kHX * CPP;                   // chunks per halo row
  constexpr int NE = kHY * kHZ * RCH;
  constexpr int NIT = (NE + 255) / 256;
  __shared__ __align__(16) unsigned char lds[kHalo * ST];
  __shared__ __align__(16) uint4 afr[KC * MT * 64];
  const int D = a.D, H = a.H, W = a.W;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 15, kq = lane >> 4;
  for (int e = tid; e < KC * MT * 64; e += 256) afr[e] = a.frag[e];
  float bi[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) bi[m][i] = a.bias[m * 16 + 4 * kq + i];
  // this workgroup's bricks: XCD x owns [x per, (x+1) per); its G8 workgroups
  // take them round robin
  const int G8 = (int)(gridDim.x >> 3);
  const int xcd = (int)(blockIdx.x & 7), j0 = (int)(blockIdx.x >> 3);
  const int bend = min(a.nb, (xcd + 1) * a.per);
  const int H2 = H >> 1, W2 = W >> 1;
  // the wavefront's 2 x 2 block of rows and the staged index of its lane's
  // output position in each
  const int yw = 2 * (wv & 1), zw = 2 * (wv >> 1);
  int hb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) hb[j] = ((zw + (j >> 1) + 1) * kHY + (yw + (j & 1) + 1)) * kHX + (n + 1);

  // per-thread staging table: for chunk e = tid + it*256 of the halo, its
  // element offset from the brick's first output position (fine level), the
  // offset of its coarse position from the brick's coarse origin (UPADD),
  // its halo coordinates (packed) and its LDS offset; bricks start at even
  // coordinates, so the coarse offsets are brick-independent
  int rel[NIT], qrel[UPADD ? NIT : 1], hpk[NIT], ldo[NIT];
  const int plane2 = H2 * W2;
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = tid + it * 256;
    const int row = e / RCH, rc = e - row * RCH;
    const int hx = rc / CPP, c8 = rc - hx * CPP;
    const int hy = row % kHY, hz = row / kHY;
    rel[it] = (((hz - 1) * H + (hy - 1)) * W + (hx - 1)) * CIN + c8 * 8;
    if constexpr (UPADD) qrel[it] = (((hz - 1) >> 1) * plane2 + ((hy - 1) >> 1) * W2 + ((hx - 1) >> 1)) * CIN + c8 * 8;
    hpk[it] = e < NE ? (hx | (hy << 8) | (hz << 16)) : -1;
    ldo[it] = (row * kHX + hx) * ST + c8 * 16;
  }
  uint4 v[NIT];
  uint4 c[UPADD ? NIT : 1];
  // issue the loads of brick b's halo into registers
  auto issue = [&](int b) {
    const int bx = b % a.nbx, brest = b / a.nbx;
    const int x0b = bx * kTX, y0b = (brest % a.nby) * kTY, z0b = (brest / a.nby) * kTZ;
    const long long base = (((long long)z0b * H + y0b) * W + x0b) * CIN;
    const long long qbase = ((((long long)(z0b >> 1)) * H2 + (y0b >> 1)) * W2 + (x0b >> 1)) * CIN;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int pk = hpk[it];
      const int gx = x0b - 1 + (pk & 255), gy = y0b - 1 + ((pk >> 8) & 255), gz = z0b - 1 + (pk >> 16);
      const bool ok = pk >= 0 && (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H && (unsigned)gz < (unsigned)D;
      v[it] = make_uint4(0u, 0u, 0u, 0u);
      if (ok) v[it] = *reinterpret_cast<const uint4*>(a.in + (base + rel[it]));
      if constexpr (UPADD) {
        c[it] = make_uint4(0u, 0u, 0u, 0u);
        if (ok) c[it] = *reinterpret_cast<const uint4*>(a.in2 + (qbase + qrel[it]));
      }
    }
  };
  // write the registers of the last issue into LDS
  auto commit = [&]() {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      if (hpk[it] >= 0) {
        uint4 w = v[it];
        if constexpr (UPADD) {
          w.x = add_bf2(w.x, c[it].x);
          w.y = add_bf2(w.y, c[it].y);
          w.z = add_bf2(w.z, c[it].z);
          w.w = add_bf2(w.w, c[it].w);
        }
        *reinterpret_cast<uint4*>(lds + ldo[it]) = w;
      }
    }
  };

  int b = xcd * a.per + j0;
  if (b < bend) issue(b);
  while (b < bend) {
    const int bx = b % a.nbx, brest = b / a.nbx;
    const int x0b = bx * kTX, y0b = (brest % a.nby) * kTY, z0b = (brest / a.nby) * kTZ;
    commit();
    __syncthreads();
    const int bn = b + G8;
    if (bn < bend) issue(bn);
    // ---- the brick's K chunks (two taps of 16 channels each), A from LDS
    f32x4 acc[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int bj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bj[j] = hb[j] * ST;
    auto load_b = [&](auto kcc, Frag (&B)[4]) {
      constexpr int kc = decltype(kcc)::value;
      constexpr int t0 = 2 * kc, t1 = 2 * kc + 1 < 27 ? 2 * kc + 1 : 26;
      const int sel = (kq >> 1) ? (tap_halo<HY>(t1) - tap_halo<HY>(t0)) * ST : 0;
      const int lo = (kq & 1) * 16 + sel + tap_halo<HY>(t0) * ST;
#pragma unroll
      for (int j = 0; j < 4; ++j) B[j].u = *reinterpret_cast<const uint4*>(lds + bj[j] + lo);
    };
    Frag An[MT], Bn[4];
#pragma unroll
    for (int m = 0; m < MT; ++m) An[m].u = afr[m * 64 + lane];
    load_b(std::integral_constant<int, 0>{}, Bn);
    static_for<0, KC>([&](auto kcc) {
      constexpr int kc = decltype(kcc)::value;
      Frag A[MT], B[4];
#pragma unroll
      for (int m = 0; m < MT; ++m) A[m] = An[m];
#pragma unroll
      for (int j = 0; j < 4; ++j) B[j] = Bn[j];
      if constexpr (kc + 1 < KC) {
#pragma unroll
        for (int m = 0; m < MT; ++m) An[m].u = afr[((kc + 1) * MT + m) * 64 + lane];
        load_b(std::integral_constant<int, kc + 1>{}, Bn);
      }
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m].v, B[j].v, acc[m][j], 0, 0, 0);
      // keep the one-chunk-ahead schedule: without this fence the scheduler
      // hoists every chunk's LDS reads and the registers triple
      __builtin_amdgcn_sched_barrier(0);
    });
    // ---- epilogue (as in k_tconv): bias, ReLU, BF16 rounding; output,
    // pooled average
    unsigned pk[MT][4][2];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        pk[m][j][0] = pack_bf2(fmaxf(acc[m][j][0] + bi[m][0], 0.f), fmaxf(acc[m][j][1] + bi[m][1], 0.f));
        pk[m][j][1] = pack_bf2(fmaxf(acc[m][j][2] + bi[m][2], 0.f), fmaxf(acc[m][j][3] + bi[m][3], 0.f));
        acc[m][j][0] = lo_bf(pk[m][j][0]);
        acc[m][j][1] = hi_bf(pk[m][j][0]);
        acc[m][j][2] = lo_bf(pk[m][j][1]);
        acc[m][j][3] = hi_bf(pk[m][j][1]);
      }
    const int x = x0b + n;
    if (a.out) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int y = y0b + yw + (j & 1), z = z0b + zw + (j >> 1);
        if (x < W && y < H && z < D) {
          const long long p = ((long long)z * H + y) * W + x;
#pragma unroll
          for (int m = 0; m < MT; ++m)
            *reinterpret_cast<uint2*>(a.out + p * COUT + m * 16 + 4 * kq) = make_uint2(pk[m][j][0], pk[m][j][1]);
        }
      }
    }
    if (a.pooled) {
      const int y = y0b + yw, z = z0b + zw;
      const bool ok = (n & 1) == 0 && x < W && y < H && z < D;
      const long long q = ((long long)(z >> 1) * (H >> 1) + (y >> 1)) * (W >> 1) + (x >> 1);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        float pv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float t = (acc[m][0][i] + acc[m][1][i]) + (acc[m][2][i] + acc[m][3][i]);
          t += __shfl_xor(t, 1);
          pv[i] = t * 0.125f;
        }
        if (ok)
          *reinterpret_cast<uint2*>(a.pooled + q * COUT + m * 16 + 4 * kq) =
              make_uint2(pack_bf2(pv[0], pv[1]), pack_bf2(pv[2], pv[3]));
      }
    }
    b = bn;
    __syncthreads();   // every wavefront is done with this brick's LDS before the next commit
  }
}

// ------------------------------------------------------------ z-marching form of the decoders
// The CIN -> 16 decoders with the skip sum bf16(a_l + up(d_(l+1))) (and, on
// the finest level, the head in the epilogue), on runs of ZB bricks stacked
// in z, one run per workgroup.  Consecutive bricks of a run share two halo
// planes: after the first brick they are moved inside LDS (planes 4, 5 ->
// 0, 1) and only the four new planes are loaded and summed, a third fewer
// per output than separate bricks.  The brick, its LDS layout, the multiply
// and the epilogue are those of k_tconv, so the result is bitwise its.  Per
// brick: the moved planes' LDS reads (and the new planes' loads, when they
// fit in one batch of registers) are issued first, one barrier ends every
// wavefront's reads of the previous brick, the LDS writes follow, and a
// second barrier opens the multiply.
// Registers are held to five wavefronts per SIMD (100 for the 16-channel
// form, no spills); LDS then allows four and three workgroups per CU.
// Measured at 25M cells: the finest decoder 559-575 against 578-585 us with
// the registers unbounded (121).
template <int CIN, int ZB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_tconv_zm(const TconvArgs a) {
  if (solve_done(a.sc)) return;
  static_assert(CIN == 16 || CIN == 32, "one staged group of 16 or 32 channels");
  constexpr int KC = (27 * CIN + 31) / 32;          // K chunks: two taps of 16 channels, or one of 32
  constexpr int kTY = Brick<1>::TY, kTZ = Brick<1>::TZ, kHY = Brick<1>::HY, HY = kHY;
  constexpr int kHalo = Brick<1>::HALO;
  constexpr int ST = lds_stride<CIN>();             // bytes per staged position
  constexpr int CPP = CIN / 8;                      // 16-byte chunks per position
  constexpr int RCH = kHX * CPP;                    // chunks per halo row
  constexpr int PLANE = kHX * kHY;                  // positions per halo plane
  constexpr int NSH = 2 * PLANE * ST / 16;          // chunks of the two moved planes
  constexpr int NITS = (NSH + 255) / 256;
  __shared__ __align__(16) unsigned char lds[kHalo * ST];
  // the 16-channel form keeps its A fragments in LDS for the whole run (the
  // multiply then waits on LDS reads only); the 32-channel one reads them
  // through the caches, since 27.6 KB more LDS would cost it a workgroup per CU
  constexpr bool AL = CIN == 16;
  __shared__ __align__(16) uint4 afr[AL ? KC * 64 : 1];
  // runs in contiguous ranges per XCD (workgroups are dealt to the XCDs round robin)
  const int item = (int)(blockIdx.x & 7) * a.per + (int)(blockIdx.x >> 3);
  if (item >= a.nb) return;
  if constexpr (AL) {
    for (int e = threadIdx.x; e < KC * 64; e += 256) afr[e] = a.frag[e];
  }
  const int D = a.D, H = a.H, W = a.W, H2 = H >> 1, W2 = W >> 1;
  const int nbz = (D + kTZ - 1) / kTZ;
  const int bx = item % a.nbx, rest = item / a.nbx;
  const int x0b = bx * kTX, y0b = (rest % a.nby) * kTY;
  const int zb0 = (rest / a.nby) * ZB;              // the run's first brick in z
  const int nrun = min(ZB, nbz - zb0);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 15, kq = lane >> 4;
  float bi[4], wp[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bi[i] = a.bias[4 * kq + i];
    wp[i] = a.z ? a.wproj[4 * kq + i] : 0.f;
  }
  const float pb = a.z ? a.pbias[0] : 0.f;
  const double rr = a.z ? *a.rr : 0.0;
  // the wavefront's 2 x 2 block of rows and the staged offset of its lane's
  // output position in each
  const int yw = 2 * (wv & 1), zw = 2 * (wv >> 1);
  int bj[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bj[j] = (((zw + (j >> 1) + 1) * kHY + (yw + (j & 1) + 1)) * kHX + (n + 1)) * ST;

  // halo planes [P0, 6) of the brick whose first output plane is z0b, in
  // batches of BATCH chunks per thread: loads into registers (issue), then
  // the skip sum into LDS (commit)
  constexpr int BATCH = 6;
  uint4 v[BATCH], c[BATCH];
  int lo[BATCH];
  auto issue = [&](auto p0c, auto b0c, int z0b) {
    constexpr int P0 = decltype(p0c)::value, B0 = decltype(b0c)::value;
    constexpr int NE = (6 - P0) * kHY * RCH;
    constexpr int NIT = (NE + 255) / 256;
    // the slots' offsets are the same for every brick; formed again here
    // from an opaque copy of the thread index, since held across the run
    // they would cost more registers than the arithmetic costs issue slots
    int t0 = tid;
    asm volatile("" : "+v"(t0));
#pragma unroll
    for (int ib = 0; ib < BATCH; ++ib) {
      const int it = B0 + ib;
      const int e = t0 + it * 256;
      const bool in = it < NIT && e < NE;
      const int r0 = e / RCH, rc = e - r0 * RCH;
      const int row = r0 + P0 * kHY;
      const int hx = rc / CPP, c8 = rc - hx * CPP;
      const int hy = row % kHY, hz = row / kHY;
      const int gx = x0b - 1 + hx, gy = y0b - 1 + hy, gz = z0b - 1 + hz;
      const bool ok = in && (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H && (unsigned)gz < (unsigned)D;
      lo[ib] = in ? (row * kHX + hx) * ST + c8 * 16 : -1;
      v[ib] = make_uint4(0u, 0u, 0u, 0u);
      c[ib] = make_uint4(0u, 0u, 0u, 0u);
      if (ok) {
        const unsigned pe = ((unsigned)(gz * H + gy) * (unsigned)W + (unsigned)gx) * CIN + c8 * 8;
        const unsigned qe =
            ((unsigned)((gz >> 1) * H2 + (gy >> 1)) * (unsigned)W2 + (unsigned)(gx >> 1)) * CIN + c8 * 8;
        v[ib] = *reinterpret_cast<const uint4*>(a.in + pe);
        c[ib] = *reinterpret_cast<const uint4*>(a.in2 + qe);
      }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int ib = 0; ib < BATCH; ++ib) {
      if (lo[ib] >= 0) {
        uint4 w = v[ib];
        w.x = add_bf2(w.x, c[ib].x);
        w.y = add_bf2(w.y, c[ib].y);
        w.z = add_bf2(w.z, c[ib].z);
        w.w = add_bf2(w.w, c[ib].w);
        *reinterpret_cast<uint4*>(lds + lo[ib]) = w;
      }
    }
  };
  // every batch of planes [P0, 6): issue, commit
  auto stage = [&](auto p0c, int z0b) {
    constexpr int P0 = decltype(p0c)::value;
    constexpr int NIT = ((6 - P0) * kHY * RCH + 255) / 256;
    static_for<0, (NIT + BATCH - 1) / BATCH>([&](auto bb) {
      issue(p0c, std::integral_constant<int, decltype(bb)::value * BATCH>{}, z0b);
      commit();
    });
  };

  for (int i = 0; i < nrun; ++i) {
    const int z0b = (zb0 + i) * kTZ;
    // the head's inputs at this lane's output position (row kq of the block)
    long long hp = -1;
    float hr = 0.f, hd = 0.f;
    if (a.z) {
      const int x = x0b + n, y = y0b + yw + (kq & 1), z = z0b + zw + (kq >> 1);
      if (x < W && y < H && z < D) {
        hp = ((long long)z * H + y) * W + x;
        hr = a.r[hp];
        hd = a.dinv[hp];
      }
    }
    constexpr int NIT4 = ((6 - 2) * kHY * RCH + 255) / 256;   // slots of the four new planes
    if (i == 0) {
      stage(std::integral_constant<int, 0>{}, z0b);
    } else {
      uint4 sh[NITS];
      if constexpr (NIT4 <= BATCH) issue(std::integral_constant<int, 2>{}, std::integral_constant<int, 0>{}, z0b);
#pragma unroll
      for (int k = 0; k < NITS; ++k) {
        const int e = tid + k * 256;
        sh[k] = make_uint4(0u, 0u, 0u, 0u);
        if (e < NSH) sh[k] = *reinterpret_cast<const uint4*>(lds + 4 * PLANE * ST + e * 16);
      }
      __syncthreads();   // every wavefront is done reading the previous brick
#pragma unroll
      for (int k = 0; k < NITS; ++k) {
        const int e = tid + k * 256;
        if (e < NSH) *reinterpret_cast<uint4*>(lds + e * 16) = sh[k];
      }
      if constexpr (NIT4 <= BATCH) commit();
      else stage(std::integral_constant<int, 2>{}, z0b);
    }
    __syncthreads();
    // keep each phase's registers to itself: without these fences the
    // scheduler overlaps the staging and the multiply and the registers double
    __builtin_amdgcn_sched_barrier(0);

    // ---- K chunks, unrolled so that every tap offset is an immediate; A from
    // the packed fragments one chunk ahead, B from LDS one chunk ahead
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto load_b = [&](auto kcc, Frag (&B)[4]) {
      constexpr int kc = decltype(kcc)::value;
      if constexpr (CIN == 16) {
        // a chunk holds two taps of 16 channels: lanes kq < 2 the even one
        constexpr int t0 = 2 * kc, t1 = 2 * kc + 1 < 27 ? 2 * kc + 1 : 26;
        const int sel = (kq >> 1) ? (tap_halo<HY>(t1) - tap_halo<HY>(t0)) * ST : 0;
        const int lb = (kq & 1) * 16 + sel + tap_halo<HY>(t0) * ST;
#pragma unroll
        for (int j = 0; j < 4; ++j) B[j].u = *reinterpret_cast<const uint4*>(lds + bj[j] + lb);
      } else {
        // a chunk is one tap of the 32 channels
#pragma unroll
        for (int j = 0; j < 4; ++j)
          B[j].u = *reinterpret_cast<const uint4*>(lds + bj[j] + kq * 16 + tap_halo<HY>(kc) * ST);
      }
    };
    // the A fragments are the same for every brick: reloaded (from LDS, or
    // L1 / L2 hits) from an opaque copy of the lane index rather than held
    // across the run, which cost 56 registers (193 against 121 before the
    // register bound)
    int lv = lane;
    asm volatile("" : "+v"(lv));
    const uint4* fr = a.frag + lv;
    auto load_a = [&](int kc) { return AL ? afr[kc * 64 + lane] : fr[kc * 64]; };
    Frag An, Bn[4];
    An.u = load_a(0);
    load_b(std::integral_constant<int, 0>{}, Bn);
    static_for<0, KC>([&](auto kcc) {
      constexpr int kc = decltype(kcc)::value;
      Frag A = An, B[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) B[j] = Bn[j];
      if constexpr (kc + 1 < KC) {
        An.u = load_a(kc + 1);
        load_b(std::integral_constant<int, kc + 1>{}, Bn);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.v, B[j].v, acc[j], 0, 0, 0);
    });

    // ---- epilogue: bias, ReLU, the BF16 storage rounding; the output (when
    // kept) and the head z = dinv (x0[.,0] + (b + w . out))
    unsigned pk[4][2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      pk[j][0] = pack_bf2(fmaxf(acc[j][0] + bi[0], 0.f), fmaxf(acc[j][1] + bi[1], 0.f));
      pk[j][1] = pack_bf2(fmaxf(acc[j][2] + bi[2], 0.f), fmaxf(acc[j][3] + bi[3], 0.f));
      acc[j][0] = lo_bf(pk[j][0]);
      acc[j][1] = hi_bf(pk[j][0]);
      acc[j][2] = lo_bf(pk[j][1]);
      acc[j][3] = hi_bf(pk[j][1]);
    }
    const int x = x0b + n;
    if (a.out) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int y = y0b + yw + (j & 1), z = z0b + zw + (j >> 1);
        if (x < W && y < H && z < D) {
          const long long p = ((long long)z * H + y) * W + x;
          *reinterpret_cast<uint2*>(a.out + p * 16 + 4 * kq) = make_uint2(pk[j][0], pk[j][1]);
        }
      }
    }
    if (a.z) {
      const double ms = rr / a.nred;
      const double inv = ms > 0 ? 1.0 / sqrt(ms) : 1.0;
      float tk = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float t = 0.f;
#pragma unroll
        for (int i2 = 0; i2 < 4; ++i2) t += wp[i2] * acc[j][i2];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        if (kq == j) tk = t;
      }
      if (hp >= 0) {
        const float x00 = __uint_as_float((unsigned)f2bf((float)((double)hr * inv)) << 16);
        a.z[hp] = hd * ((x00 + pb) + tk);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ------------------------------------------------------------ weight gradient (MFMA)
// partial[t][blk][ci][co] = sum over this workgroup's positions m of
//   in'[m + off_t][ci] * dout[m][co]
template <int CIN, int COUT, bool UPADD>
__global__ __launch_bounds__(256) void k_wgrad(int D, int H, int W, const bf16_t* __restrict__ in,
                                               const bf16_t* __restrict__ in2,
                                               const bf16_t* __restrict__ dout,
                                               float* __restrict__ partial) {
  constexpr int MT = COUT / 16;
  constexpr int NT = CIN >= 16 ? CIN / 16 : 1;
  __shared__ float red[4][MT * NT * 4 * 64];
  const int t = blockIdx.y;
  int dz, dy, dx;
  tap_offset(t, dz, dy, dx);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const long long N = (long long)D * H * W;
  const int H2 = H >> 1, W2 = W >> 1;
  f32x4 acc[MT][NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long long chunk = (long long)blockIdx.x * 4 + wv; chunk * 32 < N; chunk += (long long)gridDim.x * 4) {
    const long long m0 = chunk * 32 + kq * 8;
    Frag A[MT], B[NT];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long long m = m0 + j;
      const bool mok = m < N;
#pragma unroll
      for (int a = 0; a < MT; ++a) A[a].h[j] = mok ? dout[m * COUT + a * 16 + col] : (bf16_t)0;
      bool ok = false;
      long long p = 0, q = 0;
      if (mok) {
        const int x = (int)(m % W);
        const long long r2 = m / W;
        const int y = (int)(r2 % H), z = (int)(r2 / H);
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        ok = zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
        p = ((long long)zz * H + yy) * W + xx;
        q = ((long long)(zz >> 1) * H2 + (yy >> 1)) * W2 + (xx >> 1);
      }
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const int ci = b * 16 + col;
        bf16_t v = 0;
        if (ok && ci < CIN) {
          v = in[p * CIN + ci];
          if constexpr (UPADD) v = f2bf(bf2f(v) + bf2f(in2[q * CIN + ci]));
        }
        B[b].h[j] = v;
      }
    }
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a].v, B[b].v, acc[a][b], 0, 0, 0);
  }
  // D[co][ci]: lane holds co = a*16 + 4*kq + i, ci = b*16 + col
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wv][((a * NT + b) * 4 + i) * 64 + lane] = acc[a][b][i];
  __syncthreads();
  float* out = partial + ((long long)t * gridDim.x + blockIdx.x) * CIN * COUT;
  for (int e = threadIdx.x; e < MT * NT * 4 * 64; e += blockDim.x) {
    const float s = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    const int ln = e & 63, rest = e >> 6;
    const int i = rest & 3, ab = rest >> 2;
    const int a = ab / NT, b = ab % NT;
    const int co = a * 16 + 4 * (ln >> 4) + i, ci = b * 16 + (ln & 15);
    if (ci < CIN) out[ci * COUT + co] = s;
  }
}

// The same weight gradient for the shapes with at most two 16 x 16 output
// tiles (CIN, COUT in {16, 32}, (CIN / 16) (COUT / 16) <= 2), the taps of one z
// offset (nine) per pass over the positions: their accumulators stay in
// registers, dout and the positions' coordinates are taken once per chunk of
// 32 positions and pass, and the input's nine shifted reads of a chunk hit the
// caches (one workgroup per tap reads dout and the input from memory 27
// times).  partial[t][blk][ci][co] as k_wgrad, over gridDim.x blocks.
constexpr int kWgrad27Blocks = 1024;
template <int CIN, int COUT, bool UPADD>
__global__ __launch_bounds__(256) void k_wgrad27(int D, int H, int W, const bf16_t* __restrict__ in,
                                                 const bf16_t* __restrict__ in2,
                                                 const bf16_t* __restrict__ dout, float* __restrict__ partial) {
  constexpr int MT = COUT / 16, NT = (CIN + 15) / 16;
  static_assert(COUT % 16 == 0 && MT * NT <= 2, "at most two 16 x 16 output tiles");
  __shared__ float red[4][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  // positions fit in 32 bits (the network's grids have at most 2^28 cells)
  const unsigned N = (unsigned)D * (unsigned)H * (unsigned)W;
  const unsigned nchunk = (N + 31u) / 32u;
  const int H2 = H >> 1, W2 = W >> 1;
#pragma unroll 1
  for (int g = 0; g < 3; ++g) {
    const int dz = g - 1;
    f32x4 acc[9][MT][NT];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[k][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (unsigned chunk = blockIdx.x * 4u + wv; chunk < nchunk; chunk += gridDim.x * 4u) {
      const unsigned m0 = chunk * 32u + kq * 8u;
      // this lane's 8 positions: dout (co = a 16 + col), and the coordinates
      // in the plane z + dz (-4 when outside the grid: every tap then falls
      // outside)
      Frag A[MT];
      int xs[8], ys[8], zs[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const unsigned m = m0 + j;
        const bool mok = m < N;
#pragma unroll
        for (int a = 0; a < MT; ++a) A[a].h[j] = mok ? dout[(size_t)m * COUT + a * 16 + col] : (bf16_t)0;
        const unsigned r2 = m / (unsigned)W;
        const int zz = (int)(r2 / (unsigned)H) + dz;
        const bool zok = mok && (unsigned)zz < (unsigned)D;
        xs[j] = zok ? (int)(m - r2 * (unsigned)W) : -4;
        ys[j] = (int)(r2 % (unsigned)H);
        zs[j] = zz;
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int dy = k / 3 - 1, dx = k % 3 - 1;
        Frag B[NT];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int yy = ys[j] + dy, xx = xs[j] + dx;
          const bool ok = (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
          // element offsets in 32 bits (at most 2^28 cells of 16 channels)
          const unsigned pe = ok ? ((unsigned)(zs[j] * H + yy) * (unsigned)W + (unsigned)xx) * CIN : 0u;
          const unsigned qe =
              ok && UPADD ? ((unsigned)((zs[j] >> 1) * H2 + (yy >> 1)) * (unsigned)W2 + (unsigned)(xx >> 1)) * CIN : 0u;
#pragma unroll
          for (int b = 0; b < NT; ++b) {
            const int ci = b * 16 + col;
            bf16_t v = 0;
            if (ok && ci < CIN) {
              v = in[pe + ci];
              if constexpr (UPADD) v = f2bf(bf2f(v) + bf2f(in2[qe + ci]));
            }
            B[b].h[j] = v;
          }
        }
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
          for (int b = 0; b < NT; ++b)
            acc[k][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a].v, B[b].v, acc[k][a][b], 0, 0, 0);
        // at most three taps' loads in flight: the registers stay bounded
        if (k % 3 == 2) __builtin_amdgcn_sched_barrier(0);
      }
    }
    // D[co][ci] per tap and tile: lane holds co = a 16 + 4 kq + i, ci = b 16
    // + col; the four wavefronts' tiles added in order
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) {
#pragma unroll
          for (int i = 0; i < 4; ++i) red[wv][i * 64 + lane] = acc[k][a][b][i];
          __syncthreads();
          const int e = threadIdx.x, ln = e & 63, i = e >> 6;
          const int co = a * 16 + 4 * (ln >> 4) + i, ci = b * 16 + (ln & 15);
          const float sum = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
          if (ci < CIN)
            partial[((size_t)(9 * g + k) * gridDim.x + blockIdx.x) * (CIN * COUT) + ci * COUT + co] = sum;
          __syncthreads();
        }
  }
}

// The first encoder's weight gradient (CIN = 2, COUT = 16) with the 54
// (tap, channel) pairs as the MFMA's columns, 16 to a tile: column n of tile
// T is tap 8 T + n / 2, channel n % 2 (taps past 26 are zero), so a chunk of
// 32 positions takes four multiplies instead of one per tap; one pass over
// the positions.  partial[t][blk][ci][co] as k_wgrad.
template <int BLK>
__global__ __launch_bounds__(256) void k_wgrad_c2(int D, int H, int W, const bf16_t* __restrict__ in,
                                                  const bf16_t* __restrict__ dout, float* __restrict__ partial) {
  constexpr int CIN = 2, COUT = 16;
  __shared__ float red[4][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const unsigned N = (unsigned)D * (unsigned)H * (unsigned)W;
  const unsigned nchunk = (N + 31u) / 32u;
  // this lane's column in each tile: tap offsets and channel
  int tdz[4], tdy[4], tdx[4];
  bool tok[4];
  const int ci = col & 1;
#pragma unroll
  for (int T = 0; T < 4; ++T) {
    const int t = 8 * T + (col >> 1);
    tok[T] = t < 27;
    tdz[T] = t / 9 - 1;
    tdy[T] = (t / 3) % 3 - 1;
    tdx[T] = t % 3 - 1;
  }
  f32x4 acc[4];
#pragma unroll
  for (int T = 0; T < 4; ++T) acc[T] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (unsigned chunk = blockIdx.x * 4u + wv; chunk < nchunk; chunk += gridDim.x * 4u) {
    const unsigned m0 = chunk * 32u + kq * 8u;
    Frag A;
    int xs[8], ys[8], zs[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned m = m0 + j;
      const bool mok = m < N;
      A.h[j] = mok ? dout[(size_t)m * COUT + col] : (bf16_t)0;
      const unsigned r2 = m / (unsigned)W;
      xs[j] = mok ? (int)(m - r2 * (unsigned)W) : -4;     // -4: every tap falls outside
      ys[j] = (int)(r2 % (unsigned)H);
      zs[j] = (int)(r2 / (unsigned)H);
    }
#pragma unroll
    for (int T = 0; T < 4; ++T) {
      Frag B;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int zz = zs[j] + tdz[T], yy = ys[j] + tdy[T], xx = xs[j] + tdx[T];
        const bool ok = tok[T] && (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
        B.h[j] = ok ? in[((unsigned)(zz * H + yy) * (unsigned)W + (unsigned)xx) * CIN + ci] : (bf16_t)0;
      }
      acc[T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.v, B.v, acc[T], 0, 0, 0);
    }
  }
  // D[co][n] per tile: lane holds co = 4 kq + i, column n = col; the four
  // wavefronts' tiles added in order
#pragma unroll
  for (int T = 0; T < 4; ++T) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wv][i * 64 + lane] = acc[T][i];
    __syncthreads();
    const int e = threadIdx.x, ln = e & 63, i = e >> 6;
    const int co = 4 * (ln >> 4) + i, n = ln & 15, t = 8 * T + (n >> 1);
    const float sum = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    if (t < 27) partial[((size_t)t * BLK + blockIdx.x) * (CIN * COUT) + (n & 1) * COUT + co] = sum;
    __syncthreads();
  }
}

// out[p][c] = bf16(a[p][c] + up(d)[p][c]), the decoder's skip sum (as the
// weight-gradient kernels form it on the fly), 8 channels per thread
template <int C>
__global__ void k_skipsum(int D, int H, int W, const bf16_t* __restrict__ a, const bf16_t* __restrict__ d,
                          bf16_t* __restrict__ out) {
  const long long n = (long long)D * H * W * (C / 8);
  const int H2 = H >> 1, W2 = W >> 1;
  GRID_STRIDE(e, n) {
    const int g = (int)(e % (C / 8));
    const long long p = e / (C / 8);
    const int x = (int)(p % W);
    const long long r = p / W;
    const int y = (int)(r % H), z = (int)(r / H);
    const long long q = ((long long)(z >> 1) * H2 + (y >> 1)) * W2 + (x >> 1);
    Frag va, vd, o;
    va.u = *reinterpret_cast<const uint4*>(a + p * C + g * 8);
    vd.u = *reinterpret_cast<const uint4*>(d + q * C + g * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) o.h[j] = f2bf(bf2f(va.h[j]) + bf2f(vd.h[j]));
    *reinterpret_cast<uint4*>(out + p * C + g * 8) = o.u;
  }
}

// g[t][ci][co] = sum_blk partial[t][blk][ci][co] (fixed order)
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int nblk, int per_tap, float* __restrict__ g) {
  GRID_STRIDE(e, 27LL * per_tap) {
    const long long t = e / per_tap, k = e % per_tap;
    const float* src = partial + t * nblk * per_tap + k;
    // eight running sums (block b into sum b % 8, their loads independent),
    // added in a fixed order
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 8 <= nblk; b += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += src[(long long)(b + u) * per_tap];
    }
    for (; b < nblk; ++b) s[0] += src[(long long)b * per_tap];
    g[e] = (float)(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
  }
}

// column sums of dout [n][C] -> partial[blk][C] (C = 16, 32 or 64): a
// thread sums 8 channels of one position per 16-byte load, four positions
// in flight, on a grid-stride walk over the positions; fixed order throughout
constexpr int kColsumBlocks = 1024;
template <int C>
__global__ __launch_bounds__(256) void k_colsum(long long n, const bf16_t* __restrict__ dout, float* __restrict__ partial) {
  static_assert(C == 16 || C == 32 || C == 64, "channels: 16, 32 or 64");
  constexpr int TPP = C / 8;               // threads per position
  constexpr int PPW = 256 / TPP;           // positions per workgroup and step
  __shared__ float red[8][256];
  const int g = threadIdx.x % TPP, sub = threadIdx.x / TPP;
  const long long step = (long long)gridDim.x * PPW;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  long long m = (long long)blockIdx.x * PPW + sub;
  for (; m + 3 * step < n; m += 4 * step) {
    Frag v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u].u = *reinterpret_cast<const uint4*>(dout + (m + u * step) * C + g * 8);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += bf2f(v[u].h[j]);
  }
  for (; m < n; m += step) {
    Frag v;
    v.u = *reinterpret_cast<const uint4*>(dout + m * C + g * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += bf2f(v.h[j]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) red[j][threadIdx.x] = s[j];
  __syncthreads();
  if (threadIdx.x < C) {
    // channel c = 8 gg + j: the threads (q, gg) of every position slot q
    const int gg = threadIdx.x / 8, j = threadIdx.x % 8;
    float a = 0.f;
    for (int q = 0; q < PPW; ++q) a += red[j][q * TPP + gg];
    partial[blockIdx.x * C + threadIdx.x] = a;
  }
}

// g[c] = sum_b partial[b*width + c] for c < C (C divides 256), in FP64: the
// 256 / C threads of a channel take every (256 / C)-th partial, then their
// sums are added in thread order
__global__ __launch_bounds__(256) void k_colsum_reduce(const float* __restrict__ partial, int nblk, int width, int C,
                                                       float* __restrict__ g) {
  __shared__ double red[256];
  const int S = 256 / C, c = threadIdx.x % C, sub = threadIdx.x / C;
  double acc = 0.0;
  for (int b = sub; b < nblk; b += S) acc += partial[(long long)b * width + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < C) {
    double a = 0.0;
    for (int q = 0; q < S; ++q) a += red[q * C + threadIdx.x];
    g[threadIdx.x] = (float)a;
  }
}

// ------------------------------------------------------------ pooling / upsampling
// coarse[p][c] = bf16((sum of the 8 fine children of grad) * (mask[p][c] > 0))
template <int C>
__global__ void k_upT_mask(int Dc, int Hc, int Wc, const bf16_t* __restrict__ fine,
                           const bf16_t* __restrict__ mask, bf16_t* __restrict__ coarse) {
  const long long n = (long long)Dc * Hc * Wc * (C / 8);
  const int Hf = 2 * Hc, Wf = 2 * Wc;
  GRID_STRIDE(e, n) {
    const int g = (int)(e % (C / 8));
    const long long p = e / (C / 8);
    const int x = (int)(p % Wc);
    const long long r = p / Wc;
    const int y = (int)(r % Hc), z = (int)(r / Hc);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const long long f = ((long long)(2 * z + c) * Hf + (2 * y + b)) * Wf + (2 * x + a);
          Frag v;
          v.u = *reinterpret_cast<const uint4*>(fine + f * C + g * 8);
#pragma unroll
          for (int j = 0; j < 8; ++j) s[j] += bf2f(v.h[j]);
        }
    Frag m, o;
    m.u = *reinterpret_cast<const uint4*>(mask + p * C + g * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) o.h[j] = f2bf(bf2f(m.h[j]) > 0.f ? s[j] : 0.f);
    *reinterpret_cast<uint4*>(coarse + p * C + g * 8) = o.u;
  }
}

// fine[p][c] = bf16((skip[p][c] + coarse[parent][c] / 8) * (mask[p][c] > 0))
template <int C>
__global__ void k_skip_poolT_mask(int D, int H, int W, const bf16_t* __restrict__ skip,
                                  const bf16_t* __restrict__ coarse, const bf16_t* __restrict__ mask,
                                  bf16_t* __restrict__ fine) {
  const long long n = (long long)D * H * W * (C / 8);
  const int H2 = H >> 1, W2 = W >> 1;
  GRID_STRIDE(e, n) {
    const int g = (int)(e % (C / 8));
    const long long p = e / (C / 8);
    const int x = (int)(p % W);
    const long long r = p / W;
    const int y = (int)(r % H), z = (int)(r / H);
    const long long q = ((long long)(z >> 1) * H2 + (y >> 1)) * W2 + (x >> 1);
    Frag s, c, m, o;
    s.u = *reinterpret_cast<const uint4*>(skip + p * C + g * 8);
    c.u = *reinterpret_cast<const uint4*>(coarse + q * C + g * 8);
    m.u = *reinterpret_cast<const uint4*>(mask + p * C + g * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = bf2f(s.h[j]) + bf2f(c.h[j]) * 0.125f;
      o.h[j] = f2bf(bf2f(m.h[j]) > 0.f ? v : 0.f);
    }
    *reinterpret_cast<uint4*>(fine + p * C + g * 8) = o.u;
  }
}

// ------------------------------------------------------------ head (1 x 1 x 1, 16 -> 1)
// data gradient through the head into the finest decoder's pre-activation:
// dd0[p][c] = bf16(w6[c] dy[p]) where d0[p][c] > 0, else 0;  dy = dinv * dz
__global__ void k_head_dgrad(long long n, const float* __restrict__ dz, const float* __restrict__ dinv,
                             const float* __restrict__ w6, const bf16_t* __restrict__ d0, bf16_t* __restrict__ dd0) {
  GRID_STRIDE(p, n) {
    const float g = dinv[p] * dz[p];
    Frag m0, m1, o0, o1;
    m0.u = *reinterpret_cast<const uint4*>(d0 + p * 16);
    m1.u = *reinterpret_cast<const uint4*>(d0 + p * 16 + 8);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      o0.h[c] = bf2f(m0.h[c]) > 0.f ? f2bf(w6[c] * g) : (bf16_t)0;
      o1.h[c] = bf2f(m1.h[c]) > 0.f ? f2bf(w6[8 + c] * g) : (bf16_t)0;
    }
    *reinterpret_cast<uint4*>(dd0 + p * 16) = o0.u;
    *reinterpret_cast<uint4*>(dd0 + p * 16 + 8) = o1.u;
  }
}

// weight gradient of the head, per workgroup: partial[blk][c] = sum_p dy[p]
// d0[p][c] for c < 16, partial[blk][16] = sum_p dy[p]
constexpr int kHeadBlocks = 256;
__global__ __launch_bounds__(256) void k_head_wgrad(long long n, const float* __restrict__ dz,
                                                    const float* __restrict__ dinv, const bf16_t* __restrict__ d0,
                                                    float* __restrict__ partial) {
  __shared__ float red[17][256];
  float acc[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) acc[c] = 0.f;
  GRID_STRIDE(p, n) {
    const float g = dinv[p] * dz[p];
    Frag a[2];
    a[0].u = *reinterpret_cast<const uint4*>(d0 + p * 16);
    a[1].u = *reinterpret_cast<const uint4*>(d0 + p * 16 + 8);
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] += g * bf2f(a[c >> 3].h[c & 7]);
    acc[16] += g;
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  if (threadIdx.x < 17) {
    float t = 0.f;
    for (int k = 0; k < 256; ++k) t += red[threadIdx.x][k];
    partial[blockIdx.x * 17 + threadIdx.x] = t;
  }
}

// g[c] = sum_blk partial[blk][c] (fixed order, FP64): weights g[0..16), bias gb
__global__ void k_head_wgrad_reduce(const float* __restrict__ partial, int nblk, float* __restrict__ gw,
                                    float* __restrict__ gb) {
  const int c = threadIdx.x;
  if (c >= 17) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += partial[b * 17 + c];
  if (c < 16) gw[c] = (float)t;
  else gb[0] = (float)t;
}

// ------------------------------------------------------------ loss gradient
// coef = (a = z.r, c = z.Az); dz = -(2a/(c eAe)) (r - (a/c) Az)
__global__ void k_loss_grad(long long n, const float* __restrict__ r, const float* __restrict__ Az,
                            const double* __restrict__ coef, double eAe, float* __restrict__ dz) {
  const double a = coef[0], c = coef[1];
  const double f = -2.0 * a / (c * eAe), g = a / c;
  GRID_STRIDE(i, n) dz[i] = (float)(f * ((double)r[i] - g * (double)Az[i]));
}

// ------------------------------------------------------------ parameters
__global__ void k_adam(long long n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  GRID_STRIDE(i, n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// forward fragments of the tiled convolution: frag[(kc*MT+mt)*64 + lane][j] =
// W[t][g*CG + c][co] for k = kc*32 + (lane/16)*8 + j taken in the order of the
// staged channel groups, k = g*(27*CG) + t*CG + c (CG = min(cin, 32) channels
// per group), co = mt*16 + lane%16; 0 beyond K = 27*cin
__global__ void k_pack_tile(const float* __restrict__ w, int cin, int cout, bf16_t* __restrict__ frag) {
  const int K = 27 * cin, KS = (K + 31) / 32, MT = cout / 16, CG = cin < 32 ? cin : 32;
  GRID_STRIDE(e, (long long)KS * MT * 64 * 8) {
    const int j = (int)(e % 8);
    const long long f = e / 8;
    const int lane = (int)(f % 64);
    const long long km = f / 64;
    const int mt = (int)(km % MT), ks = (int)(km / MT);
    const int k = ks * 32 + (lane >> 4) * 8 + j, co = mt * 16 + (lane & 15);
    bf16_t v = 0;
    if (k < K) {
      const int g = k / (27 * CG), kl = k % (27 * CG);
      const int t = kl / CG, ci = g * CG + kl % CG;
      v = f2bf(w[((long long)t * cin + ci) * cout + co]);
    }
    frag[e] = v;
  }
}

// data-gradient fragments: the conv cout -> cin with W'[t'][co][ci] = W[26-t'][ci][co]
__global__ void k_pack_bwd(const float* __restrict__ w, int cin, int cout, bf16_t* __restrict__ frag) {
  const int K = 27 * cout, KS = (K + 31) / 32, MT = cin / 16;
  GRID_STRIDE(e, (long long)KS * MT * 64 * 8) {
    const int j = (int)(e % 8);
    const long long f = e / 8;
    const int lane = (int)(f % 64);
    const long long km = f / 64;
    const int mt = (int)(km % MT), ks = (int)(km / MT);
    const int k = ks * 32 + (lane >> 4) * 8 + j, ci = mt * 16 + (lane & 15);
    bf16_t v = 0;
    if (k < K) {
      const int tp = k / cout, co = k % cout;
      v = f2bf(w[((long long)(26 - tp) * cin + ci) * cout + co]);
    }
    frag[e] = v;
  }
}

// head weights rounded to BF16 (kept as float)
__global__ void k_pack_head(const float* __restrict__ w, float* __restrict__ wq) {
  for (int e = threadIdx.x; e < 16; e += blockDim.x) wq[e] = bf2f(f2bf(w[e]));
}

}  // namespace

// ============================================================== host side
// Channels per level 16, 32, 64, 64, ...; convolutions in parameter order:
// encoder e_0..e_{L-1}, bottleneck b, decoder d_{L-2}..d_0, head (16 -> 1,
// 1 x 1 x 1); all others 3 x 3 x 3.
inline int level_channels(int l) { return l == 0 ? 16 : l == 1 ? 32 : 64; }

struct UNet {
  int nx = 0, ny = 0, nz = 0, L = 3;
  long long npos[kMaxLevels] = {0};
  int nlayers = 0;
  std::vector<int> cin, cout;
  std::vector<long long> off_w, off_b;
  long long nparam = 0;
  DevBuf params, grads, adam_m, adam_v;              // FP32, nparam
  std::vector<DevBuf> frag_t, frag_b;                // packed BF16 weight fragments (forward tiles, data gradient)
  DevBuf head_w;                                     // 16 head weights, BF16 values
  DevBuf x0, ell;
  DevBuf a[kMaxLevels], p[kMaxLevels], d[kMaxLevels];            // activations (BF16)
  DevBuf skip[kMaxLevels], dd[kMaxLevels], da[kMaxLevels], dp[kMaxLevels];  // gradients (BF16)
  DevBuf zt, Az, dz;                                 // FP32 cells
  DevBuf wpart, cpart, hpart;                        // FP32 partials of the weight gradients
  DevBuf scal;                                       // double: rr, a, c
  const void* ell_op = nullptr;
  int ell_version = -1;
  // what the activations of the last forward belong to (nfa_unet_backward)
  long long param_version = 0;        // counts parameter changes (pack_all)
  const void* fwd_op = nullptr;
  int fwd_version = -1;
  long long fwd_params = -1;
  bool fwd_kept = false;
  int E(int l) const { return l; }
  int B() const { return L; }
  int Dl(int l) const { return L + 1 + (L - 2 - l); }
  int Hd() const { return 2 * L; }
  void dims(int l, int& D, int& H, int& W) const { D = nz >> l; H = ny >> l; W = nx >> l; }
};

}  // namespace nfa

struct nfa_unet_s : nfa::UNet {};

namespace nfa {
namespace {

void layer_shapes(int L, std::vector<int>& ci, std::vector<int>& co) {
  ci.clear();
  co.clear();
  ci.push_back(2);
  co.push_back(16);
  for (int l = 1; l < L; ++l) { ci.push_back(level_channels(l - 1)); co.push_back(level_channels(l)); }
  ci.push_back(level_channels(L - 1));
  co.push_back(level_channels(L - 2));
  for (int l = L - 2; l >= 1; --l) { ci.push_back(level_channels(l)); co.push_back(level_channels(l - 1)); }
  ci.push_back(16);   // decoder d_0
  co.push_back(16);
  ci.push_back(16);   // head
  co.push_back(1);
}

long long count_params(int L, std::vector<long long>* off_w, std::vector<long long>* off_b) {
  std::vector<int> ci, co;
  layer_shapes(L, ci, co);
  long long o = 0;
  for (size_t l = 0; l < ci.size(); ++l) {
    const long long taps = l + 1 == ci.size() ? 1 : 27;
    if (off_w) off_w->push_back(o);
    o += taps * ci[l] * co[l];
    if (off_b) off_b->push_back(o);
    o += co[l];
  }
  return o;
}

inline int eblocks(long long n) { return blocks_for(n, kBlock, 8192); }
inline long long tile_frag_bytes(int cin, int cout) { return (long long)((27 * cin + 31) / 32) * (cout / 16) * 64 * 16; }

nfa_status pack_all(UNet& u, hipStream_t s) {
  ++u.param_version;
  const float* P = u.params.as<float>();
  for (int l = 0; l < u.nlayers - 1; ++l) {
    const int cin = u.cin[l], cout = u.cout[l];
    k_pack_tile<<<eblocks(tile_frag_bytes(cin, cout) / 2), kBlock, 0, s>>>(P + u.off_w[l], cin, cout,
                                                                            u.frag_t[l].as<bf16_t>());
    if (l > 0) {
      const long long nb = (long long)((27 * cout + 31) / 32) * (cin / 16) * 64 * 8;
      k_pack_bwd<<<eblocks(nb), kBlock, 0, s>>>(P + u.off_w[l], cin, cout, u.frag_b[l].as<bf16_t>());
    }
  }
  k_pack_head<<<1, 64, 0, s>>>(P + u.off_w[u.Hd()], u.head_w.as<float>());
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

// ---------------------------------------------------------------- forward convolutions
template <int CIN, int COUT, bool UPADD, bool FEAT, int SUB = 1>
void tconv_t(TconvArgs a, hipStream_t s) {
  a.nbx = (a.W + kTX - 1) / kTX;
  a.nby = (a.H + Brick<SUB>::TY - 1) / Brick<SUB>::TY;
  a.nb = a.nbx * a.nby * ((a.D + Brick<SUB>::TZ - 1) / Brick<SUB>::TZ);
  a.per = (a.nb + 7) / 8;
  k_tconv<CIN, COUT, UPADD, FEAT, SUB><<<8 * a.per, 256, 0, s>>>(a);
}

// persistent launch of k_tconv_pipe: as many workgroups as fit on the device
// at once (a multiple of 8, so that each XCD gets the same number)
template <int COUT> void tconv_pipe_t(TconvArgs a, hipStream_t s) {
  a.nbx = (a.W + kTX - 1) / kTX;
  a.nby = (a.H + Brick<1>::TY - 1) / Brick<1>::TY;
  a.nb = a.nbx * a.nby * ((a.D + Brick<1>::TZ - 1) / Brick<1>::TZ);
  a.per = (a.nb + 7) / 8;
  const int res = resident_blocks(reinterpret_cast<const void*>(&k_tconv_pipe<COUT>), 256);
  const int g8 = std::max(1, std::min(res / 8, a.per));
  k_tconv_pipe<COUT><<<8 * g8, 256, 0, s>>>(a);
}

// runs of ZB bricks in z, one per workgroup
template <int CIN, int ZB> void tconv_zm_t(TconvArgs a, hipStream_t s) {
  a.nbx = (a.W + kTX - 1) / kTX;
  a.nby = (a.H + Brick<1>::TY - 1) / Brick<1>::TY;
  const int nbz = (a.D + Brick<1>::TZ - 1) / Brick<1>::TZ;
  a.nb = a.nbx * a.nby * ((nbz + ZB - 1) / ZB);
  a.per = (a.nb + 7) / 8;
  k_tconv_zm<CIN, ZB><<<8 * a.per, 256, 0, s>>>(a);
}

nfa_status tconv(int cin, int cout, bool upadd, const TconvArgs& a, hipStream_t s) {
  if (cin == 16 && cout == 32 && !upadd) { tconv_pipe_t<32>(a, s); return NFA_OK; }
  // run lengths measured at 25M cells: the finest decoder 654 / 637 / 613 / 635
  // us with runs of 4 / 8 / 16 / 24 bricks, the 32 -> 16 one 192 / 186 / 284 /
  // 206 us (runs of 16 leave its level too few workgroups)
  if (cin == 16 && cout == 16 && upadd && !a.pooled) { tconv_zm_t<16, 16>(a, s); return NFA_OK; }
  if (cin == 32 && cout == 16 && upadd && !a.pooled) { tconv_zm_t<32, 8>(a, s); return NFA_OK; }
#define T_(A, B, U) \
  if (cin == A && cout == B && upadd == U) { tconv_t<A, B, U, false>(a, s); return NFA_OK; }
  T_(32, 64, false) T_(64, 64, false) T_(64, 32, false)
  T_(32, 16, true) T_(64, 32, true) T_(64, 64, true) T_(16, 16, true)
#undef T_
  return fail(NFA_ERR_INVALID, "learned preconditioner: no convolution kernel for this shape");
}

// data-gradient convolutions (direct gathers)
template <int CIN, int COUT, bool UPADD>
void conv_t(int D, int H, int W, const bf16_t* in, const bf16_t* in2, const DevBuf& frag, const float* bias,
            int relu, const bf16_t* mask, bf16_t* out, const SolveScalars* sc, hipStream_t s) {
  const long long waves = (long long)D * H * ((W + 15) / 16);
  k_conv<CIN, COUT, UPADD><<<(int)((waves + 3) / 4), 256, 0, s>>>(
      D, H, W, in, in2, reinterpret_cast<const uint4*>(frag.p), bias, relu, mask, out, sc);
}

nfa_status conv(int cin, int cout, bool upadd, int D, int H, int W, const bf16_t* in, const bf16_t* in2,
                const DevBuf& frag, const float* bias, int relu, const bf16_t* mask, bf16_t* out,
                const SolveScalars* sc, hipStream_t s) {
#define C_(A, B, U) \
  if (cin == A && cout == B && upadd == U) { conv_t<A, B, U>(D, H, W, in, in2, frag, bias, relu, mask, out, sc, s); return NFA_OK; }
  C_(16, 32, false) C_(32, 64, false) C_(64, 64, false) C_(32, 16, false) C_(64, 32, false) C_(16, 16, false)
#undef C_
  return fail(NFA_ERR_INVALID, "learned preconditioner: no data-gradient kernel for this shape");
}

template <int CIN, int COUT, bool UPADD>
void wgrad_t(UNet& u, float* gw, float* gb, int D, int H, int W, const bf16_t* in, const bf16_t* in2,
             const bf16_t* dout, hipStream_t s) {
  if constexpr (CIN == 2 && COUT == 16 && !UPADD) {
    static_assert((long long)kWgrad27Blocks * CIN * COUT <= (long long)kWgradBlocks * 64 * 64, "partials buffer");
    k_wgrad_c2<kWgrad27Blocks><<<kWgrad27Blocks, 256, 0, s>>>(D, H, W, in, dout, u.wpart.as<float>());
    k_wgrad_reduce<<<eblocks(27LL * CIN * COUT), kBlock, 0, s>>>(u.wpart.as<float>(), kWgrad27Blocks, CIN * COUT, gw);
  } else if constexpr ((COUT == 16 || COUT == 32) && (CIN == 16 || CIN == 32) && (CIN / 16) * (COUT / 16) <= 2) {
    // as many workgroups as the partials buffer takes (27 x 64 x 64 x 64 floats)
    constexpr int BLK = kWgrad27Blocks * 256 / (CIN * COUT) < kWgrad27Blocks ? kWgrad27Blocks * 256 / (CIN * COUT)
                                                                            : kWgrad27Blocks;
    static_assert((long long)BLK * CIN * COUT <= (long long)kWgradBlocks * 64 * 64, "partials buffer");
    k_wgrad27<CIN, COUT, UPADD><<<BLK, 256, 0, s>>>(D, H, W, in, in2, dout, u.wpart.as<float>());
    k_wgrad_reduce<<<eblocks(27LL * CIN * COUT), kBlock, 0, s>>>(u.wpart.as<float>(), BLK, CIN * COUT, gw);
  } else {
    dim3 grid(kWgradBlocks, 27);
    k_wgrad<CIN, COUT, UPADD><<<grid, 256, 0, s>>>(D, H, W, in, in2, dout, u.wpart.as<float>());
    k_wgrad_reduce<<<eblocks(27LL * CIN * COUT), kBlock, 0, s>>>(u.wpart.as<float>(), kWgradBlocks, CIN * COUT, gw);
  }
  const long long n = (long long)D * H * W;
  k_colsum<COUT><<<kColsumBlocks, 256, 0, s>>>(n, dout, u.cpart.as<float>());
  k_colsum_reduce<<<1, 256, 0, s>>>(u.cpart.as<float>(), kColsumBlocks, COUT, COUT, gb);
}

nfa_status wgrad(UNet& u, int layer, bool upadd, int level, const bf16_t* in, const bf16_t* in2,
                 const bf16_t* dout, hipStream_t s) {
  int D, H, W;
  u.dims(level, D, H, W);
  float* gw = u.grads.as<float>() + u.off_w[layer];
  float* gb = u.grads.as<float>() + u.off_b[layer];
  const int cin = u.cin[layer], cout = u.cout[layer];
#define W_(A, B, U) \
  if (cin == A && cout == B && upadd == U) { wgrad_t<A, B, U>(u, gw, gb, D, H, W, in, in2, dout, s); return NFA_OK; }
  W_(2, 16, false) W_(16, 32, false) W_(32, 64, false) W_(64, 64, false) W_(64, 32, false)
  W_(32, 16, true) W_(64, 32, true) W_(64, 64, true) W_(16, 16, true) W_(16, 16, false) W_(32, 16, false)
#undef W_
  return fail(NFA_ERR_INVALID, "learned preconditioner: no weight-gradient kernel for this shape");
}

void upT_mask(int C, int level_out, const UNet& u, const bf16_t* fine, const bf16_t* mask, bf16_t* coarse,
              hipStream_t s) {
  int D, H, W;
  u.dims(level_out, D, H, W);
  const long long n = (long long)D * H * W * (C / 8);
  if (C == 16) k_upT_mask<16><<<eblocks(n), kBlock, 0, s>>>(D, H, W, fine, mask, coarse);
  else if (C == 32) k_upT_mask<32><<<eblocks(n), kBlock, 0, s>>>(D, H, W, fine, mask, coarse);
  else k_upT_mask<64><<<eblocks(n), kBlock, 0, s>>>(D, H, W, fine, mask, coarse);
}

void skip_poolT_mask(int C, int level, const UNet& u, const bf16_t* skip, const bf16_t* coarse,
                     const bf16_t* mask, bf16_t* fine, hipStream_t s) {
  int D, H, W;
  u.dims(level, D, H, W);
  const long long n = (long long)D * H * W * (C / 8);
  if (C == 16) k_skip_poolT_mask<16><<<eblocks(n), kBlock, 0, s>>>(D, H, W, skip, coarse, mask, fine);
  else if (C == 32) k_skip_poolT_mask<32><<<eblocks(n), kBlock, 0, s>>>(D, H, W, skip, coarse, mask, fine);
  else k_skip_poolT_mask<64><<<eblocks(n), kBlock, 0, s>>>(D, H, W, skip, coarse, mask, fine);
}

#define B16(buf) (buf).as<bf16_t>()

// forward on the operator's grid; rr / nred give the residual scale.  keep:
// store every activation (training, export); otherwise only what a later
// layer reads: the pooled encoder outputs, the skips and the decoder outputs
// of the coarser levels.  The finest decoder's epilogue applies the head and
// writes z.
nfa_status forward(UNet& u, Poisson& op, const float* r, float* z, const double* rr, double nred,
                   const SolveScalars* sc, bool keep, hipStream_t s) {
  Grid& g = *op.g;
  if (g.nx != u.nx || g.ny != u.ny || g.nz != u.nz)
    return fail(NFA_ERR_INVALID, "learned preconditioner: network and operator grids differ");
  if (u.ell_op != (const void*)&op || u.ell_version != op.version) {
    k_ell<<<eblocks(u.npos[0]), kBlock, 0, s>>>(u.npos[0], op.rho.as<double>(), B16(u.ell));
    u.ell_op = &op;
    u.ell_version = op.version;
  }
  const int L = u.L;
  const float* P = u.params.as<float>();
  u.fwd_op = &op;
  u.fwd_version = op.version;
  u.fwd_params = u.param_version;
  u.fwd_kept = keep;
  TconvArgs a{};
  a.sc = sc;
  // first encoder: features formed while staging, pooled output
  u.dims(0, a.D, a.H, a.W);
  a.r = r;
  a.ell = B16(u.ell);
  a.rr = rr;
  a.nred = nred;
  a.x0 = keep ? B16(u.x0) : nullptr;
  a.frag = reinterpret_cast<const uint4*>(u.frag_t[0].p);
  a.bias = P + u.off_b[0];
  a.out = B16(u.a[0]);
  a.pooled = B16(u.p[0]);
  tconv_t<2, 16, false, true, 2>(a, s);
  a.ell = nullptr;
  a.x0 = nullptr;
  nfa_status e = NFA_OK;
  for (int l = 1; l < L && e == NFA_OK; ++l) {
    u.dims(l, a.D, a.H, a.W);
    a.in = B16(u.p[l - 1]);
    a.frag = reinterpret_cast<const uint4*>(u.frag_t[u.E(l)].p);
    a.bias = P + u.off_b[u.E(l)];
    a.out = B16(u.a[l]);
    a.pooled = l + 1 < L ? B16(u.p[l]) : nullptr;
    e = tconv(u.cin[u.E(l)], u.cout[u.E(l)], false, a, s);
  }
  if (e != NFA_OK) return e;
  u.dims(L - 1, a.D, a.H, a.W);
  a.in = B16(u.a[L - 1]);
  a.frag = reinterpret_cast<const uint4*>(u.frag_t[u.B()].p);
  a.bias = P + u.off_b[u.B()];
  a.out = B16(u.d[L - 1]);
  a.pooled = nullptr;
  if ((e = tconv(u.cin[u.B()], u.cout[u.B()], false, a, s)) != NFA_OK) return e;
  for (int l = L - 2; l >= 0 && e == NFA_OK; --l) {
    u.dims(l, a.D, a.H, a.W);
    a.in = B16(u.a[l]);
    a.in2 = B16(u.d[l + 1]);
    a.frag = reinterpret_cast<const uint4*>(u.frag_t[u.Dl(l)].p);
    a.bias = P + u.off_b[u.Dl(l)];
    a.out = (l > 0 || keep) ? B16(u.d[l]) : nullptr;
    if (l == 0) {   // the head on d0, fused into its epilogue
      a.z = z;
      a.wproj = u.head_w.as<float>();
      a.pbias = P + u.off_b[u.Hd()];
      a.dinv = op.dinv32.as<float>();
    }
    e = tconv(u.cin[u.Dl(l)], u.cout[u.Dl(l)], true, a, s);
  }
  if (e != NFA_OK) return e;
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

// gradients of all parameters from dL/dz, after a forward with keep
nfa_status backward(UNet& u, Poisson& op, const float* dz, hipStream_t s) {
  const int L = u.L;
  int D, H, W;
  u.dims(0, D, H, W);
  float* G = u.grads.as<float>();
  const float* dinv = op.dinv32.as<float>();
  const long long n0 = u.npos[0];
  // head (1 x 1 x 1) on d0: its gradient into d0's pre-activation; weights and
  // bias summed over positions against d0
  k_head_dgrad<<<eblocks(n0), kBlock, 0, s>>>(n0, dz, dinv, u.head_w.as<float>(), B16(u.d[0]),
                                              B16(u.dd[0]));
  k_head_wgrad<<<kHeadBlocks, 256, 0, s>>>(n0, dz, dinv, B16(u.d[0]), u.hpart.as<float>());
  k_head_wgrad_reduce<<<1, 64, 0, s>>>(u.hpart.as<float>(), kHeadBlocks, G + u.off_w[u.Hd()],
                                       G + u.off_b[u.Hd()]);
  // finest decoder: weights against up(d1) + a0, formed once into skip[0]
  // (free until the data gradient below writes it), then the data gradient
  // into skip[0]
  if (u.cin[u.Dl(0)] != 16 || level_channels(0) != 16)
    return fail(NFA_ERR_INVALID, "learned preconditioner: the finest decoder takes 16 channels");
  k_skipsum<16><<<eblocks(n0 * 2), kBlock, 0, s>>>(D, H, W, B16(u.a[0]), B16(u.d[1]), B16(u.skip[0]));
  nfa_status e = wgrad(u, u.Dl(0), false, 0, B16(u.skip[0]), nullptr, B16(u.dd[0]), s);
  if (e != NFA_OK) return e;
  e = conv(u.cout[u.Dl(0)], u.cin[u.Dl(0)], false, D, H, W, B16(u.dd[0]), nullptr, u.frag_b[u.Dl(0)], nullptr, 0,
           nullptr, B16(u.skip[0]), nullptr, s);
  if (e != NFA_OK) return e;
  // decoder, fine to coarse
  for (int l = 1; l <= L - 2 && e == NFA_OK; ++l) {
    const int ly = u.Dl(l);
    upT_mask(level_channels(l - 1), l, u, B16(u.skip[l - 1]), B16(u.d[l]), B16(u.dd[l]), s);
    if (u.cin[ly] == 32 && level_channels(l) == 32) {
      // the skip sum up(d_(l+1)) + a_l formed once into skip[l] (free until
      // the data gradient below writes it), then the weights against it
      int Dl, Hl, Wl;
      u.dims(l, Dl, Hl, Wl);
      k_skipsum<32><<<eblocks(u.npos[l] * 4), kBlock, 0, s>>>(Dl, Hl, Wl, B16(u.a[l]), B16(u.d[l + 1]), B16(u.skip[l]));
      e = wgrad(u, ly, false, l, B16(u.skip[l]), nullptr, B16(u.dd[l]), s);
    } else {
      e = wgrad(u, ly, true, l, B16(u.a[l]), B16(u.d[l + 1]), B16(u.dd[l]), s);
    }
    if (e != NFA_OK) break;
    u.dims(l, D, H, W);
    e = conv(u.cout[ly], u.cin[ly], false, D, H, W, B16(u.dd[l]), nullptr, u.frag_b[ly], nullptr, 0, nullptr,
             B16(u.skip[l]), nullptr, s);
  }
  if (e != NFA_OK) return e;
  // bottleneck
  upT_mask(level_channels(L - 2), L - 1, u, B16(u.skip[L - 2]), B16(u.d[L - 1]), B16(u.dd[L - 1]), s);
  e = wgrad(u, u.B(), false, L - 1, B16(u.a[L - 1]), nullptr, B16(u.dd[L - 1]), s);
  if (e != NFA_OK) return e;
  u.dims(L - 1, D, H, W);
  e = conv(u.cout[u.B()], u.cin[u.B()], false, D, H, W, B16(u.dd[L - 1]), nullptr, u.frag_b[u.B()], nullptr, 0,
           B16(u.a[L - 1]), B16(u.da[L - 1]), nullptr, s);
  // encoder, coarse to fine
  for (int l = L - 1; l >= 1 && e == NFA_OK; --l) {
    const int ly = u.E(l);
    e = wgrad(u, ly, false, l, B16(u.p[l - 1]), nullptr, B16(u.da[l]), s);
    if (e != NFA_OK) break;
    u.dims(l, D, H, W);
    e = conv(u.cout[ly], u.cin[ly], false, D, H, W, B16(u.da[l]), nullptr, u.frag_b[ly], nullptr, 0, nullptr,
             B16(u.dp[l - 1]), nullptr, s);
    if (e != NFA_OK) break;
    skip_poolT_mask(level_channels(l - 1), l - 1, u, B16(u.skip[l - 1]), B16(u.dp[l - 1]), B16(u.a[l - 1]),
                    B16(u.da[l - 1]), s);
  }
  if (e != NFA_OK) return e;
  e = wgrad(u, u.E(0), false, 0, B16(u.x0), nullptr, B16(u.da[0]), s);
  if (e != NFA_OK) return e;
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

nfa_status grad_step(UNet& u, Poisson& op, const float* r, double eAe, double* loss, hipStream_t s) {
  if (const nfa_status e = require_assembled(op, "learned preconditioner")) return e;
  if (!(eAe > 0)) return fail(NFA_ERR_INVALID, "learned preconditioner: eAe must be > 0");
  double* scal = u.scal.as<double>();
  double* parts = op.partials.as<double>();
  const long long n = u.npos[0];
  int nb = launch_dot<float>(r, r, n, parts, nullptr, s);
  launch_sum_partials(parts, nb, 1, scal, s);
  nfa_status e = forward(u, op, r, u.zt.as<float>(), scal, (double)op.g->n_reduced, nullptr, true, s);
  if (e != NFA_OK) return e;
  e = nfa_poisson_apply(&static_cast<nfa_poisson_s&>(op), u.zt.p, u.Az.p, NFA_F32, s);
  if (e != NFA_OK) return e;
  nb = launch_dot<float>(u.zt.as<float>(), r, n, parts, nullptr, s);
  launch_sum_partials(parts, nb, 1, scal + 1, s);
  nb = launch_dot<float>(u.zt.as<float>(), u.Az.as<float>(), n, parts, nullptr, s);
  launch_sum_partials(parts, nb, 1, scal + 2, s);
  k_loss_grad<<<eblocks(n), kBlock, 0, s>>>(n, r, u.Az.as<float>(), scal + 1, eAe, u.dz.as<float>());
  NFA_CHECK_LAUNCH();
  if ((e = backward(u, op, u.dz.as<float>(), s)) != NFA_OK) return e;
  double h[3];
  NFA_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s));
  NFA_HIP(hipStreamSynchronize(s));
  if (loss) *loss = 1.0 - h[1] * h[1] / (h[2] * eAe);
  if (!std::isfinite(h[1]) || !std::isfinite(h[2]) || !(h[2] > 0))
    return fail(NFA_ERR_NUMERIC, "learned preconditioner: non-finite loss");
  return NFA_OK;
}

}  // namespace

nfa_status unet_precond_apply(void* unet, Poisson& op, const float* r, float* z,
                              const SolveScalars* sc, hipStream_t s) {
  if (!unet) return fail(NFA_ERR_INVALID, "learned preconditioner: no network");
  UNet& u = *static_cast<nfa_unet_s*>(unet);
  return forward(u, op, r, z, &sc->rr, (double)op.g->n_reduced, sc, false, s);
}

}  // namespace nfa

using namespace nfa;

extern "C" long long nfa_unet_param_count(int levels) {
  if (levels < 3 || levels > kMaxLevels) return -1;
  return count_params(levels, nullptr, nullptr);
}

namespace nfa {
namespace {
nfa_status unet_check(int nx, int ny, int nz, int levels, const char* who) {
  if (levels < 3 || levels > kMaxLevels) return fail(NFA_ERR_INVALID, std::string(who) + ": levels must be in [3, 6]");
  const int q = 1 << (levels - 1);
  if (nx < q || ny < q || nz < q || nx % q || ny % q || nz % q)
    return fail(NFA_ERR_INVALID, std::string(who) + ": grid sizes must be multiples of 2^(levels-1)");
  // the kernels index channels-last arrays with 32-bit element offsets; the
  // largest is a 16-channel array over the fine grid
  if ((long long)nx * ny * nz * 16 >= (1LL << 32))
    return fail(NFA_ERR_INVALID, std::string(who) + ": at most 2^28 cells");
  return NFA_OK;
}

void unet_shape(UNet& u, int nx, int ny, int nz, int levels) {
  u.nx = nx;
  u.ny = ny;
  u.nz = nz;
  u.L = levels;
  for (int l = 0; l < levels; ++l) u.npos[l] = (long long)(nx >> l) * (ny >> l) * (nz >> l);
  layer_shapes(levels, u.cin, u.cout);
  u.nlayers = (int)u.cin.size();
  u.off_w.clear();
  u.off_b.clear();
  u.nparam = count_params(levels, &u.off_w, &u.off_b);
  u.frag_t.resize(u.nlayers);
  u.frag_b.resize(u.nlayers);
}

// Every device buffer of a network, in one fixed order: parameters, their
// gradients and Adam moments (FP32, nparam each), packed weight fragments,
// activations and their gradients (BF16), head terms and partial sums.
hipError_t unet_buffers(UNet& u, Carver& c) {
  hipError_t e = hipSuccess;
#define TAKE(buf, bytes) if ((e = c.take(u.buf, (size_t)(bytes))) != hipSuccess) return e
  TAKE(params, u.nparam * 4);
  TAKE(grads, u.nparam * 4);
  TAKE(adam_m, u.nparam * 4);
  TAKE(adam_v, u.nparam * 4);
  for (int l = 0; l < u.nlayers - 1; ++l) {
    TAKE(frag_t[l], tile_frag_bytes(u.cin[l], u.cout[l]));
    if (l > 0) TAKE(frag_b[l], (long long)((27 * u.cout[l] + 31) / 32) * (u.cin[l] / 16) * 64 * 16);
  }
  TAKE(head_w, 16 * 4);
  const long long n0 = u.npos[0];
  TAKE(ell, n0 * 2);
  TAKE(x0, n0 * 2 * 2);
  for (int l = 0; l < u.L; ++l) {
    const long long nl = u.npos[l];
    const int ch = level_channels(l);
    TAKE(a[l], nl * ch * 2);
    TAKE(da[l], nl * ch * 2);
    if (l + 1 < u.L) {
      TAKE(p[l], u.npos[l + 1] * ch * 2);
      TAKE(dp[l], u.npos[l + 1] * ch * 2);
      TAKE(skip[l], nl * ch * 2);
    }
    // decoder outputs: d_l has level l-1's channels, d_0 16
    const int cd = l >= 1 ? level_channels(l - 1) : 16;
    TAKE(d[l], nl * cd * 2);
    TAKE(dd[l], nl * cd * 2);
  }
  TAKE(zt, n0 * 4);
  TAKE(Az, n0 * 4);
  TAKE(dz, n0 * 4);
  TAKE(wpart, 27LL * kWgradBlocks * 64 * 64 * 4);
  TAKE(cpart, (long long)kColsumBlocks * 64 * 4);
  TAKE(hpart, (long long)kHeadBlocks * 17 * 4);
  TAKE(scal, 8 * 8);
#undef TAKE
  return hipSuccess;
}
}  // namespace
}  // namespace nfa

extern "C" size_t nfa_unet_workspace_bytes(int nx, int ny, int nz, int levels) {
  if (unet_check(nx, ny, nz, levels, "nfa_unet_workspace_bytes") != NFA_OK) return 0;
  UNet u;
  unet_shape(u, nx, ny, nz, levels);
  Carver c;
  c.measure = true;
  (void)unet_buffers(u, c);
  return c.used;
}

extern "C" nfa_status nfa_unet_create(int nx, int ny, int nz, int levels, int seed, void* workspace,
                                      size_t ws_bytes, nfa_unet* out) {
  if (!out) return fail(NFA_ERR_INVALID, "nfa_unet_create: out is NULL");
  *out = nullptr;
  if (const nfa_status e = unet_check(nx, ny, nz, levels, "nfa_unet_create")) return e;
  if (workspace) {
    const size_t need = nfa_unet_workspace_bytes(nx, ny, nz, levels);
    if (ws_bytes < need)
      return fail(NFA_ERR_NOMEM, "nfa_unet_create: workspace of " + std::to_string(ws_bytes) +
                                     " bytes, the network needs " + std::to_string(need));
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
      return fail(NFA_ERR_INVALID, "nfa_unet_create: workspace must be 256-byte aligned");
  }
  auto* u = new nfa_unet_s();
  unet_shape(*u, nx, ny, nz, levels);
  auto bad = [&](hipError_t e) {
    delete u;
    return fail(NFA_ERR_HIP, std::string("nfa_unet_create: ") + hipGetErrorString(e));
  };
  Carver c;
  c.base = static_cast<unsigned char*>(workspace);
  c.cap = ws_bytes;
  hipError_t e = unet_buffers(*u, c);
  if (e != hipSuccess) return bad(e);
  // He-normal initial weights, zero biases, head zero (the Jacobi step)
  std::vector<float> h(u->nparam, 0.0f);
  std::mt19937_64 rng((unsigned long long)seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int l = 0; l < u->nlayers - 1; ++l) {
    const double sd = std::sqrt(2.0 / (27.0 * u->cin[l]));
    for (long long i = 0; i < 27LL * u->cin[l] * u->cout[l]; ++i) h[u->off_w[l] + i] = (float)(nd(rng) * sd);
  }
  nfa_status st = nfa_unet_set_params(u, h.data());
  if (st != NFA_OK) {
    delete u;
    return st;
  }
  if ((e = hipMemset(u->adam_m.p, 0, u->nparam * 4)) != hipSuccess) return bad(e);
  if ((e = hipMemset(u->adam_v.p, 0, u->nparam * 4)) != hipSuccess) return bad(e);
  if ((e = hipMemset(u->grads.p, 0, u->nparam * 4)) != hipSuccess) return bad(e);
  if ((e = hipDeviceSynchronize()) != hipSuccess) return bad(e);
  *out = u;
  return NFA_OK;
}

extern "C" nfa_status nfa_unet_bind(nfa_unet u, float* params, float* grads, float* adam_m, float* adam_v,
                                    int copy) {
  if (!u || !params || !grads || !adam_m || !adam_v) return fail(NFA_ERR_INVALID, "nfa_unet_bind: NULL argument");
  float* dst[4] = {params, grads, adam_m, adam_v};
  DevBuf* src[4] = {&u->params, &u->grads, &u->adam_m, &u->adam_v};
  for (int i = 0; i < 4; ++i)
    for (int k = i + 1; k < 4; ++k)
      if (dst[i] == dst[k]) return fail(NFA_ERR_INVALID, "nfa_unet_bind: the four arrays must differ");
  const size_t bytes = (size_t)u->nparam * 4;
  NFA_HIP(hipDeviceSynchronize());
  for (int i = 0; i < 4; ++i) {
    if (copy && src[i]->p != dst[i]) NFA_HIP(hipMemcpy(dst[i], src[i]->p, bytes, hipMemcpyDeviceToDevice));
    src[i]->borrow(dst[i], bytes);
  }
  const nfa_status st = pack_all(*u, nullptr);
  if (st != NFA_OK) return st;
  NFA_HIP(hipDeviceSynchronize());
  return NFA_OK;
}

extern "C" int nfa_unet_levels(nfa_unet u) { return u ? u->L : -1; }

extern "C" nfa_status nfa_unet_set_params(nfa_unet u, const float* host) {
  if (!u || !host) return fail(NFA_ERR_INVALID, "nfa_unet_set_params: NULL argument");
  NFA_HIP(hipMemcpy(u->params.p, host, u->nparam * 4, hipMemcpyHostToDevice));
  nfa_status st = pack_all(*u, nullptr);
  if (st != NFA_OK) return st;
  NFA_HIP(hipDeviceSynchronize());
  return NFA_OK;
}

extern "C" nfa_status nfa_unet_get_params(nfa_unet u, float* host) {
  if (!u || !host) return fail(NFA_ERR_INVALID, "nfa_unet_get_params: NULL argument");
  NFA_HIP(hipDeviceSynchronize());
  NFA_HIP(hipMemcpy(host, u->params.p, u->nparam * 4, hipMemcpyDeviceToHost));
  return NFA_OK;
}

extern "C" nfa_status nfa_unet_get_grads(nfa_unet u, float* host) {
  if (!u || !host) return fail(NFA_ERR_INVALID, "nfa_unet_get_grads: NULL argument");
  NFA_HIP(hipDeviceSynchronize());
  NFA_HIP(hipMemcpy(host, u->grads.p, u->nparam * 4, hipMemcpyDeviceToHost));
  return NFA_OK;
}

extern "C" nfa_status nfa_unet_forward(nfa_unet u, nfa_poisson op, const float* r, float* z, int keep,
                                       nfa_stream s) {
  if (!u || !op || !r || !z) return fail(NFA_ERR_INVALID, "nfa_unet_forward: NULL argument");
  if ((reinterpret_cast<uintptr_t>(z) & 15) != 0)
    return fail(NFA_ERR_INVALID, "nfa_unet_forward: z must be 16-byte aligned");
  if (const nfa_status e = require_assembled(*op, "nfa_unet_forward")) return e;
  const hipStream_t st = S(s);
  double* parts = op->partials.as<double>();
  const int nb = launch_dot<float>(r, r, u->npos[0], parts, nullptr, st);
  launch_sum_partials(parts, nb, 1, u->scal.as<double>(), st);
  return forward(*u, *op, r, z, u->scal.as<double>(), (double)op->g->n_reduced, nullptr, keep != 0, st);
}

extern "C" nfa_status nfa_unet_grad(nfa_unet u, nfa_poisson op, const float* r, double eAe, double* loss,
                                    nfa_stream s) {
  if (!u || !op || !r) return fail(NFA_ERR_INVALID, "nfa_unet_grad: NULL argument");
  return grad_step(*u, *op, r, eAe, loss, S(s));
}

namespace nfa {
namespace {
nfa_status adam_step(UNet& u, float lr, float b1, float b2, float eps, int t, hipStream_t st) {
  const float bc1 = 1.0f - std::pow(b1, (float)t), bc2 = 1.0f - std::pow(b2, (float)t);
  k_adam<<<eblocks(u.nparam), kBlock, 0, st>>>(u.nparam, u.params.as<float>(), u.grads.as<float>(),
                                               u.adam_m.as<float>(), u.adam_v.as<float>(), lr, b1, b2, eps, bc1, bc2);
  NFA_CHECK_LAUNCH();
  return pack_all(u, st);
}
}  // namespace
}  // namespace nfa

extern "C" nfa_status nfa_unet_backward(nfa_unet u, nfa_poisson op, const float* dz, nfa_stream s) {
  if (!u || !op || !dz) return fail(NFA_ERR_INVALID, "nfa_unet_backward: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_unet_backward")) return e;
  if (!u->fwd_kept || u->fwd_op != (const void*)op || u->fwd_version != op->version ||
      u->fwd_params != u->param_version)
    return fail(NFA_ERR_INVALID,
                "nfa_unet_backward: needs a forward with keep = 1 on this operator, with the current parameters");
  return backward(*u, *op, dz, S(s));
}

extern "C" nfa_status nfa_unet_adam_step(nfa_unet u, float lr, float b1, float b2, float eps, int t, nfa_stream s) {
  if (!u || t < 1 || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(NFA_ERR_INVALID, "nfa_unet_adam_step: bad argument");
  return adam_step(*u, lr, b1, b2, eps, t, S(s));
}

extern "C" nfa_status nfa_unet_train_step(nfa_unet u, nfa_poisson op, const float* r, double eAe, float lr,
                                          int t, double* loss, nfa_stream s) {
  if (!u || !op || !r || t < 1) return fail(NFA_ERR_INVALID, "nfa_unet_train_step: bad argument");
  const hipStream_t st = S(s);
  nfa_status e = grad_step(*u, *op, r, eAe, loss, st);
  if (e != NFA_OK) return e;
  if ((e = adam_step(*u, lr, 0.9f, 0.999f, 1e-8f, t, st)) != NFA_OK) return e;
  NFA_HIP(hipStreamSynchronize(st));
  return NFA_OK;
}

extern "C" nfa_status nfa_unet_export(nfa_unet u, int what, void* dst, nfa_stream s) {
  if (!u || !dst) return fail(NFA_ERR_INVALID, "nfa_unet_export: NULL argument");
  const DevBuf* b = nullptr;
  if (what == NFA_UNET_X0) b = &u->x0;
  else if (what >= NFA_UNET_A && what < NFA_UNET_A + u->L) b = &u->a[what - NFA_UNET_A];
  else if (what >= NFA_UNET_P && what < NFA_UNET_P + u->L - 1) b = &u->p[what - NFA_UNET_P];
  else if (what >= NFA_UNET_D && what < NFA_UNET_D + u->L) b = &u->d[what - NFA_UNET_D];
  else if (what == NFA_UNET_DZ) b = &u->dz;
  else if (what >= NFA_UNET_DD && what < NFA_UNET_DD + u->L) b = &u->dd[what - NFA_UNET_DD];
  else if (what >= NFA_UNET_SKIP && what < NFA_UNET_SKIP + u->L - 1) b = &u->skip[what - NFA_UNET_SKIP];
  else if (what >= NFA_UNET_DA && what < NFA_UNET_DA + u->L) b = &u->da[what - NFA_UNET_DA];
  else if (what >= NFA_UNET_DP && what < NFA_UNET_DP + u->L - 1) b = &u->dp[what - NFA_UNET_DP];
  else return fail(NFA_ERR_INVALID, "nfa_unet_export: unknown item");
  NFA_HIP(hipMemcpyAsync(dst, b->p, b->bytes, hipMemcpyDeviceToDevice, S(s)));
  return NFA_OK;
}

extern "C" void nfa_unet_destroy(nfa_unet u) {
  if (!u) return;
  (void)hipDeviceSynchronize();
  delete u;
}
