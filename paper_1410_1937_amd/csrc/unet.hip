// libnfa: learned preconditioner (3-D U-Net) for flexible CG.
//
// Convolutions are implicit GEMMs on the BF16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): for a 16-cell x-segment a
// wavefront computes out[channel][position] = W^T [channel][k] x in[k][position]
// with k = (tap, input channel), the weights pre-packed as per-lane A
// fragments and the input gathered as B fragments (8 consecutive channels of
// one tap per lane = one 16-byte load, channels-last activations).  The
// data gradient is the same kernel run on the flipped, transposed weights;
// the weight gradient is an MFMA GEMM over positions with per-workgroup
// partials summed in a fixed order.  The 16 -> 1 head and the elementwise
// glue (features, pooling, upsampling, ReLU masks, loss gradient, Adam) are
// plain vector kernels.  Activations are stored as BF16 (round to nearest
// even), exactly where the CPU oracle rounds.
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/nfa_unet.h"
#include "device_util.h"
#include "nfa_internal.h"
#include "vecops.h"

namespace nfa {
namespace {

typedef unsigned short bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double kL0 = -3.5, kL1 = 3.4;   // log(1/rho) normalisation
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

__global__ void k_prep(long long n, const float* __restrict__ r, const bf16_t* __restrict__ ell,
                       const double* __restrict__ rr, double nred, bf16_t* __restrict__ x0,
                       const SolveScalars* __restrict__ sc) {
  if (solve_done(sc)) return;
  const double ms = *rr / nred;
  const double inv = ms > 0 ? 1.0 / sqrt(ms) : 1.0;
  GRID_STRIDE(c, n) {
    x0[2 * c] = f2bf((float)((double)r[c] * inv));
    x0[2 * c + 1] = ell[c];
  }
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

// g[t][ci][co] = sum_blk partial[t][blk][ci][co] (fixed order)
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int nblk, int per_tap, float* __restrict__ g) {
  GRID_STRIDE(e, 27LL * per_tap) {
    const long long t = e / per_tap, k = e % per_tap;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(t * nblk + b) * per_tap + k];
    g[e] = (float)s;
  }
}

// column sums of dout [n][C] -> partial[blk][C]
template <int C>
__global__ __launch_bounds__(256) void k_colsum(long long n, const bf16_t* __restrict__ dout, float* __restrict__ partial) {
  __shared__ float red[256];
  const int ch = threadIdx.x % C, lanes = 256 / C, sub = threadIdx.x / C;
  float s = 0.f;
  for (long long m = (long long)blockIdx.x * lanes + sub; m < n; m += (long long)gridDim.x * lanes)
    s += bf2f(dout[m * C + ch]);
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < C) {
    float a = 0.f;
    for (int q = 0; q < lanes; ++q) a += red[q * C + threadIdx.x];
    partial[blockIdx.x * C + threadIdx.x] = a;
  }
}

// g[c] = sum_b partial[b*width + c] for c < C
__global__ void k_colsum_reduce(const float* __restrict__ partial, int nblk, int width, int C,
                                float* __restrict__ g) {
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b * width + c];
    g[c] = (float)s;
  }
}

// ------------------------------------------------------------ pooling / upsampling
// coarse[p][c] = bf16(sum of the 8 fine children / 8), 8 channels per thread
template <int C>
__global__ void k_pool(int Dc, int Hc, int Wc, const bf16_t* __restrict__ fine, bf16_t* __restrict__ coarse) {
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
    Frag o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o.h[j] = f2bf(s[j] * 0.125f);
    *reinterpret_cast<uint4*>(coarse + p * C + g * 8) = o.u;
  }
}

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

// ------------------------------------------------------------ head (16 -> 1)
// z = dinv * (x0[.,0] + b5 + sum_{t,ci} w5[t][ci] s0[p + off_t][ci]),  s0 = bf16(a0 + up(d1))
__global__ __launch_bounds__(256) void k_head_fwd(int D, int H, int W, const bf16_t* __restrict__ x0,
                                                  const bf16_t* __restrict__ a0,
                                                  const bf16_t* __restrict__ d1,
                                                  const float* __restrict__ w5, const float* __restrict__ b5,
                                                  const float* __restrict__ dinv, float* __restrict__ z,
                                                  const SolveScalars* __restrict__ sc) {
  if (solve_done(sc)) return;
  __shared__ float w[27 * 16];
  for (int e = threadIdx.x; e < 27 * 16; e += blockDim.x) w[e] = w5[e];
  __syncthreads();
  const long long n = (long long)D * H * W;
  const int H2 = H >> 1, W2 = W >> 1;
  GRID_STRIDE(p, n) {
    const int x = (int)(p % W);
    const long long r = p / W;
    const int y = (int)(r % H), zc = (int)(r / H);
    float u = b5[0];
    for (int t = 0; t < 27; ++t) {
      int dz, dy, dx;
      tap_offset(t, dz, dy, dx);
      const int zz = zc + dz, yy = y + dy, xx = x + dx;
      if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      const long long pp = ((long long)zz * H + yy) * W + xx;
      const long long qq = ((long long)(zz >> 1) * H2 + (yy >> 1)) * W2 + (xx >> 1);
      Frag a[2], b[2];
      a[0].u = *reinterpret_cast<const uint4*>(a0 + pp * 16);
      a[1].u = *reinterpret_cast<const uint4*>(a0 + pp * 16 + 8);
      b[0].u = *reinterpret_cast<const uint4*>(d1 + qq * 16);
      b[1].u = *reinterpret_cast<const uint4*>(d1 + qq * 16 + 8);
#pragma unroll
      for (int ci = 0; ci < 16; ++ci) {
        const float s = bf2f(f2bf(bf2f(a[ci >> 3].h[ci & 7]) + bf2f(b[ci >> 3].h[ci & 7])));
        u += w[t * 16 + ci] * s;
      }
    }
    z[p] = dinv[p] * (bf2f(x0[2 * p]) + u);
  }
}

// ds0[p][ci] = bf16(sum_t w5[t][ci] dy[p - off_t]),  dy = dinv * dz
__global__ __launch_bounds__(256) void k_head_bwd_data(int D, int H, int W, const float* __restrict__ dz,
                                                       const float* __restrict__ dinv,
                                                       const float* __restrict__ w5,
                                                       bf16_t* __restrict__ ds0) {
  __shared__ float w[27 * 16];
  for (int e = threadIdx.x; e < 27 * 16; e += blockDim.x) w[e] = w5[e];
  __syncthreads();
  const long long n = (long long)D * H * W;
  GRID_STRIDE(p, n) {
    const int x = (int)(p % W);
    const long long r = p / W;
    const int y = (int)(r % H), zc = (int)(r / H);
    float acc[16];
#pragma unroll
    for (int ci = 0; ci < 16; ++ci) acc[ci] = 0.f;
    for (int t = 0; t < 27; ++t) {
      int dz_, dy_, dx_;
      tap_offset(t, dz_, dy_, dx_);
      const int zz = zc - dz_, yy = y - dy_, xx = x - dx_;
      if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      const long long pp = ((long long)zz * H + yy) * W + xx;
      const float g = dinv[pp] * dz[pp];
#pragma unroll
      for (int ci = 0; ci < 16; ++ci) acc[ci] += w[t * 16 + ci] * g;
    }
    Frag o0, o1;
#pragma unroll
    for (int ci = 0; ci < 8; ++ci) {
      o0.h[ci] = f2bf(acc[ci]);
      o1.h[ci] = f2bf(acc[8 + ci]);
    }
    *reinterpret_cast<uint4*>(ds0 + p * 16) = o0.u;
    *reinterpret_cast<uint4*>(ds0 + p * 16 + 8) = o1.u;
  }
}

// the head's upstream gradient dy = dinv * dz as channel 0 of a 16-channel
// BF16 tensor, so that the weight gradient runs on the MFMA kernel
__global__ void k_pad_dy(long long n, const float* __restrict__ dz, const float* __restrict__ dinv,
                         bf16_t* __restrict__ out) {
  GRID_STRIDE(p, n) {
    Frag a, b;
    a.u = make_uint4(0u, 0u, 0u, 0u);
    b.u = make_uint4(0u, 0u, 0u, 0u);
    a.h[0] = f2bf(dinv[p] * dz[p]);
    *reinterpret_cast<uint4*>(out + p * 16) = a.u;
    *reinterpret_cast<uint4*>(out + p * 16 + 8) = b.u;
  }
}

// g[t*16 + ci] = full[t][ci][0]
__global__ void k_head_extract(const float* __restrict__ full, float* __restrict__ g) {
  for (int e = threadIdx.x; e < 27 * 16; e += blockDim.x) g[e] = full[e * 16];
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

// forward fragments: frag[(ks*MT+mt)*64 + lane][j] = W[k][co], k = ks*32 + (lane/16)*8 + j,
// co = mt*16 + lane%16 (0 beyond K)
__global__ void k_pack_fwd(const float* __restrict__ w, int cin, int cout, bf16_t* __restrict__ frag) {
  const int K = 27 * cin, KS = (K + 31) / 32, MT = cout / 16;
  GRID_STRIDE(e, (long long)KS * MT * 64 * 8) {
    const int j = (int)(e % 8);
    const long long f = e / 8;
    const int lane = (int)(f % 64);
    const long long km = f / 64;
    const int mt = (int)(km % MT), ks = (int)(km / MT);
    const int k = ks * 32 + (lane >> 4) * 8 + j, co = mt * 16 + (lane & 15);
    frag[e] = k < K ? f2bf(w[(long long)k * cout + co]) : (bf16_t)0;
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
  for (int e = threadIdx.x; e < 27 * 16; e += blockDim.x) wq[e] = bf2f(f2bf(w[e]));
}

}  // namespace

// ============================================================== host side
// Channels per level 16, 32, 64, 64, ...; convolutions in parameter order:
// encoder e_0..e_{L-1}, bottleneck b, decoder d_{L-2}..d_1, head (16 -> 1).
inline int level_channels(int l) { return l == 0 ? 16 : l == 1 ? 32 : 64; }

struct UNet {
  int nx = 0, ny = 0, nz = 0, L = 3;
  long long npos[kMaxLevels] = {0};
  int nlayers = 0;
  std::vector<int> cin, cout;
  std::vector<long long> off_w, off_b;
  long long nparam = 0;
  DevBuf params, grads, adam_m, adam_v;              // FP32, nparam
  std::vector<DevBuf> frag_f, frag_b;                // packed BF16 weight fragments
  DevBuf head_w;
  DevBuf x0, ell;
  DevBuf a[kMaxLevels], p[kMaxLevels], d[kMaxLevels];            // activations (BF16)
  DevBuf skip[kMaxLevels], dd[kMaxLevels], da[kMaxLevels], dp[kMaxLevels];  // gradients (BF16)
  DevBuf zt, Az, dz;                                 // FP32 cells
  DevBuf wpart, cpart, htmp, dypad;                  // FP32 partials, head scratch
  DevBuf scal;                                       // double: rr, a, c
  const void* ell_op = nullptr;
  int ell_version = -1;
  int E(int l) const { return l; }
  int B() const { return L; }
  int Dl(int l) const { return L + 1 + (L - 2 - l); }
  int Hd() const { return 2 * L - 1; }
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
  ci.push_back(16);
  co.push_back(1);
}

long long count_params(int L, std::vector<long long>* off_w, std::vector<long long>* off_b) {
  std::vector<int> ci, co;
  layer_shapes(L, ci, co);
  long long o = 0;
  for (size_t l = 0; l < ci.size(); ++l) {
    if (off_w) off_w->push_back(o);
    o += 27LL * ci[l] * co[l];
    if (off_b) off_b->push_back(o);
    o += co[l];
  }
  return o;
}

inline int eblocks(long long n) { return blocks_for(n, kBlock, 8192); }

nfa_status pack_all(UNet& u, hipStream_t s) {
  const float* P = u.params.as<float>();
  for (int l = 0; l < u.nlayers - 1; ++l) {
    const int cin = u.cin[l], cout = u.cout[l];
    const long long nf = (long long)((27 * cin + 31) / 32) * (cout / 16) * 64 * 8;
    k_pack_fwd<<<eblocks(nf), kBlock, 0, s>>>(P + u.off_w[l], cin, cout, u.frag_f[l].as<bf16_t>());
    if (l > 0) {
      const long long nb = (long long)((27 * cout + 31) / 32) * (cin / 16) * 64 * 8;
      k_pack_bwd<<<eblocks(nb), kBlock, 0, s>>>(P + u.off_w[l], cin, cout, u.frag_b[l].as<bf16_t>());
    }
  }
  k_pack_head<<<1, 512, 0, s>>>(P + u.off_w[u.Hd()], u.head_w.as<float>());
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

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
  C_(2, 16, false) C_(16, 32, false) C_(32, 64, false) C_(64, 64, false) C_(64, 32, false)
  C_(32, 16, false) C_(32, 16, true) C_(64, 32, true) C_(64, 64, true) C_(16, 32, false) C_(32, 64, true)
#undef C_
  return fail(NFA_ERR_INVALID, "learned preconditioner: no convolution kernel for this shape");
}

template <int CIN, int COUT, bool UPADD>
void wgrad_t(UNet& u, float* gw, float* gb, int D, int H, int W, const bf16_t* in, const bf16_t* in2,
             const bf16_t* dout, hipStream_t s) {
  dim3 grid(kWgradBlocks, 27);
  k_wgrad<CIN, COUT, UPADD><<<grid, 256, 0, s>>>(D, H, W, in, in2, dout, u.wpart.as<float>());
  k_wgrad_reduce<<<eblocks(27LL * CIN * COUT), kBlock, 0, s>>>(u.wpart.as<float>(), kWgradBlocks, CIN * COUT, gw);
  const long long n = (long long)D * H * W;
  k_colsum<COUT><<<kWgradBlocks, 256, 0, s>>>(n, dout, u.cpart.as<float>());
  k_colsum_reduce<<<1, 64, 0, s>>>(u.cpart.as<float>(), kWgradBlocks, COUT, COUT, gb);
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
  W_(32, 16, true) W_(64, 32, true) W_(64, 64, true)
#undef W_
  return fail(NFA_ERR_INVALID, "learned preconditioner: no weight-gradient kernel for this shape");
}

void pool(int C, int level_out, const UNet& u, const bf16_t* fine, bf16_t* coarse, hipStream_t s) {
  int D, H, W;
  u.dims(level_out, D, H, W);
  const long long n = (long long)D * H * W * (C / 8);
  if (C == 16) k_pool<16><<<eblocks(n), kBlock, 0, s>>>(D, H, W, fine, coarse);
  else if (C == 32) k_pool<32><<<eblocks(n), kBlock, 0, s>>>(D, H, W, fine, coarse);
  else k_pool<64><<<eblocks(n), kBlock, 0, s>>>(D, H, W, fine, coarse);
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

// forward on the operator's grid; rr / nred give the residual scale
nfa_status forward(UNet& u, Poisson& op, const float* r, float* z, const double* rr, double nred,
                   const SolveScalars* sc, hipStream_t s) {
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
  int D, H, W;
  k_prep<<<eblocks(u.npos[0]), kBlock, 0, s>>>(u.npos[0], r, B16(u.ell), rr, nred, B16(u.x0), sc);
  u.dims(0, D, H, W);
  nfa_status e = conv(2, 16, false, D, H, W, B16(u.x0), nullptr, u.frag_f[0], P + u.off_b[0], 1, nullptr,
                      B16(u.a[0]), sc, s);
  for (int l = 1; l < L && e == NFA_OK; ++l) {
    pool(level_channels(l - 1), l, u, B16(u.a[l - 1]), B16(u.p[l - 1]), s);
    u.dims(l, D, H, W);
    e = conv(u.cin[u.E(l)], u.cout[u.E(l)], false, D, H, W, B16(u.p[l - 1]), nullptr, u.frag_f[u.E(l)],
             P + u.off_b[u.E(l)], 1, nullptr, B16(u.a[l]), sc, s);
  }
  if (e != NFA_OK) return e;
  u.dims(L - 1, D, H, W);
  e = conv(u.cin[u.B()], u.cout[u.B()], false, D, H, W, B16(u.a[L - 1]), nullptr, u.frag_f[u.B()],
           P + u.off_b[u.B()], 1, nullptr, B16(u.d[L - 1]), sc, s);
  for (int l = L - 2; l >= 1 && e == NFA_OK; --l) {
    u.dims(l, D, H, W);
    e = conv(u.cin[u.Dl(l)], u.cout[u.Dl(l)], true, D, H, W, B16(u.a[l]), B16(u.d[l + 1]), u.frag_f[u.Dl(l)],
             P + u.off_b[u.Dl(l)], 1, nullptr, B16(u.d[l]), sc, s);
  }
  if (e != NFA_OK) return e;
  u.dims(0, D, H, W);
  k_head_fwd<<<eblocks(u.npos[0]), kBlock, 0, s>>>(D, H, W, B16(u.x0), B16(u.a[0]), B16(u.d[1]),
                                                   u.head_w.as<float>(), P + u.off_b[u.Hd()],
                                                   op.dinv32.as<float>(), z, sc);
  NFA_CHECK_LAUNCH();
  return NFA_OK;
}

// gradients of all parameters from dL/dz (in u.dz)
nfa_status backward(UNet& u, Poisson& op, hipStream_t s) {
  const int L = u.L;
  int D, H, W;
  u.dims(0, D, H, W);
  float* G = u.grads.as<float>();
  const float* dinv = op.dinv32.as<float>();
  const long long n0 = u.npos[0];
  // head: data gradient into skip[0], weights through the MFMA weight gradient
  // with dy = dinv*dz as channel 0 of a 16-channel tensor
  k_head_bwd_data<<<eblocks(n0), kBlock, 0, s>>>(D, H, W, u.dz.as<float>(), dinv, u.head_w.as<float>(),
                                                 B16(u.skip[0]));
  k_pad_dy<<<eblocks(n0), kBlock, 0, s>>>(n0, u.dz.as<float>(), dinv, B16(u.dypad));
  {
    dim3 grid(kWgradBlocks, 27);
    k_wgrad<16, 16, true><<<grid, 256, 0, s>>>(D, H, W, B16(u.a[0]), B16(u.d[1]), B16(u.dypad),
                                               u.wpart.as<float>());
    k_wgrad_reduce<<<eblocks(27LL * 256), kBlock, 0, s>>>(u.wpart.as<float>(), kWgradBlocks, 256,
                                                         u.htmp.as<float>());
    k_head_extract<<<1, 512, 0, s>>>(u.htmp.as<float>(), G + u.off_w[u.Hd()]);
    k_colsum<16><<<kWgradBlocks, 256, 0, s>>>(n0, B16(u.dypad), u.cpart.as<float>());
    k_colsum_reduce<<<1, 64, 0, s>>>(u.cpart.as<float>(), kWgradBlocks, 16, 1, G + u.off_b[u.Hd()]);
  }
  nfa_status e = NFA_OK;
  // decoder, fine to coarse
  for (int l = 1; l <= L - 2 && e == NFA_OK; ++l) {
    const int ly = u.Dl(l);
    upT_mask(level_channels(l - 1), l, u, B16(u.skip[l - 1]), B16(u.d[l]), B16(u.dd[l]), s);
    e = wgrad(u, ly, true, l, B16(u.a[l]), B16(u.d[l + 1]), B16(u.dd[l]), s);
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
  nfa_status e = forward(u, op, r, u.zt.as<float>(), scal, (double)op.g->n_reduced, nullptr, s);
  if (e != NFA_OK) return e;
  e = nfa_poisson_apply(&static_cast<nfa_poisson_s&>(op), u.zt.p, u.Az.p, NFA_F32, s);
  if (e != NFA_OK) return e;
  nb = launch_dot<float>(u.zt.as<float>(), r, n, parts, nullptr, s);
  launch_sum_partials(parts, nb, 1, scal + 1, s);
  nb = launch_dot<float>(u.zt.as<float>(), u.Az.as<float>(), n, parts, nullptr, s);
  launch_sum_partials(parts, nb, 1, scal + 2, s);
  k_loss_grad<<<eblocks(n), kBlock, 0, s>>>(n, r, u.Az.as<float>(), scal + 1, eAe, u.dz.as<float>());
  NFA_CHECK_LAUNCH();
  if ((e = backward(u, op, s)) != NFA_OK) return e;
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
  return forward(u, op, r, z, &sc->rr, (double)op.g->n_reduced, sc, s);
}

}  // namespace nfa

using namespace nfa;

extern "C" long long nfa_unet_param_count(int levels) {
  if (levels < 3 || levels > kMaxLevels) return -1;
  return count_params(levels, nullptr, nullptr);
}

extern "C" nfa_status nfa_unet_create(int nx, int ny, int nz, int levels, int seed, nfa_unet* out) {
  if (!out) return fail(NFA_ERR_INVALID, "nfa_unet_create: out is NULL");
  *out = nullptr;
  if (levels < 3 || levels > kMaxLevels) return fail(NFA_ERR_INVALID, "nfa_unet_create: levels must be in [3, 6]");
  const int q = 1 << (levels - 1);
  if (nx < q || ny < q || nz < q || nx % q || ny % q || nz % q)
    return fail(NFA_ERR_INVALID, "nfa_unet_create: grid sizes must be multiples of 2^(levels-1)");
  auto* u = new nfa_unet_s();
  u->nx = nx;
  u->ny = ny;
  u->nz = nz;
  u->L = levels;
  for (int l = 0; l < levels; ++l) u->npos[l] = (long long)(nx >> l) * (ny >> l) * (nz >> l);
  layer_shapes(levels, u->cin, u->cout);
  u->nlayers = (int)u->cin.size();
  u->nparam = count_params(levels, &u->off_w, &u->off_b);
  u->frag_f.resize(u->nlayers);
  u->frag_b.resize(u->nlayers);
  auto bad = [&](hipError_t e) {
    delete u;
    return fail(NFA_ERR_HIP, std::string("nfa_unet_create: ") + hipGetErrorString(e));
  };
  hipError_t e;
#define UALLOC(buf, bytes) if ((e = u->buf.alloc(bytes)) != hipSuccess) return bad(e)
  UALLOC(params, u->nparam * 4);
  UALLOC(grads, u->nparam * 4);
  UALLOC(adam_m, u->nparam * 4);
  UALLOC(adam_v, u->nparam * 4);
  for (int l = 0; l < u->nlayers - 1; ++l) {
    UALLOC(frag_f[l], (size_t)((27 * u->cin[l] + 31) / 32) * (u->cout[l] / 16) * 64 * 16);
    if (l > 0) UALLOC(frag_b[l], (size_t)((27 * u->cout[l] + 31) / 32) * (u->cin[l] / 16) * 64 * 16);
  }
  UALLOC(head_w, 27 * 16 * 4);
  const long long n0 = u->npos[0];
  UALLOC(ell, n0 * 2);
  UALLOC(x0, n0 * 2 * 2);
  for (int l = 0; l < levels; ++l) {
    const long long nl = u->npos[l];
    const int c = level_channels(l);
    UALLOC(a[l], nl * c * 2);
    UALLOC(da[l], nl * c * 2);
    if (l + 1 < levels) {
      UALLOC(p[l], u->npos[l + 1] * c * 2);
      UALLOC(dp[l], u->npos[l + 1] * c * 2);
      UALLOC(skip[l], nl * c * 2);
    }
    if (l >= 1) {
      UALLOC(d[l], nl * level_channels(l - 1) * 2);
      UALLOC(dd[l], nl * level_channels(l - 1) * 2);
    }
  }
  UALLOC(zt, n0 * 4);
  UALLOC(Az, n0 * 4);
  UALLOC(dz, n0 * 4);
  UALLOC(wpart, 27LL * kWgradBlocks * 64 * 64 * 4);
  UALLOC(cpart, (size_t)kWgradBlocks * 64 * 4);
  UALLOC(htmp, 27 * 256 * 4);
  UALLOC(dypad, n0 * 16 * 2);
  UALLOC(scal, 8 * 8);
#undef UALLOC
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

extern "C" nfa_status nfa_unet_forward(nfa_unet u, nfa_poisson op, const float* r, float* z, nfa_stream s) {
  if (!u || !op || !r || !z) return fail(NFA_ERR_INVALID, "nfa_unet_forward: NULL argument");
  if (const nfa_status e = require_assembled(*op, "nfa_unet_forward")) return e;
  const hipStream_t st = S(s);
  double* parts = op->partials.as<double>();
  const int nb = launch_dot<float>(r, r, u->npos[0], parts, nullptr, st);
  launch_sum_partials(parts, nb, 1, u->scal.as<double>(), st);
  return forward(*u, *op, r, z, u->scal.as<double>(), (double)op->g->n_reduced, nullptr, st);
}

extern "C" nfa_status nfa_unet_grad(nfa_unet u, nfa_poisson op, const float* r, double eAe, double* loss,
                                    nfa_stream s) {
  if (!u || !op || !r) return fail(NFA_ERR_INVALID, "nfa_unet_grad: NULL argument");
  return grad_step(*u, *op, r, eAe, loss, S(s));
}

extern "C" nfa_status nfa_unet_train_step(nfa_unet u, nfa_poisson op, const float* r, double eAe, float lr,
                                          int t, double* loss, nfa_stream s) {
  if (!u || !op || !r || t < 1) return fail(NFA_ERR_INVALID, "nfa_unet_train_step: bad argument");
  const hipStream_t st = S(s);
  nfa_status e = grad_step(*u, *op, r, eAe, loss, st);
  if (e != NFA_OK) return e;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.0f - std::pow(b1, (float)t), bc2 = 1.0f - std::pow(b2, (float)t);
  k_adam<<<eblocks(u->nparam), kBlock, 0, st>>>(u->nparam, u->params.as<float>(), u->grads.as<float>(),
                                                u->adam_m.as<float>(), u->adam_v.as<float>(), lr, b1, b2, 1e-8f,
                                                bc1, bc2);
  NFA_CHECK_LAUNCH();
  e = pack_all(*u, st);
  if (e != NFA_OK) return e;
  NFA_HIP(hipStreamSynchronize(st));
  return NFA_OK;
}

extern "C" nfa_status nfa_unet_export(nfa_unet u, int what, void* dst, nfa_stream s) {
  if (!u || !dst) return fail(NFA_ERR_INVALID, "nfa_unet_export: NULL argument");
  const DevBuf* b = nullptr;
  if (what == NFA_UNET_X0) b = &u->x0;
  else if (what >= NFA_UNET_A && what < NFA_UNET_A + u->L) b = &u->a[what - NFA_UNET_A];
  else if (what >= NFA_UNET_P && what < NFA_UNET_P + u->L - 1) b = &u->p[what - NFA_UNET_P];
  else if (what > NFA_UNET_D && what < NFA_UNET_D + u->L) b = &u->d[what - NFA_UNET_D];
  else return fail(NFA_ERR_INVALID, "nfa_unet_export: unknown item");
  NFA_HIP(hipMemcpyAsync(dst, b->p, b->bytes, hipMemcpyDeviceToDevice, S(s)));
  return NFA_OK;
}

extern "C" void nfa_unet_destroy(nfa_unet u) {
  if (!u) return;
  (void)hipDeviceSynchronize();
  delete u;
}
