// Learned coarse-flow proposal: a 6-layer 3x3 convolutional network that maps
// the stacked RGB pair to a 2-channel flow on the 1/8 grid (the seed grid of
// a 3-level hierarchy); its rounded output enters the seed step as one extra
// candidate, so the exact data term still decides every match.
//
// Layers (Cin, Cout, stride, dilation, ReLU): (6,32,2,1,y) (32,32,2,1,y)
// (32,32,2,1,y) (32,32,1,4,y) (32,32,1,8,y) (32,2,1,1,n); padding =
// dilation; flow in px = 32 * output.  Weights and activations are bf16,
// every product sum accumulates in fp32 on the matrix cores
// (gfx950's v_mfma_f32_16x16x32_bf16: 16 x 16 outputs, 32 products each);
// master weights and Adam state are fp32.
//
// All three convolutions are implicit GEMMs on 16x16x32 MFMA tiles:
//   forward        M = output pixels, N = Cout, K = 9 taps x Cin
//   backward-data  M = input pixels,  N = Cin,  K = 9 taps x Cout
//   backward-weight per tap: M = Cout, N = Cin, K = pixels, split over fixed
//                  pixel chunks and reduced in a fixed order (deterministic)
// Tensors are NHWC; Cin is padded to 8 (input) or 32 channels so that one
// lane's 8 consecutive K values are 8 contiguous channels of one tap (one
// 16-byte load).  Lane l of a 16x16x32 MFMA holds A[m = l % 16][k = 8 (l / 16)
// .. + 7], B[k = 8 (l / 16) .. + 7][n = l % 16] and D[m = 4 (l / 16) + i][n =
// l % 16], i = 0..3.  The forward and backward-data kernels stage the layer's
// packed weight fragments (at most 18 KB) in LDS once per workgroup; every
// wavefront then runs several 16-pixel tiles against them.
#include <math.h>

#include "ff_internal.h"

namespace ff {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetLayers = 6;
constexpr int kWChunks = 512;   // most backward-weight partials per layer
constexpr int kKStep = 32;      // K per MFMA
constexpr int kMaxKChunks = 9;  // 9 taps x 32 channels / 32
constexpr int kTilesPerWave = 4;   // 16-pixel tiles per wavefront (forward, backward-data)

struct NetLayer {
  int cin, cout, stride, dil, relu;
  int cinp, coutp;   // padded channel counts of the input / output tensors
};
static const NetLayer kNet[kNetLayers] = {{6, 32, 2, 1, 1, 8, 32},  {32, 32, 2, 1, 1, 32, 32},
                                          {32, 32, 2, 1, 1, 32, 32}, {32, 32, 1, 4, 1, 32, 32},
                                          {32, 32, 1, 8, 1, 32, 32}, {32, 2, 1, 1, 0, 32, 8}};

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

static int param_offset(int layer) {
  int o = 0;
  for (int l = 0; l < layer; ++l) o += kNet[l].cout * kNet[l].cin * 9 + kNet[l].cout;
  return o;
}
static int param_total() { return param_offset(kNetLayers); }
static int chunks_of(int cinp) { return (9 * cinp + kKStep - 1) / kKStep; }
static int tiles_of(int c) { return (c + 15) / 16; }

// ---------------------------------------------------------------- packing
// forward B fragments, one 16-byte fragment per (chunk, tile, lane):
// Wb[c][nt][g][n][i] = W[co = 16 nt + n][ci][tap] for K index
// k = 32 c + 8 g + i = tap * cinp + ci (zero where out of range)
__global__ void k_pack_fwd(const float* __restrict__ theta, int off, int cin, int cout, int cinp, int nchunks,
                           int ntiles, uint16_t* __restrict__ wb) {
  const int total = nchunks * ntiles * 64 * 8;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e & 7, n = (e >> 3) & 15, g = (e >> 7) & 3, rest = e >> 9;
    const int nt = rest % ntiles, c = rest / ntiles;
    const int k = kKStep * c + 8 * g + i;
    const int tap = k / cinp, ci = k % cinp, co = 16 * nt + n;
    float w = 0.f;
    if (tap < 9 && ci < cin && co < cout) w = theta[off + (co * cin + ci) * 9 + tap];
    wb[e] = f2bf(w);
  }
}

// backward-data B fragments: K index k = tap * coutp + co, N = ci
__global__ void k_pack_bwd(const float* __restrict__ theta, int off, int cin, int cout, int coutp, int nchunks,
                           int ntiles, uint16_t* __restrict__ wb) {
  const int total = nchunks * ntiles * 64 * 8;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e & 7, n = (e >> 3) & 15, g = (e >> 7) & 3, rest = e >> 9;
    const int nt = rest % ntiles, c = rest / ntiles;
    const int k = kKStep * c + 8 * g + i;
    const int tap = k / coutp, co = k % coutp, ci = 16 * nt + n;
    float w = 0.f;
    if (tap < 9 && co < cout && ci < cin) w = theta[off + (co * cin + ci) * 9 + tap];
    wb[e] = f2bf(w);
  }
}

// u8 RGB pair (B x H x W x 3 each) -> bf16 NHWC with 8 channels:
// RGB1/255 - 1/2, RGB2/255 - 1/2, 0, 0
__global__ void k_pack_input(const uint8_t* __restrict__ i1, const uint8_t* __restrict__ i2, size_t npx,
                             uint16_t* __restrict__ x) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (size_t)gridDim.x * blockDim.x) {
    uint16_t v[8];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = f2bf((float)i1[p * 3 + c] / 255.0f - 0.5f);
      v[3 + c] = f2bf((float)i2[p * 3 + c] / 255.0f - 0.5f);
    }
    v[6] = v[7] = 0;
    uint4 o;
    o.x = v[0] | ((uint32_t)v[1] << 16);
    o.y = v[2] | ((uint32_t)v[3] << 16);
    o.z = v[4] | ((uint32_t)v[5] << 16);
    o.w = v[6] | ((uint32_t)v[7] << 16);
    reinterpret_cast<uint4*>(x)[p] = o;
  }
}

// eight bf16 (16 bytes, 16-byte aligned) as an MFMA operand
__device__ __forceinline__ bf16x8 ld_bf16x8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 bf16x8_of(uint4 u) { return __builtin_bit_cast(bf16x8, u); }
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- forward
// One wavefront = kTilesPerWave tiles of 16 output pixels x NT*16 output
// channels, against the layer's weight fragments staged in LDS.  Epilogue
// adds the bias, applies ReLU and stores bf16 (or fp32 for the last layer).
template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, int Bn, int H, int W, int cinp,
                                                  int Ho, int Wo, int stride, int dil, int nchunks,
                                                  const uint4* __restrict__ wb, const float* __restrict__ bias,
                                                  int cout, int coutp, int relu, uint16_t* __restrict__ y,
                                                  float* __restrict__ yf) {
  __shared__ uint4 sW[kMaxKChunks * NT * 64];
  for (int e = threadIdx.x; e < nchunks * NT * 64; e += blockDim.x) sW[e] = wb[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t npx = (size_t)Bn * Ho * Wo;
  const int m = lane & 15, g = lane >> 4;
  for (int ti = 0; ti < kTilesPerWave; ++ti) {
    const size_t base = (((size_t)blockIdx.x * 4 + wave) * kTilesPerWave + ti) * 16;
    if (base >= npx) break;
    const size_t p = base + m;
    const bool pv = p < npx;
    const int ox = pv ? (int)(p % Wo) : 0;
    const int oy = pv ? (int)((p / Wo) % Ho) : 0;
    const int b = pv ? (int)(p / ((size_t)Wo * Ho)) : 0;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nchunks; ++c) {
      const int k0 = kKStep * c + 8 * g;
      const int tap = k0 / cinp, ci0 = k0 % cinp;
      uint4 av = make_uint4(0, 0, 0, 0);
      if (pv && tap < 9) {
        const int iy = oy * stride - dil + (tap / 3) * dil, ix = ox * stride - dil + (tap % 3) * dil;
        if (iy >= 0 && iy < H && ix >= 0 && ix < W)
          av = *reinterpret_cast<const uint4*>(x + (((size_t)b * H + iy) * W + ix) * cinp + ci0);
      }
      const bf16x8 a = bf16x8_of(av);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma32(a, bf16x8_of(sW[(c * NT + t) * 64 + lane]), acc[t]);
    }
    // D[row = 4 g + i][col = m]: pixel base + 4 g + i, channel 16 t + m
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = 16 * t + m;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const size_t q = base + 4 * g + i;
        if (q >= npx || co >= coutp) continue;
        float v = co < cout ? acc[t][i] + bias[co] : 0.f;
        if (relu) v = fmaxf(v, 0.f);
        if (yf) {
          if (co < cout) yf[q * cout + co] = v;
        } else {
          y[q * coutp + co] = f2bf(v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- backward-data
// dX[q][ci] = sum over taps and co of G[p(q, tap)][co] W[co][ci][tap], with
// p = ((y + dil - ky dil) / s, (x + dil - kx dil) / s) where divisible and
// inside; then the ReLU of the producing layer: stored gradient =
// dX * (Aprev > 0), bf16.  Tiles and LDS staging as in the forward kernel.
template <int NT>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const uint16_t* __restrict__ G, int Bn, int Ho, int Wo, int coutp,
                                                       int H, int W, int stride, int dil, int nchunks,
                                                       const uint4* __restrict__ wbt, int cinp,
                                                       const uint16_t* __restrict__ aprev, uint16_t* __restrict__ gprev) {
  __shared__ uint4 sW[kMaxKChunks * NT * 64];
  for (int e = threadIdx.x; e < nchunks * NT * 64; e += blockDim.x) sW[e] = wbt[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t npx = (size_t)Bn * H * W;
  const int m = lane & 15, g = lane >> 4;
  for (int ti = 0; ti < kTilesPerWave; ++ti) {
    const size_t base = (((size_t)blockIdx.x * 4 + wave) * kTilesPerWave + ti) * 16;
    if (base >= npx) break;
    const size_t q = base + m;
    const bool qv = q < npx;
    const int x = qv ? (int)(q % W) : 0;
    const int y = qv ? (int)((q / W) % H) : 0;
    const int b = qv ? (int)(q / ((size_t)W * H)) : 0;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nchunks; ++c) {
      const int k0 = kKStep * c + 8 * g;
      const int tap = k0 / coutp, co0 = k0 % coutp;
      uint4 av = make_uint4(0, 0, 0, 0);
      if (qv && tap < 9) {
        const int ty = y + dil - (tap / 3) * dil, tx = x + dil - (tap % 3) * dil;
        if (ty >= 0 && tx >= 0 && ty % stride == 0 && tx % stride == 0) {
          const int oy = ty / stride, ox = tx / stride;
          if (oy < Ho && ox < Wo) av = *reinterpret_cast<const uint4*>(G + (((size_t)b * Ho + oy) * Wo + ox) * coutp + co0);
        }
      }
      const bf16x8 a = bf16x8_of(av);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma32(a, bf16x8_of(sW[(c * NT + t) * 64 + lane]), acc[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int ci = 16 * t + m;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const size_t r = base + 4 * g + i;
        if (r >= npx || ci >= cinp) continue;
        const float mask = bf2f(aprev[r * cinp + ci]) > 0.f ? 1.f : 0.f;
        gprev[r * cinp + ci] = f2bf(acc[t][i] * mask);
      }
    }
  }
}

// ---------------------------------------------------------------- backward-weight
// Block = one fixed chunk of `chunk` output pixels (a multiple of 64, chosen
// per layer so that a launch has up to kWChunks blocks); for every tap:
// part[chunk][tap][co][ci] = sum_p G[p][co] X[p_in(p, tap)][ci] on MFMA
// (A = G^T from LDS, B = X_tap from LDS, K = pixels, 8 per lane), bias
// partial sum_p G[p][co].  Wave w handles taps w, w + 4, w + 8.  Staging
// reads 8 channels (16 bytes) per load and transposes them into
// channel-major LDS rows (pitch 72: rows start 16-byte aligned).
constexpr int kWPitch = 64 + 8;
__global__ __launch_bounds__(256) void k_conv_bwd_w(const uint16_t* __restrict__ G, int Bn, int Ho, int Wo, int coutp,
                                                    const uint16_t* __restrict__ X, int H, int W, int cinp, int stride,
                                                    int dil, int chunk, float* __restrict__ part,
                                                    float* __restrict__ partb) {
  __shared__ __align__(16) uint16_t sG[32][kWPitch];      // [co][pixel]
  __shared__ __align__(16) uint16_t sX[9][32][kWPitch];   // [tap][ci][pixel]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const size_t npx = (size_t)Bn * Ho * Wo;
  const size_t c0 = (size_t)blockIdx.x * chunk;
  const int MT = (coutp + 15) / 16, NTt = (cinp + 15) / 16;
  f32x4 acc[3][2][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) acc[a][b2][c2] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;   // thread t < coutp: bias partial of channel t
  __shared__ int sPix[64][3];   // b, oy, ox of the 64 staged output pixels
  // channel rows beyond the padded channel counts stay zero
  for (int e = threadIdx.x; e < 32 * kWPitch; e += 256) (&sG[0][0])[e] = 0;
  for (int e = threadIdx.x; e < 9 * 32 * kWPitch; e += 256) (&sX[0][0][0])[e] = 0;
  const int gq = coutp / 8, xq = cinp / 8;   // 16-byte quads per pixel
  for (size_t s0 = c0; s0 < c0 + chunk && s0 < npx; s0 += 64) {
    if (threadIdx.x < 64) {
      const size_t p = s0 + threadIdx.x;
      sPix[threadIdx.x][0] = p < npx ? (int)(p / ((size_t)Wo * Ho)) : -1;
      sPix[threadIdx.x][1] = (int)((p / Wo) % Ho);
      sPix[threadIdx.x][2] = (int)(p % Wo);
    }
    for (int e = threadIdx.x; e < 64 * gq; e += 256) {
      const int q = e % gq, px = e / gq;
      const size_t p = s0 + px;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (p < npx) v = reinterpret_cast<const uint4*>(G + p * coutp)[q];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) sG[8 * q + i][px] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 9 * 64 * xq; e += 256) {
      const int q = e % xq, px = (e / xq) & 63, tap = e / (64 * xq);
      const int b = sPix[px][0];
      uint4 v = make_uint4(0, 0, 0, 0);
      if (b >= 0) {
        const int iy = sPix[px][1] * stride - dil + (tap / 3) * dil, ix = sPix[px][2] * stride - dil + (tap % 3) * dil;
        if (iy >= 0 && iy < H && ix >= 0 && ix < W)
          v = reinterpret_cast<const uint4*>(X + (((size_t)b * H + iy) * W + ix) * cinp)[q];
      }
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) sX[tap][8 * q + i][px] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
    }
    __syncthreads();
    if ((int)threadIdx.x < coutp)
      for (int px = 0; px < 64; ++px) bsum += bf2f(sG[threadIdx.x][px]);
#pragma unroll
    for (int ks = 0; ks < 64 / kKStep; ++ks) {
      const int pk = kKStep * ks + 8 * g;   // this lane's 8 pixels
#pragma unroll
      for (int ti = 0; ti < 3; ++ti) {
        const int tap = wave + 4 * ti;
        if (tap >= 9) continue;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          if (mt >= MT) continue;
          const bf16x8 a = ld_bf16x8(&sG[16 * mt + m][pk]);
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            if (nt >= NTt) continue;
            acc[ti][mt][nt] = mfma32(a, ld_bf16x8(&sX[tap][16 * nt + m][pk]), acc[ti][mt][nt]);
          }
        }
      }
    }
    __syncthreads();
  }
  // D[row = co = 16 mt + 4 g + i][col = ci = 16 nt + m]
  float* pc = part + (size_t)blockIdx.x * 9 * 32 * 32;
#pragma unroll
  for (int ti = 0; ti < 3; ++ti) {
    const int tap = wave + 4 * ti;
    if (tap >= 9) continue;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = 16 * mt + 4 * g + i, ci = 16 * nt + m;
          pc[((size_t)tap * 32 + co) * 32 + ci] = (mt < MT && nt < NTt) ? acc[ti][mt][nt][i] : 0.f;
        }
  }
  if (threadIdx.x < 32) partb[(size_t)blockIdx.x * 32 + threadIdx.x] = (int)threadIdx.x < coutp ? bsum : 0.f;
}

// fixed-order reduction of the partials into the parameter-layout gradient:
// thread e owns partial slot e = (tap * 32 + co) * 32 + ci, so the threads
// of a wavefront read consecutive words of each chunk's partials
__global__ void k_reduce_w(const float* __restrict__ part, const float* __restrict__ partb, int nchunk, int cin,
                           int cout, int off, float* __restrict__ grad) {
  constexpr int kSlots = 9 * 32 * 32;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kSlots + 32; e += gridDim.x * blockDim.x) {
    if (e < kSlots) {
      const int ci = e % 32, co = (e / 32) % 32, tap = e / (32 * 32);
      if (ci >= cin || co >= cout) continue;
      float s = 0.f;
      for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * kSlots + e];
      grad[off + (co * cin + ci) * 9 + tap] = s;
    } else {
      const int co = e - kSlots;
      if (co >= cout) continue;
      float s = 0.f;
      for (int c = 0; c < nchunk; ++c) s += partb[(size_t)c * 32 + co];
      grad[off + cout * cin * 9 + co] = s;
    }
  }
}

// ---------------------------------------------------------------- loss
// masked L1 on the 1/8 grid: labels in 1/Q px (FF_EMPTY = none), output in
// px / 32.  Count first (integer atomics), then per-element gradient
// sign(out - t) / count into the bf16 gradient tensor (8 channels), and
// per-block loss partials summed in a fixed order.
__global__ void k_loss_count(const int32_t* __restrict__ labels, size_t n, int32_t* __restrict__ count) {
  int c = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    c += labels[i] != kEmpty;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void k_loss_grad(const float* __restrict__ out, const int32_t* __restrict__ labels, size_t n, float inv_q,
                            const int32_t* __restrict__ count, uint16_t* __restrict__ g6, float* __restrict__ lpart) {
  __shared__ float red[256];
  const float inv_n = 1.f / (float)max(*count, 1);
  float ls = 0.f;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t lb = labels[i];
    float gx = 0.f, gy = 0.f;
    if (lb != kEmpty) {
      const float tx = (float)fx_of(lb) * inv_q / 32.f, ty = (float)fy_of(lb) * inv_q / 32.f;
      const float dx = out[i * 2] - tx, dy = out[i * 2 + 1] - ty;
      ls = fabsf(dx) + fabsf(dy);
      gx = (dx > 0.f ? 1.f : (dx < 0.f ? -1.f : 0.f)) * inv_n;
      gy = (dy > 0.f ? 1.f : (dy < 0.f ? -1.f : 0.f)) * inv_n;
    }
    uint16_t* o = g6 + i * 8;
    o[0] = f2bf(gx);
    o[1] = f2bf(gy);
#pragma unroll
    for (int c = 2; c < 8; ++c) o[c] = 0;
  }
  red[threadIdx.x] = ls;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] * inv_n;
}

__global__ void k_sum_fixed(const float* __restrict__ v, int n, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += v[i];
    *out = s;
  }
}

// ---------------------------------------------------------------- Adam
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------- proposal
// round the network's flow to packed 1/Q px (nearest even), clamp to int16
__global__ void k_to_proposal(const float* __restrict__ out, size_t n, float q, int32_t* __restrict__ prop) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float fx = fminf(fmaxf(rintf(out[2 * i] * 32.f * q), -32767.f), 32767.f);
    const float fy = fminf(fmaxf(rintf(out[2 * i + 1] * 32.f * q), -32767.f), 32767.f);
    prop[i] = packf((int)fx, (int)fy);
  }
}

// ---------------------------------------------------------------- workspace plan
struct NetPlan {
  int H[kNetLayers + 1], W[kNetLayers + 1];   // tensor sizes: [0] input, [l+1] output of layer l
  size_t off_x[kNetLayers + 1];               // activations (bf16, padded channels); [6] = fp32 output
  size_t off_g[kNetLayers + 1];               // gradients w.r.t. pre-activation outputs (bf16)
  size_t off_wb[kNetLayers], off_wbt[kNetLayers];
  size_t off_grad, off_part, off_partb, off_lpart, off_count, off_loss;
  size_t part_chunks, lparts;
  size_t bytes;
};

static NetPlan net_plan(int Bn, int W, int H) {
  NetPlan P{};
  P.H[0] = H;
  P.W[0] = W;
  for (int l = 0; l < kNetLayers; ++l) {
    P.H[l + 1] = (P.H[l] + kNet[l].stride - 1) / kNet[l].stride;
    P.W[l + 1] = (P.W[l] + kNet[l].stride - 1) / kNet[l].stride;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += bytes;
    return o;
  };
  for (int l = 0; l <= kNetLayers; ++l) {
    const size_t px = (size_t)Bn * P.H[l] * P.W[l];
    const int ch = l == 0 ? 8 : kNet[l - 1].coutp;
    P.off_x[l] = take(l == kNetLayers ? px * 2 * 4 : px * ch * 2);
    P.off_g[l] = l == 0 ? 0 : take(px * (l == kNetLayers ? 8 : ch) * 2);
  }
  size_t maxpx = 0;
  for (int l = 0; l < kNetLayers; ++l) {
    P.off_wb[l] = take((size_t)chunks_of(kNet[l].cinp) * tiles_of(kNet[l].cout) * 64 * 16);
    P.off_wbt[l] = take((size_t)chunks_of(kNet[l].coutp) * tiles_of(kNet[l].cin) * 64 * 16);
    maxpx = std::max(maxpx, (size_t)Bn * P.H[l + 1] * P.W[l + 1]);
  }
  (void)maxpx;
  P.part_chunks = kWChunks;
  P.off_grad = take((size_t)param_total() * 4);
  P.off_part = take(P.part_chunks * 9 * 32 * 32 * 4);
  P.off_partb = take(P.part_chunks * 32 * 4);
  const size_t nout = (size_t)Bn * P.H[kNetLayers] * P.W[kNetLayers];
  P.lparts = (nout + 255) / 256;
  P.off_lpart = take(P.lparts * 4);
  P.off_count = take(4);
  P.off_loss = take(4);
  P.bytes = align_up(off, 256);
  return P;
}

static void enqueue_forward(const NetPlan& P, int Bn, const float* theta, const uint8_t* i1, const uint8_t* i2, char* ws,
                            hipStream_t s) {
  const size_t npx0 = (size_t)Bn * P.H[0] * P.W[0];
  k_pack_input<<<(unsigned)std::min<size_t>((npx0 + 255) / 256, 65535), 256, 0, s>>>(
      i1, i2, npx0, reinterpret_cast<uint16_t*>(ws + P.off_x[0]));
  for (int l = 0; l < kNetLayers; ++l) {
    const NetLayer& L = kNet[l];
    const int nch = chunks_of(L.cinp), nt = tiles_of(L.cout);
    uint16_t* wb = reinterpret_cast<uint16_t*>(ws + P.off_wb[l]);
    k_pack_fwd<<<64, 256, 0, s>>>(theta, param_offset(l), L.cin, L.cout, L.cinp, nch, nt, wb);
    const float* bias = theta + param_offset(l) + L.cout * L.cin * 9;
    const size_t npx = (size_t)Bn * P.H[l + 1] * P.W[l + 1];
    const unsigned blocks = (unsigned)((npx + 64 * kTilesPerWave - 1) / (64 * kTilesPerWave));
    const uint16_t* xin = reinterpret_cast<const uint16_t*>(ws + P.off_x[l]);
    uint16_t* yout = l + 1 < kNetLayers ? reinterpret_cast<uint16_t*>(ws + P.off_x[l + 1]) : nullptr;
    float* yf = l + 1 == kNetLayers ? reinterpret_cast<float*>(ws + P.off_x[l + 1]) : nullptr;
    const uint4* wbv = reinterpret_cast<const uint4*>(wb);
    if (nt == 2)
      k_conv_fwd<2><<<blocks, 256, 0, s>>>(xin, Bn, P.H[l], P.W[l], L.cinp, P.H[l + 1], P.W[l + 1], L.stride, L.dil, nch,
                                           wbv, bias, L.cout, L.coutp, L.relu, yout, yf);
    else
      k_conv_fwd<1><<<blocks, 256, 0, s>>>(xin, Bn, P.H[l], P.W[l], L.cinp, P.H[l + 1], P.W[l + 1], L.stride, L.dil, nch,
                                           wbv, bias, L.cout, L.coutp, L.relu, yout, yf);
  }
}

static ff_status check_net(int Bn, int W, int H) {
  if (Bn < 1 || Bn > 256 || W < 8 || H < 8 || W > kMaxDim || H > kMaxDim) return FF_ERR_ARG;
  if ((int64_t)Bn * W * H > (int64_t)1 << 30) return FF_ERR_SIZE;
  return FF_OK;
}

}  // namespace ff

using namespace ff;

extern "C" {

int32_t ff_net_param_count(void) { return param_total(); }

size_t ff_net_workspace_bytes(int32_t batch, int32_t width, int32_t height) {
  if (check_net(batch, width, height) != FF_OK) return 0;
  return net_plan(batch, width, height).bytes;
}

ff_status ff_proposal_forward(const float* params, const uint8_t* img1, const uint8_t* img2, int32_t batch,
                              int32_t width, int32_t height, int32_t subpel, int32_t* proposal, float* flow_out,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!params || !img1 || !img2 || !proposal || !workspace) return FF_ERR_ARG;
  if (subpel != 1 && subpel != 2 && subpel != 4 && subpel != 8) return FF_ERR_ARG;
  ff_status st = check_net(batch, width, height);
  if (st != FF_OK) return st;
  const NetPlan P = net_plan(batch, width, height);
  if (workspace_bytes < P.bytes) return FF_ERR_WORKSPACE;
  char* ws = static_cast<char*>(workspace);
  prof_mark(FF_PROF_PROPOSAL, stream, true);
  enqueue_forward(P, batch, params, img1, img2, ws, stream);
  const size_t n = (size_t)batch * P.H[kNetLayers] * P.W[kNetLayers];
  const float* out = reinterpret_cast<const float*>(ws + P.off_x[kNetLayers]);
  k_to_proposal<<<(unsigned)std::min<size_t>((n + 255) / 256, 65535), 256, 0, stream>>>(out, n, (float)subpel, proposal);
  prof_mark(FF_PROF_PROPOSAL, stream, false);
  if (flow_out && hipMemcpyAsync(flow_out, out, n * 2 * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return FF_ERR_HIP;
  return launch_status();
}

ff_status ff_proposal_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                                 const uint8_t* img1, const uint8_t* img2, const int32_t* labels, int32_t batch,
                                 int32_t width, int32_t height, int32_t subpel, float* grad_out, float* loss_out,
                                 void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!params || !img1 || !img2 || !labels || !workspace) return FF_ERR_ARG;
  if (subpel != 1 && subpel != 2 && subpel != 4 && subpel != 8) return FF_ERR_ARG;
  const bool update = adam_m && adam_v;
  if ((adam_m != nullptr) != (adam_v != nullptr) || (update && step < 1)) return FF_ERR_ARG;
  ff_status st = check_net(batch, width, height);
  if (st != FF_OK) return st;
  const NetPlan P = net_plan(batch, width, height);
  if (workspace_bytes < P.bytes) return FF_ERR_WORKSPACE;
  char* ws = static_cast<char*>(workspace);
  prof_mark(FF_PROF_TRAIN, stream, true);
  enqueue_forward(P, batch, params, img1, img2, ws, stream);
  // loss and dL/d(out)
  const size_t n6 = (size_t)batch * P.H[kNetLayers] * P.W[kNetLayers];
  int32_t* count = reinterpret_cast<int32_t*>(ws + P.off_count);
  float* lpart = reinterpret_cast<float*>(ws + P.off_lpart);
  fill_i32(count, 1, 0, stream);
  k_loss_count<<<(unsigned)std::min<size_t>((n6 + 255) / 256, 1024), 256, 0, stream>>>(labels, n6, count);
  k_loss_grad<<<(unsigned)P.lparts, 256, 0, stream>>>(reinterpret_cast<const float*>(ws + P.off_x[kNetLayers]), labels,
                                                     n6, 1.f / (float)subpel, count,
                                                     reinterpret_cast<uint16_t*>(ws + P.off_g[kNetLayers]), lpart);
  k_sum_fixed<<<1, 64, 0, stream>>>(lpart, (int)P.lparts, reinterpret_cast<float*>(ws + P.off_loss));
  // backward, last layer first
  float* grad = reinterpret_cast<float*>(ws + P.off_grad);
  float* part = reinterpret_cast<float*>(ws + P.off_part);
  float* partb = reinterpret_cast<float*>(ws + P.off_partb);
  for (int l = kNetLayers - 1; l >= 0; --l) {
    const NetLayer& L = kNet[l];
    const uint16_t* G = reinterpret_cast<const uint16_t*>(ws + P.off_g[l + 1]);
    const uint16_t* X = reinterpret_cast<const uint16_t*>(ws + P.off_x[l]);
    const int gch = l + 1 == kNetLayers ? 8 : L.coutp;
    const size_t npx = (size_t)batch * P.H[l + 1] * P.W[l + 1];
    // fixed chunking for a given size (run-to-run identical sums): chunks of
    // a multiple of 64 pixels, at most kWChunks of them
    const size_t chunk = std::max<size_t>(64, ((npx + kWChunks - 1) / kWChunks + 63) / 64 * 64);
    const int nchunk = (int)((npx + chunk - 1) / chunk);
    k_conv_bwd_w<<<nchunk, 256, 0, stream>>>(G, batch, P.H[l + 1], P.W[l + 1], gch, X, P.H[l], P.W[l], L.cinp, L.stride,
                                             L.dil, (int)chunk, part, partb);
    k_reduce_w<<<64, 256, 0, stream>>>(part, partb, nchunk, L.cin, L.cout, param_offset(l), grad);
    if (l > 0) {
      const int nchb = chunks_of(gch), ntb = tiles_of(L.cin);
      uint16_t* wbt = reinterpret_cast<uint16_t*>(ws + P.off_wbt[l]);
      k_pack_bwd<<<64, 256, 0, stream>>>(params, param_offset(l), L.cin, L.cout, gch, nchb, ntb, wbt);
      const size_t nin = (size_t)batch * P.H[l] * P.W[l];
      const unsigned blocks = (unsigned)((nin + 64 * kTilesPerWave - 1) / (64 * kTilesPerWave));
      uint16_t* gprev = reinterpret_cast<uint16_t*>(ws + P.off_g[l]);
      const uint16_t* aprev = X;
      const uint4* wbtv = reinterpret_cast<const uint4*>(wbt);
      if (ntb == 2)
        k_conv_bwd_data<2><<<blocks, 256, 0, stream>>>(G, batch, P.H[l + 1], P.W[l + 1], gch, P.H[l], P.W[l], L.stride,
                                                       L.dil, nchb, wbtv, L.cinp, aprev, gprev);
      else
        k_conv_bwd_data<1><<<blocks, 256, 0, stream>>>(G, batch, P.H[l + 1], P.W[l + 1], gch, P.H[l], P.W[l], L.stride,
                                                       L.dil, nchb, wbtv, L.cinp, aprev, gprev);
    }
  }
  const int np = param_total();
  if (update) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_adam<<<64, 256, 0, stream>>>(params, adam_m, adam_v, grad, np, lr, b1, b2, 1e-8f, c1, c2);
  }
  prof_mark(FF_PROF_TRAIN, stream, false);
  if (grad_out && hipMemcpyAsync(grad_out, grad, (size_t)np * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return FF_ERR_HIP;
  if (loss_out && hipMemcpyAsync(loss_out, ws + P.off_loss, 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return FF_ERR_HIP;
  return launch_status();
}

}  // extern "C"
