// Per-image descriptors for the Flow Fields data term and kd-tree keys:
// 8-bit CIELab, the smoothed full-resolution images I^n, census planes per
// level and subpixel phase, and WHT patch vectors (sections 3.1-3.3).
//
// All kernels are streaming (HBM-bound): one thread per output pixel,
// row-major planes, coalesced along x.
#include <math.h>

#include <mutex>

#include "ff_internal.h"

namespace ff {

// ---------------------------------------------------------------- tables
// Section 3.3 computes the census in CIELab.  The conversion is integer:
// sRGB decode (IEC 61966-2-1) as a Q16 table, the sRGB->XYZ matrix with each
// row scaled to sum to exactly 2^14 (white -> (1,1,1), grays keep a = b = 0),
// the CIE cube-root compression with its linear toe as a Q15 table over Q16
// inputs.  L8 = round(2.55 L), a8/b8 = round(a/b) + 128, half up, clamped.
__device__ int32_t g_gamma[256];
__device__ int32_t g_mat[9];
__device__ uint16_t g_fcurve[65537];
// Section 3.2: Lanczos-3 upsampling weights, Q14, per scale n = 2,4,8,16
// (index log2 n - 1), phase x mod n, tap -3..3 around floor(x/n).
__constant__ int32_t c_lanczos[4][16][7];

// The tables are computed on the device, in fp64, by the kernels below (one
// thread per entry; a matrix row and a Lanczos phase each need their own sum,
// so they take one thread per row).  Every entry is at least 2.4e-6 away
// from a rounding tie, far more than the few ulps by which device and host
// fp64 functions may differ, so the rounded tables are exact.
__device__ int32_t g_lanczos_stage[4][16][7];   // copied to the constant table

__global__ void k_lab_tables() {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= 65536) {
    // CIE companding f over t in [0, 1] (Q16 in, Q15 out): a cube root above
    // delta^3, its tangent line through 4/29 below, delta = 6/29
    const double delta = 6.0 / 29.0, t = (double)i / 65536.0;
    const double f = t > delta * delta * delta ? cbrt(t) : t / (3.0 * delta * delta) + 4.0 / 29.0;
    g_fcurve[i] = (uint16_t)floor(32768.0 * f + 0.5);
  }
  if (i < 256) {
    // the sRGB transfer function inverted: 8-bit code -> linear, Q16
    const double e = (double)i / 255.0;
    const double lin = e > 0.04045 ? pow((e + 0.055) / 1.055, 2.4) : e / 12.92;
    g_gamma[i] = (int32_t)floor(65536.0 * lin + 0.5);
  }
  if (i < 3) {
    // linear sRGB -> XYZ (D65), each row divided by its sum (the white
    // point) and taken to Q14; the row's rounding residual goes to its
    // largest entry, so every row sums to exactly 2^14
    const double M[3][3] = {{0.4124564, 0.3575761, 0.1804375},
                            {0.2126729, 0.7151522, 0.0721750},
                            {0.0193339, 0.1191920, 0.9503041}};
    const double w = M[i][0] + M[i][1] + M[i][2];
    int32_t q[3];
    int top = 0;
    for (int j = 0; j < 3; ++j) {
      q[j] = (int32_t)floor(16384.0 * (M[i][j] / w) + 0.5);
      top = M[i][j] > M[i][top] ? j : top;
    }
    q[top] += 16384 - q[0] - q[1] - q[2];
    for (int j = 0; j < 3; ++j) g_mat[3 * i + j] = q[j];
  }
}

// Lanczos-3 weights (sinc(x) sinc(x / 3) on |x| < 3) for the upsampling of
// section 3.2, per scale n = 2 << li and phase ph < n: output pixel x of
// phase ph sits at u = (ph + 1/2) / n - 1/2 on the coarse grid, taps
// k = -3..3 around floor(x / n); Q14, the rounding residual on the centre tap
// (each phase sums to exactly 2^14).  One thread per (scale, phase).
__global__ void k_lanczos_table() {
  const int li = blockIdx.x, ph = threadIdx.x, n = 2 << li;
  if (ph >= 16) return;
  int32_t sum = 0;
  for (int k = -3; k <= 3; ++k) {
    int32_t wq = 0;
    if (ph < n) {
      const double x = (ph + 0.5) / n - 0.5 - k;
      double L = 1.0;
      if (x != 0.0) L = fabs(x) < 3.0 ? 3.0 * sinpi(x) * sinpi(x / 3.0) / (M_PI * M_PI * x * x) : 0.0;
      wq = (int32_t)floor(16384.0 * L + 0.5);
    }
    g_lanczos_stage[li][ph][k + 3] = wq;
    sum += wq;
  }
  if (ph < n) g_lanczos_stage[li][ph][3] += 16384 - sum;
}

static std::mutex g_init_mu;
static bool g_init_done[64];

ff_status ensure_init() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FF_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_init_done[dev]) return FF_OK;
  k_lab_tables<<<(65537 + 255) / 256, 256>>>();
  k_lanczos_table<<<4, 64>>>();
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return FF_ERR_HIP;
  void* stage = nullptr;
  if (hipGetSymbolAddress(&stage, HIP_SYMBOL(g_lanczos_stage)) != hipSuccess || !stage) return FF_ERR_HIP;
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_lanczos), stage, sizeof(g_lanczos_stage), 0, hipMemcpyDeviceToDevice) !=
      hipSuccess)
    return FF_ERR_HIP;
  if (hipDeviceSynchronize() != hipSuccess) return FF_ERR_HIP;
  g_init_done[dev] = true;
  return FF_OK;
}

ff_status launch_status() { return hipGetLastError() == hipSuccess ? FF_OK : FF_ERR_HIP; }

__global__ void k_fill_i32(int32_t* p, size_t n, int32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

void fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t s) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_i32<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
}

// ---------------------------------------------------------------- Lab8
__global__ void k_lab8(const uint8_t* __restrict__ img, int W, int H, int C, int stride, uint8_t* __restrict__ lab) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  const size_t N = (size_t)W * H;
  const uint8_t* px = img + (size_t)y * stride + (size_t)x * C;
  const size_t o = (size_t)y * W + x;
  if (C == 1) {
    lab[o] = px[0];
    return;
  }
  const int32_t lr = g_gamma[px[0]], lg = g_gamma[px[1]], lb = g_gamma[px[2]];
  int32_t f[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int32_t acc = g_mat[3 * i] * lr + g_mat[3 * i + 1] * lg + g_mat[3 * i + 2] * lb;
    f[i] = g_fcurve[(acc + 8192) >> 14];
  }
  // L = 116 fY - 16 scaled by 2.55: (2958 fY - 408 * 2^15) / (10 * 2^15), >= 0
  const int32_t L = (2958 * f[1] - 408 * 32768 + 163840) / 327680;
  const int32_t a = ((500 * (f[0] - f[1]) + 16384) >> 15) + 128;
  const int32_t b = ((200 * (f[1] - f[2]) + 16384) >> 15) + 128;
  lab[o] = (uint8_t)clampi(L, 0, 255);
  lab[N + o] = (uint8_t)clampi(a, 0, 255);
  lab[2 * N + o] = (uint8_t)clampi(b, 0, 255);
}

// ---------------------------------------------------------------- I^n
// Every level in three launches: (1) level 0 (Lab8 with 4 fractional bits)
// and the n x n block sums of the replicate-padded planes of every coarser
// level, (2) every level's horizontal Lanczos pass (coarse rows to
// full-resolution columns, rounded back to block-sum units), (3) every
// level's vertical pass (divided by 2^14 n^2, 4 fractional bits kept).  One
// thread per output element over the levels laid end to end; each level has
// its own block-sum and pass buffers in the scratch region.
constexpr int kMaxLevels = 5;   // k <= 4

struct SmoothPlan {
  int W, H, C, k;
  int Wc[kMaxLevels], Hc[kMaxLevels];
  int64_t end1[kMaxLevels];   // stage 1: level 0's C N samples, then each level's C Hc Wc block sums
  int64_t end2[kMaxLevels];   // stage 2: each level's C Hc W horizontal outputs (end2[0] = 0)
  int64_t offA[kMaxLevels], offT[kMaxLevels];   // int32 offsets of a level's buffers in the scratch
};

SmoothPlan smooth_plan(int W, int H, int C, int k) {
  SmoothPlan p{};
  p.W = W;
  p.H = H;
  p.C = C;
  p.k = k;
  const int64_t N = (int64_t)W * H;
  p.end1[0] = C * N;
  p.end2[0] = 0;
  int64_t off = 0;
  for (int l = 1; l <= k; ++l) {
    const int n = 1 << l;
    p.Wc[l] = (W + n - 1) / n;
    p.Hc[l] = (H + n - 1) / n;
    p.end1[l] = p.end1[l - 1] + (int64_t)C * p.Hc[l] * p.Wc[l];
    p.end2[l] = p.end2[l - 1] + (int64_t)C * p.Hc[l] * W;
    p.offA[l] = off;
    off += (int64_t)C * p.Hc[l] * p.Wc[l];
    p.offT[l] = off;
    off += (int64_t)C * p.Hc[l] * W;
  }
  return p;
}

// int32 words of scratch the smoothing needs
size_t smooth_scratch_words(int W, int H, int C, int k) {
  const SmoothPlan p = smooth_plan(W, H, C, k);
  return k == 0 ? 0 : (size_t)(p.offT[k] + (int64_t)C * p.Hc[k] * W);
}

__global__ void k_smooth_blocks(const uint8_t* __restrict__ J, SmoothPlan p, int16_t* __restrict__ S,
                                int32_t* __restrict__ scratch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.end1[p.k]) return;
  if (i < p.end1[0]) {
    S[i] = (int16_t)(16 * J[i]);
    return;
  }
  int l = 1;
  while (l < p.k && i >= p.end1[l]) ++l;
  const int64_t e = i - p.end1[l - 1];
  const int Wc = p.Wc[l], Hc = p.Hc[l], n = 1 << l, W = p.W, H = p.H;
  const int j = (int)(e % Wc);
  const int64_t r = e / Wc;
  const int ii = (int)(r % Hc), c = (int)(r / Hc);
  const uint8_t* P = J + (size_t)c * W * H;
  int32_t s = 0;
  for (int u = 0; u < n; ++u) {
    const uint8_t* row = P + (size_t)min(ii * n + u, H - 1) * W;
    for (int v = 0; v < n; ++v) s += row[min(j * n + v, W - 1)];
  }
  scratch[p.offA[l] + e] = s;
}

__global__ void k_smooth_h(SmoothPlan p, int32_t* __restrict__ scratch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.end2[p.k]) return;
  int l = 1;
  while (l < p.k && i >= p.end2[l]) ++l;
  const int64_t e = i - p.end2[l - 1];
  const int Wc = p.Wc[l], Hc = p.Hc[l], n = 1 << l, W = p.W;
  const int x = (int)(e % W);
  const int64_t rc = e / W;   // c Hc + i
  (void)Hc;
  const int32_t* row = scratch + p.offA[l] + rc * Wc;
  const int ph = x % n, base = x / n;
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) s += c_lanczos[l - 1][ph][k] * row[clampi(base + k - 3, 0, Wc - 1)];
  scratch[p.offT[l] + e] = (s + 8192) >> 14;
}

__global__ void k_smooth_v(SmoothPlan p, const int32_t* __restrict__ scratch, int16_t* __restrict__ S) {
  const int64_t N = (int64_t)p.W * p.H, CN = p.C * N;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.k * CN) return;
  const int l = 1 + (int)(i / CN);
  const int64_t e = i - (l - 1) * CN;
  const int Hc = p.Hc[l], n = 1 << l, W = p.W, H = p.H;
  const int x = (int)(e % W);
  const int64_t r = e / W;
  const int y = (int)(r % H), c = (int)(r / H);
  const int32_t* P = scratch + p.offT[l] + (int64_t)c * Hc * W;
  const int ph = y % n, base = y / n;
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) s += c_lanczos[l - 1][ph][k] * P[(size_t)clampi(base + k - 3, 0, Hc - 1) * W + x];
  const int shift = 14 + 2 * l - 4;
  S[l * CN + e] = (int16_t)((s + (1 << (shift - 1))) >> shift);
}

// ---------------------------------------------------------------- census
// Every level in one launch (grid z = level).  A workgroup owns a 32 x 32
// tile of output pixels, a thread four of them (one column, rows 8 apart).
// The smoothed input of the tile grown by n + 1 (clamped to the image) is
// staged in LDS for every channel.
//
// A census bit compares the bilinear phase-(a, b) interpolant at a
// neighbour with the one at the centre; by linearity their difference is the
// interpolant of the four corner differences D = s(neighbour) - s(centre),
//   d(a, b) = (Q - b) ((Q - a) D00 + a D01) + b ((Q - a) D10 + a D11),
// the same integers as interpolating each point first.  Along a it grows by
// (Q - b)(D01 - D00) + b (D11 - D10), and that step and d(0, b) grow
// linearly in b, so a neighbour's Q^2 differences cost one add each.  The
// bit is the sign of d (|d| < 2^20): v_alignbit shifts it into the word, the
// neighbours taken from the last bit to the first, so the word reads bit
// 8c + i = neighbour i (raster order without the centre) of channel c.
//
// Each word is stored twice: row-major straight from the thread (a row of
// 32 words is one 128-byte line), and transposed (plane[x][y]) through an
// LDS buffer, so that a column of 32 words is one line as well.
constexpr int kCensusTile = 32;
constexpr int kCensusPB = 16;                // phases held in registers at once
constexpr int kCensusTP = 4;                 // phases per LDS transposition round

// One channel's comparison bits for the thread's four pixels and the PB
// phases from row b0 on.  INTERIOR: the tile grown by n + 1 lies inside the
// image, so every tap is the centre plus n (dy LW + dx) and no sample is
// clamped.
template <int Q, int PB, bool INTERIOR>
__device__ __forceinline__ void census_channel(const int16_t* __restrict__ T, int LW, int n, int W, int H, int sx0,
                                               int sy0, int xc, int ybase, int b0, uint32_t (&acc)[4][PB]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int yc = INTERIOR ? ybase + 8 * k : min(ybase + 8 * k, H - 1);
    // the four samples at tap (dx, dy): (X, Y), (X + 1, Y), (X, Y + 1),
    // (X + 1, Y + 1), clamped to the image as the smoothed images are
    auto corners = [&](int dx, int dy, int32_t& s00, int32_t& s01, int32_t& s10, int32_t& s11) {
      int o, ox, oy;
      if (INTERIOR) {
        o = (yc - sy0) * LW + (xc - sx0) + n * (dy * LW + dx);
        ox = 1;
        oy = LW;
      } else {
        const int X = clampi(xc + n * dx, 0, W - 1), Y = clampi(yc + n * dy, 0, H - 1);
        o = (Y - sy0) * LW + (X - sx0);
        ox = X + 1 <= W - 1 ? 1 : 0;
        oy = Y + 1 <= H - 1 ? LW : 0;
      }
      s00 = T[o];
      s01 = T[o + ox];
      s10 = T[o + oy];
      s11 = T[o + oy + ox];
    };
    int32_t c00, c01, c10, c11;
    corners(0, 0, c00, c01, c10, c11);
    // neighbours from the last bit to the first (a rolled loop keeps the
    // four pixels' corner reads from being hoisted into registers at once)
#pragma unroll 1
    for (int i = 7; i >= 0; --i) {
      const int t = i < 4 ? i : i + 1;
      int32_t s00, s01, s10, s11;
      corners(t % 3 - 1, t / 3 - 1, s00, s01, s10, s11);
      const int32_t D00 = s00 - c00, D01 = s01 - c01, D10 = s10 - c10, D11 = s11 - c11;
      const int32_t E = (D11 - D10) - (D01 - D00);
      // at b = b0: d(0, b) and the step along a
      int32_t d0 = Q * ((Q - b0) * D00 + b0 * D10);
      int32_t st = (Q - b0) * (D01 - D00) + b0 * (D11 - D10);
#pragma unroll
      for (int bb = 0; bb < PB / Q; ++bb) {
        int32_t d = d0;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          acc[k][bb * Q + a] = __builtin_amdgcn_alignbit(acc[k][bb * Q + a], (uint32_t)d, 31);
          d += st;
        }
        d0 += Q * (D10 - D00);
        st += E;
      }
    }
  }
}

// The tile's words for every phase block: the bits of each channel, then
// the row-major and the transposed stores.  One instance per kind of tile, so
// that the two never share a register allocation.
template <int Q, bool INTERIOR, int TP, int PB>
__device__ __forceinline__ void census_tile_impl(const int16_t* tileS, int plane,
                                                 uint32_t (*tbuf)[kCensusTile][kCensusTile + 1], int W, int H, int C,
                                                 int n, int x0, int y0, int sx0, int sy0, int LW, uint32_t* rm,
                                                 uint32_t* tr) {
  constexpr int QQ = Q * Q;
  const size_t N = (size_t)W * H;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x = x0 + tx, xc = min(x, W - 1);
  for (int pb = 0; pb < QQ; pb += PB) {
    const int b0 = pb / Q;
    uint32_t acc[4][PB];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int ph = 0; ph < PB; ++ph) acc[k][ph] = 0;
    for (int c = C - 1; c >= 0; --c) {
      census_channel<Q, PB, INTERIOR>(tileS + c * plane, LW, n, W, H, sx0, sy0, xc, y0 + ty, b0, acc);
    }
    // row-major words
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int y = y0 + ty + 8 * k;
      if (x < W && y < H) {
#pragma unroll
        for (int ph = 0; ph < PB; ++ph) rm[(size_t)(pb + ph) * N + (size_t)y * W + x] = acc[k][ph];
      }
    }
    // transposed words: TP phases per round through LDS, read back with the
    // lane on y
#pragma unroll
    for (int r = 0; r < PB / TP; ++r) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < TP; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) tbuf[j][tx][ty + 8 * k] = acc[k][r * TP + j];
      __syncthreads();
      const int yt = y0 + tx;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int xt = x0 + ty + 8 * k;
        if (xt < W && yt < H) {
#pragma unroll
          for (int j = 0; j < TP; ++j)
            tr[(size_t)(pb + r * TP + j) * N + (size_t)xt * H + yt] = tbuf[j][ty + 8 * k][tx];
        }
      }
    }
  }
}

template <int Q, bool INTERIOR>
__device__ __forceinline__ void census_tile(const int16_t* tileS, int plane,
                                            uint32_t (*tbuf)[kCensusTile][kCensusTile + 1], int W, int H, int C,
                                            int n, int x0, int y0, int sx0, int sy0, int LW, uint32_t* rm,
                                            uint32_t* tr) {
  constexpr int QQ = Q * Q, PB = QQ < kCensusPB ? QQ : kCensusPB, TP = PB < kCensusTP ? PB : kCensusTP;
  census_tile_impl<Q, INTERIOR, TP, PB>(tileS, plane, tbuf, W, H, C, n, x0, y0, sx0, sy0, LW, rm, tr);
}

template <int Q>
__global__ __launch_bounds__(256) void k_census(const int16_t* __restrict__ Sall, int W, int H, int C, int plane,
                                                uint32_t* __restrict__ outRM, uint32_t* __restrict__ outT) {
  constexpr int QQ = Q * Q, PB = QQ < kCensusPB ? QQ : kCensusPB, TP = PB < kCensusTP ? PB : kCensusTP;
  static_assert(QQ % PB == 0 && PB % TP == 0 && PB % Q == 0, "phase blocks");
  // the staged windows, C of them, LWmax^2 int16 each (sized by the
  // launch for the descriptor's coarsest level)
  extern __shared__ __align__(16) int16_t census_lds[];
  __shared__ uint32_t tbuf[TP][kCensusTile][kCensusTile + 1];
  const int lev = blockIdx.z, n = 1 << lev;
  const size_t N = (size_t)W * H;
  const int16_t* S = Sall + (size_t)lev * C * N;
  uint32_t* rm = outRM + (size_t)lev * QQ * N;
  uint32_t* tr = outT + (size_t)lev * QQ * N;
  const int x0 = blockIdx.x * kCensusTile, y0 = blockIdx.y * kCensusTile;
  const int sx0 = max(x0 - n, 0), sx1 = min(x0 + kCensusTile + n, W - 1);
  const int sy0 = max(y0 - n, 0), sy1 = min(y0 + kCensusTile + n, H - 1);
  const int LW = sx1 - sx0 + 1, LH = sy1 - sy0 + 1;
  const bool interior = x0 >= n && x0 + kCensusTile + n <= W - 1 && y0 >= n && y0 + kCensusTile + n <= H - 1;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // stage the window of every channel: rows over the 8 row groups, columns
  // over the 32 lanes
  for (int r = ty; r < C * LH; r += 8) {
    const int c = r / LH, yy = r - c * LH;
    const int16_t* src = S + (size_t)c * N + (size_t)(sy0 + yy) * W + sx0;
    for (int xx = tx; xx < LW; xx += 32) census_lds[c * plane + yy * LW + xx] = src[xx];
  }
  __syncthreads();
  if (interior) census_tile<Q, true>(census_lds, plane, tbuf, W, H, C, n, x0, y0, sx0, sy0, LW, rm, tr);
  else census_tile<Q, false>(census_lds, plane, tbuf, W, H, C, n, x0, y0, sx0, sy0, LW, rm, tr);
}

// ---------------------------------------------------------------- WHT
// The three 1-D Walsh functions on [-rho, rho] in sequency order are
// piecewise constant on four runs: A = [-rho, -rho + rho/2), B = [.., -1],
// Cs = [0, (rho+1)/2), D = [(rho+1)/2, rho] (an odd extent splits rho |
// rho + 1, the second split puts the smaller part first), so with the run
// sums  w0 = A + B + Cs + D,  w1 = A + B - Cs - D,  w2 = A - B - Cs + D.
// The 2-D basis (u on dy, v on dx) is taken in the order (0,0) (0,1) (1,0)
// (1,1) (0,2) (2,0) (1,2) (2,1) (2,2), per channel; samples are clamped to
// the image.
//
// One launch per radius.  A workgroup owns a 32 x 16 tile:
// its Lab8 window (grown by rho, clamped) goes to LDS, the three horizontal
// run combinations of every window row and tile column to LDS as int16
// (|w| <= (2 rho + 1) 255), and each thread combines vertical runs of those
// into the 9 C values of its pixels, written as one 128-byte row per pixel.
constexpr int kWhtTW = 32, kWhtTH = 16;         // 64-wide tiles measured 19 % slower (half the workgroups)
constexpr int kWhtG = 256 / kWhtTW;            // thread groups (one per tile column set)
constexpr int kWhtRPT = kWhtTH / kWhtG;        // output rows per thread

__host__ __device__ constexpr int wht_rows(int rho) { return kWhtTH + 2 * rho; }
__host__ __device__ constexpr int wht_cols(int rho) { return kWhtTW + 2 * rho; }

size_t wht_lds_bytes(int C, int rho) {
  return align_up((size_t)C * wht_rows(rho) * wht_cols(rho), 16) + (size_t)C * 3 * wht_rows(rho) * kWhtTW * 2;
}

template <int RHO>
__device__ __forceinline__ void wht_tile(const uint8_t* __restrict__ J, int W, int H, int C, int stride,
                                         int32_t* __restrict__ V) {
  constexpr int R = wht_rows(RHO), CW = wht_cols(RHO);
  constexpr int a1 = RHO / 2, m = RHO, c1 = (RHO + 1) / 2;
  extern __shared__ __align__(16) unsigned char wht_lds[];
  const size_t N = (size_t)W * H;
  const int x0 = blockIdx.x * kWhtTW, y0 = blockIdx.y * kWhtTH;
  uint8_t* jt = wht_lds;                                                                  // [C][R][CW]
  int16_t* hb = reinterpret_cast<int16_t*>(wht_lds + (((size_t)C * R * CW + 15) & ~(size_t)15));   // [C][3][R][64]
  const int lane = threadIdx.x % kWhtTW, grp = threadIdx.x / kWhtTW;
  for (int r = grp; r < C * R; r += kWhtG) {
    const int c = r / R, yy = r - c * R;
    const uint8_t* src = J + (size_t)c * N + (size_t)clampi(y0 - RHO + yy, 0, H - 1) * W;
    for (int xx = lane; xx < CW; xx += kWhtTW) jt[r * CW + xx] = src[clampi(x0 - RHO + xx, 0, W - 1)];
  }
  __syncthreads();
  // horizontal runs of every window row: a task is kWhtHS consecutive tile
  // columns of one row, summed at its first column and slid one column at a
  // time (each run loses its first sample and gains the one after its last)
  constexpr int kWhtHS = 4, kSegs = kWhtTW / kWhtHS;
  for (int task = threadIdx.x; task < C * R * kSegs; task += 256) {
    const int r = task / kSegs, x0s = (task - r * kSegs) * kWhtHS;
    const uint8_t* row = jt + r * CW + x0s;
    int32_t A = 0, B = 0, Cs = 0, D = 0;
#pragma unroll
    for (int k = 0; k <= 2 * RHO; ++k) {
      const int32_t v = row[k];
      if (k < a1) A += v;
      else if (k < m) B += v;
      else if (k < m + c1) Cs += v;
      else D += v;
    }
    const int c = r / R, yy = r - c * R;
    int16_t* h = hb + ((size_t)c * 3 * R + yy) * kWhtTW + x0s;
#pragma unroll
    for (int j = 0; j < kWhtHS; ++j) {
      if (j > 0) {
        const int32_t v0 = row[j - 1], va = row[j - 1 + a1], vm = row[j - 1 + m];
        const int32_t vc = row[j - 1 + m + c1], ve = row[j + 2 * RHO];
        A += va - v0;
        B += vm - va;
        Cs += vc - vm;
        D += ve - vc;
      }
      h[j] = (int16_t)(A + B + Cs + D);
      h[R * kWhtTW + j] = (int16_t)(A + B - Cs - D);
      h[2 * R * kWhtTW + j] = (int16_t)(A - B - Cs + D);
    }
  }
  __syncthreads();
  // vertical runs: thread (lane, grp) owns column lane and kWhtRPT rows from
  // kWhtRPT grp; the runs of the first row are summed, then slid one row at a
  // time
  const int x = x0 + lane, py0 = kWhtRPT * grp;
  int32_t run[3][3][4];   // [channel][plane][A, B, Cs, D]
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (c < C) {
        const int16_t* col = hb + ((size_t)(c * 3 + v) * R + py0) * kWhtTW + lane;
        int32_t A = 0, B = 0, Cs = 0, D = 0;
#pragma unroll
        for (int k = 0; k <= 2 * RHO; ++k) {
          const int32_t h = col[k * kWhtTW];
          if (k < a1) A += h;
          else if (k < m) B += h;
          else if (k < m + c1) Cs += h;
          else D += h;
        }
        run[c][v][0] = A;
        run[c][v][1] = B;
        run[c][v][2] = Cs;
        run[c][v][3] = D;
      }
    }
#pragma unroll
  for (int i = 0; i < kWhtRPT; ++i) {
    if (i > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          if (c < C) {
            // the runs move down one row: each loses its first row and gains
            // the one after its last
            const int16_t* col = hb + ((size_t)(c * 3 + v) * R + py0 + i - 1) * kWhtTW + lane;
            const int32_t h0 = col[0], ha = col[a1 * kWhtTW], hm = col[m * kWhtTW];
            const int32_t hc = col[(m + c1) * kWhtTW], he = col[(2 * RHO + 1) * kWhtTW];
            run[c][v][0] += ha - h0;
            run[c][v][1] += hm - ha;
            run[c][v][2] += hc - hm;
            run[c][v][3] += he - hc;
          }
        }
    }
    int32_t out[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) out[j] = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < C) {
        int32_t w[3][3];   // w[u][v]: vertical function u over horizontal plane v
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const int32_t A = run[c][v][0], B = run[c][v][1], Cs = run[c][v][2], D = run[c][v][3];
          w[0][v] = A + B + Cs + D;
          w[1][v] = A + B - Cs - D;
          w[2][v] = A - B - Cs + D;
        }
        out[9 * c + 0] = w[0][0];
        out[9 * c + 1] = w[0][1];
        out[9 * c + 2] = w[1][0];
        out[9 * c + 3] = w[1][1];
        out[9 * c + 4] = w[0][2];
        out[9 * c + 5] = w[2][0];
        out[9 * c + 6] = w[1][2];
        out[9 * c + 7] = w[2][1];
        out[9 * c + 8] = w[2][2];
      }
    }
    const int y = y0 + py0 + i;
    if (x < W && y < H) {
      typedef int32_t v4_t __attribute__((ext_vector_type(4)));
      v4_t* dst = reinterpret_cast<v4_t*>(V + ((size_t)y * W + x) * stride);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (4 * q < stride) dst[q] = v4_t{out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]};
    }
  }
}

template <int RHO>
__global__ __launch_bounds__(256) void k_wht(const uint8_t* __restrict__ J, int W, int H, int C, int stride,
                                             int32_t* __restrict__ V) {
  wht_tile<RHO>(J, W, H, C, stride, V);
}

// Both radii of a descriptor in one launch (grid z = radius): each radius
// alone leaves most of the chip idle (its tiles are short chains of loads,
// two barriers and stores), side by side they overlap.
template <int RA, int RB>
__global__ __launch_bounds__(256) void k_wht2(const uint8_t* __restrict__ J, int W, int H, int C, int stride,
                                              int32_t* __restrict__ VA, int32_t* __restrict__ VB) {
  if (blockIdx.z == 0) wht_tile<RA>(J, W, H, C, stride, VA);
  else wht_tile<RB>(J, W, H, C, stride, VB);
}

template <int RHO>
static void launch_wht(const ff_desc* d, const uint8_t* lab, int32_t* V, hipStream_t stream) {
  const dim3 grid((d->width + kWhtTW - 1) / kWhtTW, (d->height + kWhtTH - 1) / kWhtTH);
  k_wht<RHO><<<grid, 256, wht_lds_bytes(d->channels, RHO), stream>>>(lab, d->width, d->height, d->channels,
                                                                      d->wht_stride, V);
}

template <int RA, int RB>
static void launch_wht2(const ff_desc* d, const uint8_t* lab, int32_t* VA, int32_t* VB, hipStream_t stream) {
  const dim3 grid((d->width + kWhtTW - 1) / kWhtTW, (d->height + kWhtTH - 1) / kWhtTH, 2);
  const size_t lds = std::max(wht_lds_bytes(d->channels, RA), wht_lds_bytes(d->channels, RB));
  k_wht2<RA, RB><<<grid, 256, lds, stream>>>(lab, d->width, d->height, d->channels, d->wht_stride, VA, VB);
}

static void enqueue_wht(const ff_desc* d, const uint8_t* lab, char* base, hipStream_t stream) {
  static_assert(kMaxRadius == 15, "one instance per radius");
  if (d->n_radii == 2) {
    // the radius pairs of the paper's two settings (r, r2) = (8, 6) and (3, 2)
    int32_t* V0 = reinterpret_cast<int32_t*>(base + d->off_wht);
    int32_t* V1 = V0 + (size_t)d->width * d->height * d->wht_stride;
    if (d->radii[0] == 8 && d->radii[1] == 6) return launch_wht2<8, 6>(d, lab, V0, V1, stream);
    if (d->radii[0] == 3 && d->radii[1] == 2) return launch_wht2<3, 2>(d, lab, V0, V1, stream);
  }
  for (int i = 0; i < d->n_radii; ++i) {
    int32_t* V = reinterpret_cast<int32_t*>(base + d->off_wht) + (size_t)i * d->width * d->height * d->wht_stride;
    switch (d->radii[i]) {
      case 1: launch_wht<1>(d, lab, V, stream); break;
      case 2: launch_wht<2>(d, lab, V, stream); break;
      case 3: launch_wht<3>(d, lab, V, stream); break;
      case 4: launch_wht<4>(d, lab, V, stream); break;
      case 5: launch_wht<5>(d, lab, V, stream); break;
      case 6: launch_wht<6>(d, lab, V, stream); break;
      case 7: launch_wht<7>(d, lab, V, stream); break;
      case 8: launch_wht<8>(d, lab, V, stream); break;
      case 9: launch_wht<9>(d, lab, V, stream); break;
      case 10: launch_wht<10>(d, lab, V, stream); break;
      case 11: launch_wht<11>(d, lab, V, stream); break;
      case 12: launch_wht<12>(d, lab, V, stream); break;
      case 13: launch_wht<13>(d, lab, V, stream); break;
      case 14: launch_wht<14>(d, lab, V, stream); break;
      default: launch_wht<15>(d, lab, V, stream); break;
    }
  }
}

// ---------------------------------------------------------------- SIFT colour levels
// The SIFT-flow colours (section 3.3) are smoothed per level as the images
// of section 3.2: the same block sums and Q14 Lanczos passes, on int16 codes
// (channels last), in 64-bit sums, the output in code units.  Level 0 is the
// codes themselves; channels S..P-1 of every level are zero.
__global__ void k_code_copy(const int16_t* __restrict__ codes, int N, int S, int P, int16_t* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)N * P) return;
  const int c = (int)(i % P);
  out[i] = c < S ? codes[(i / P) * S + c] : (int16_t)0;
}

// block sums of channel c (grid z) over n x n, replicate-padded
__global__ void k_code_blocksum(const int16_t* __restrict__ codes, int W, int H, int S, int n, int Wc, int Hc,
                                int32_t* __restrict__ A) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  if (j >= Wc) return;
  int32_t s = 0;
  for (int u = 0; u < n; ++u) {
    const int16_t* row = codes + (size_t)min(i * n + u, H - 1) * W * S + c;
    for (int v = 0; v < n; ++v) s += row[(size_t)min(j * n + v, W - 1) * S];
  }
  A[((size_t)c * Hc + i) * Wc + j] = s;
}

__global__ void k_code_lanczos_h(const int32_t* __restrict__ A, int W, int n, int li, int Wc, int Hc,
                                 int32_t* __restrict__ T) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  if (x >= W) return;
  const int32_t* row = A + ((size_t)c * Hc + i) * Wc;
  const int ph = x % n, base = x / n;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) s += (int64_t)c_lanczos[li][ph][k] * row[clampi(base + k - 3, 0, Wc - 1)];
  T[((size_t)c * Hc + i) * W + x] = (int32_t)((s + 8192) >> 14);
}

// vertical pass: divide by 2^14 n^2 (shift = 14 + 2 log2 n), round half up;
// grid z covers all P channels (the padding ones are written zero)
__global__ void k_code_lanczos_v(const int32_t* __restrict__ T, int W, int H, int n, int li, int Hc, int shift, int S,
                                 int P, int16_t* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, c = blockIdx.z;
  if (x >= W) return;
  int16_t v = 0;
  if (c < S) {
    const int32_t* Pl = T + (size_t)c * Hc * W;
    const int ph = y % n, base = y / n;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 7; ++k) s += (int64_t)c_lanczos[li][ph][k] * Pl[(size_t)clampi(base + k - 3, 0, Hc - 1) * W + x];
    v = (int16_t)((s + ((int64_t)1 << (shift - 1))) >> shift);
  }
  out[((size_t)y * W + x) * P + c] = v;
}

size_t sift_levels_scratch_bytes(int W, int H, int S) {
  const int Wc = (W + 1) / 2, Hc = (H + 1) / 2;
  return (size_t)S * ((size_t)Hc * Wc + (size_t)Hc * W) * 4;
}

void enqueue_sift_levels(const int16_t* codes, int W, int H, int S, int P, int k, int16_t* levels, int32_t* scratch,
                         hipStream_t stream) {
  const size_t N = (size_t)W * H;
  k_code_copy<<<(unsigned)((N * P + 255) / 256), 256, 0, stream>>>(codes, (int)N, S, P, levels);
  const unsigned gx = (unsigned)((W + 255) / 256);
  for (int lev = 1; lev <= k; ++lev) {
    const int n = 1 << lev;
    const int Wc = (W + n - 1) / n, Hc = (H + n - 1) / n;
    int32_t* A = scratch;
    int32_t* T = scratch + (size_t)S * Hc * Wc;
    k_code_blocksum<<<dim3((unsigned)((Wc + 255) / 256), Hc, S), 256, 0, stream>>>(codes, W, H, S, n, Wc, Hc, A);
    k_code_lanczos_h<<<dim3(gx, Hc, S), 256, 0, stream>>>(A, W, n, lev - 1, Wc, Hc, T);
    k_code_lanczos_v<<<dim3(gx, H, P), 256, 0, stream>>>(T, W, H, n, lev - 1, Hc, 14 + 2 * lev, S, P,
                                                         levels + (size_t)lev * N * P);
  }
}

// argument checks shared by the entry points that take an image
static ff_status check_image(const ff_desc* d, const ff_image* img, const uint8_t* pixels, void* blob,
                             size_t blob_bytes) {
  if (!d || !img || !pixels || !blob) return FF_ERR_ARG;
  if (img->width != d->width || img->height != d->height || img->channels != d->channels ||
      img->row_stride < img->width * img->channels)
    return FF_ERR_ARG;
  if (blob_bytes < d->bytes) return FF_ERR_WORKSPACE;
  return ensure_init();
}

// Lab8 planes and the WHT vectors of every radius
static void enqueue_lab_wht(const ff_desc* d, const ff_image* img, const uint8_t* pixels, char* base,
                            hipStream_t stream) {
  uint8_t* lab = reinterpret_cast<uint8_t*>(base + d->off_lab);
  prof_mark(FF_PROF_LAB, stream, true);
  k_lab8<<<dim3((unsigned)((d->width + 255) / 256), d->height), dim3(256), 0, stream>>>(
      pixels, d->width, d->height, d->channels, img->row_stride, lab);
  prof_mark(FF_PROF_LAB, stream, false);
  prof_mark(FF_PROF_WHT, stream, true);
  enqueue_wht(d, lab, base, stream);
  prof_mark(FF_PROF_WHT, stream, false);
}

// the smoothed levels I^n and the census planes of every level and phase,
// from the blob's Lab8 planes
static void enqueue_levels_census(const ff_desc* d, char* base, hipStream_t stream) {
  const int W = d->width, H = d->height, C = d->channels;
  const size_t N = (size_t)W * H;
  const uint8_t* lab = reinterpret_cast<const uint8_t*>(base + d->off_lab);
  int16_t* smooth = reinterpret_cast<int16_t*>(base + d->off_smooth);
  int32_t* scratch = reinterpret_cast<int32_t*>(base + d->off_census);
  const dim3 tb(256);
  prof_mark(FF_PROF_SMOOTH, stream, true);
  {
    const SmoothPlan sp = smooth_plan(W, H, C, d->k);
    const auto blocks = [](int64_t items) { return (unsigned)((items + 255) / 256); };
    k_smooth_blocks<<<blocks(sp.end1[d->k]), tb, 0, stream>>>(lab, sp, smooth, scratch);
    if (d->k > 0) {
      k_smooth_h<<<blocks(sp.end2[d->k]), tb, 0, stream>>>(sp, scratch);
      k_smooth_v<<<blocks((int64_t)d->k * C * (int64_t)N), tb, 0, stream>>>(sp, scratch, smooth);
    }
  }
  prof_mark(FF_PROF_SMOOTH, stream, false);
  prof_mark(FF_PROF_CENSUS, stream, true);
  {
    uint32_t* rm = reinterpret_cast<uint32_t*>(base + d->off_census);
    uint32_t* tr = reinterpret_cast<uint32_t*>(base + d->off_census_t);
    const dim3 cg((W + kCensusTile - 1) / kCensusTile, (H + kCensusTile - 1) / kCensusTile, d->k + 1);
    const int lw = kCensusTile + 2 * (1 << d->k) + 2, plane = lw * lw;
    const size_t lds = (size_t)C * plane * sizeof(int16_t);
    switch (d->subpel) {
      case 1: k_census<1><<<cg, tb, lds, stream>>>(smooth, W, H, C, plane, rm, tr); break;
      case 2: k_census<2><<<cg, tb, lds, stream>>>(smooth, W, H, C, plane, rm, tr); break;
      case 4: k_census<4><<<cg, tb, lds, stream>>>(smooth, W, H, C, plane, rm, tr); break;
      default: k_census<8><<<cg, tb, lds, stream>>>(smooth, W, H, C, plane, rm, tr); break;
    }
  }
  prof_mark(FF_PROF_CENSUS, stream, false);
}

}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_init(void) {
  const ff_status st = ensure_init();
  return st != FF_OK ? st : noalloc_scratch(nullptr);
}

ff_status ff_desc_init(ff_desc* d, const ff_image* img, int32_t k, int32_t subpel, const int32_t* radii,
                       int32_t n_radii) {
  if (!d || !img) return FF_ERR_ARG;
  const int W = img->width, H = img->height, C = img->channels;
  if (W < 1 || H < 1 || (C != 1 && C != 3) || img->row_stride < W * C) return FF_ERR_ARG;
  if (k < 0 || k > 4) return FF_ERR_ARG;
  if (subpel != 1 && subpel != 2 && subpel != 4 && subpel != 8) return FF_ERR_ARG;
  if (n_radii < 0 || n_radii > FF_MAX_RADII || (n_radii > 0 && !radii)) return FF_ERR_ARG;
  if (W > kMaxDim || H > kMaxDim || (int64_t)W * H > kMaxPoints) return FF_ERR_SIZE;
  if ((int64_t)W * subpel > 32767 || (int64_t)H * subpel > 32767) return FF_ERR_SIZE;
  *d = ff_desc{};
  d->width = W;
  d->height = H;
  d->channels = C;
  d->k = k;
  d->subpel = subpel;
  d->n_radii = n_radii;
  for (int i = 0; i < n_radii; ++i) {
    if (radii[i] < 1 || radii[i] > kMaxRadius) return FF_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (radii[j] == radii[i]) return FF_ERR_ARG;
    d->radii[i] = radii[i];
  }
  d->wht_dims = 9 * C;
  d->wht_stride = C == 3 ? 32 : 16;
  const size_t N = (size_t)W * H;
  size_t off = 0;
  d->off_lab = off;
  off = align_up(off + C * N, 256);
  d->off_smooth = off;
  off = align_up(off + (size_t)(k + 1) * C * N * 2, 256);
  d->off_census = off;
  d->plane_bytes = N * 4;
  size_t census = (size_t)(k + 1) * subpel * subpel * N * 4;
  // the census region doubles as the smoothing's scratch (every level's
  // block sums and horizontal pass) before the planes are written
  const size_t scratch = smooth_scratch_words(W, H, C, k) * 4;
  if (scratch > census) census = scratch;
  off = align_up(off + census, 256);
  d->off_census_t = off;
  off = align_up(off + (size_t)(k + 1) * subpel * subpel * N * 4, 256);
  d->off_wht = off;
  off = align_up(off + (size_t)n_radii * N * d->wht_stride * 4, 256);
  d->bytes = off;
  // the propagation sweep reads the row-major and the transposed census
  // planes of a level from one base with 32-bit byte offsets: its largest
  // word index, (census region words) + Q^2 N - 1, must stay below 2^30
  // (reached only at Q = 8 with k >= 2 on large images)
  if ((d->off_census_t - d->off_census) / 4 + (size_t)subpel * subpel * N > ((size_t)1 << 30)) {
    *d = ff_desc{};
    return FF_ERR_SIZE;
  }
  return FF_OK;
}

ff_status ff_compute_descriptors(const ff_desc* d, const ff_image* img, const uint8_t* pixels, void* blob,
                                 size_t blob_bytes, hipStream_t stream) {
  ff_status st = check_image(d, img, pixels, blob, blob_bytes);
  if (st != FF_OK) return st;
  prof_mark(FF_PROF_DESCRIPTORS, stream, true);
  enqueue_lab_wht(d, img, pixels, static_cast<char*>(blob), stream);
  enqueue_levels_census(d, static_cast<char*>(blob), stream);
  prof_mark(FF_PROF_DESCRIPTORS, stream, false);
  return launch_status();
}

ff_status ff_compute_census(const ff_desc* d, void* blob, size_t blob_bytes, hipStream_t stream) {
  if (!d || !blob) return FF_ERR_ARG;
  if (blob_bytes < d->bytes) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  enqueue_levels_census(d, static_cast<char*>(blob), stream);
  return launch_status();
}

ff_status ff_compute_lab_wht(const ff_desc* d, const ff_image* img, const uint8_t* pixels, void* blob,
                             size_t blob_bytes, hipStream_t stream) {
  ff_status st = check_image(d, img, pixels, blob, blob_bytes);
  if (st != FF_OK) return st;
  enqueue_lab_wht(d, img, pixels, static_cast<char*>(blob), stream);
  return launch_status();
}

}  // extern "C"
