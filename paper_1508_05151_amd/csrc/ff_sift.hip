// The SIFT-flow data term of section 3.3 on gfx950: dense SIFT "colours"
// reduced by PCA, and the Flow Field search of sections 3.1 and 3.2 with
// that data term.
//
// Colours.  Every pixel's 128-dimensional SIFT vector (Lowe 2004, upright
// and dense as in Liu et al.'s SIFT flow; 4 x 4 cells of 3 px, 8 orientation
// bins, Gaussian window of sigma 6, normalise / clamp at 0.2 / normalise) is
// computed separably: one pass bins the central-difference gradients of the
// CIELab lightness and filters them along x with the four cell-column
// windows (32 values per pixel), a second pass filters along y with the four
// cell-row windows and normalises (fp32 throughout).  The PCA basis of a
// pair comes from the fp64 covariance of both images' vectors: per-workgroup
// fp64 Gram partials, a fixed-order reduction, and a one-sided Jacobi
// eigen-solver in one workgroup whose matrix stays in LDS (128 x 130
// doubles).  The projection on the first S eigenvectors is fp64 and is
// quantised to int16 codes, round-half-even(1024 c).
//
// Search.  The colour images are smoothed per level (ff_sift_levels) and
// the data term sums, over the (2r+1)^2 samples at stride n, the exact
// integer L2 distance of the colours, the target side bilinear in its four
// neighbours at the subpixel phase: floor(sqrt(sum_s d_s^2 * 256 / Q^4)) in
// 1/16 code units.  Seeds, level entries and random searches are per-point
// kernels; a propagation sweep (Eq. 2) is an anti-diagonal wavefront over
// bands of 4 grid rows, one workgroup per band, the band's top row taking
// its vertical candidates from the band above through tagged 64-bit words.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

constexpr int kSiftDim = 128;
constexpr int kSiftReach = 7;                  // |dx| < 2.5 c with c = 3
constexpr int kSiftTaps = 2 * kSiftReach + 1;
constexpr int kSiftMaxS = 32;
constexpr double kCodeScale = 1024.0;
constexpr int kCodeMax = 2047;

// cell-column (and, the same, cell-row) windows: Gaussian times the
// bilinear cell weight, per cell index and offset
struct SiftWin {
  float w[4][kSiftTaps];
};

static SiftWin sift_window() {
  SiftWin s;
  const double c = 3.0, sig = 2.0 * c;
  for (int i = 0; i < 4; ++i)
    for (int t = 0; t < kSiftTaps; ++t) {
      const int d = t - kSiftReach;
      const double b = 1.0 - std::fabs(d / c - (i - 1.5));
      s.w[i][t] = b > 0.0 ? (float)(std::exp(-(double)(d * d) / (2.0 * sig * sig)) * b) : 0.0f;
    }
  return s;
}

// ---------------------------------------------------------------- pass 1: bin and filter along x
// One workgroup = 64 x 4 pixels.  The binned gradients of the tile grown by
// 7 columns each side (zero outside the image) are staged in LDS as 8 bins
// per pixel; each thread then sums its 15 horizontal neighbours into 4 cell
// columns x 8 bins.  Output A: per pixel 32 floats, index i * 8 + o.
constexpr int kHistTW = 64, kHistTH = 4, kHistCols = kHistTW + 2 * kSiftReach;

__global__ __launch_bounds__(256) void k_sift_hist(const uint8_t* __restrict__ L, int W, int H, SiftWin win,
                                                   float* __restrict__ A) {
  __shared__ float hs[kHistTH][kHistCols][8];
  const int x0 = blockIdx.x * kHistTW, y0 = blockIdx.y * kHistTH;
  const float kTwoPi = 6.28318530717958647692f, kInvBin = 1.27323954473516268615f;   // 4 / pi
  for (int e = threadIdx.x; e < kHistTH * kHistCols; e += 256) {
    const int ty = e / kHistCols, tx = e - ty * kHistCols;
    const int x = x0 + tx - kSiftReach, y = y0 + ty;
    float m0 = 0.0f, m1 = 0.0f;
    int o0 = 0;
    if (x >= 0 && x < W && y < H) {
      const uint8_t* row = L + (size_t)y * W;
      const float gx = 0.5f * ((float)row[min(x + 1, W - 1)] - (float)row[max(x - 1, 0)]);
      const float gy = 0.5f * ((float)L[(size_t)min(y + 1, H - 1) * W + x] - (float)L[(size_t)max(y - 1, 0) * W + x]);
      const float m = sqrtf(gx * gx + gy * gy);
      if (m > 0.0f) {
        float th = atan2f(gy, gx);
        if (th < 0.0f) th += kTwoPi;
        const float t = th * kInvBin;
        const float fl = floorf(t);
        const float w1 = t - fl;
        o0 = ((int)fl) & 7;
        m0 = m * (1.0f - w1);
        m1 = m * w1;
      }
    }
    const int o1 = (o0 + 1) & 7;
#pragma unroll
    for (int o = 0; o < 8; ++o) hs[ty][tx][o] = (o == o0 ? m0 : 0.0f) + (o == o1 ? m1 : 0.0f);
  }
  __syncthreads();
  const int tx = threadIdx.x % kHistTW, ty = threadIdx.x / kHistTW;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= W || y >= H) return;
  float acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[i][o] = 0.0f;
#pragma unroll
  for (int t = 0; t < kSiftTaps; ++t) {
    const float4 h0 = *reinterpret_cast<const float4*>(&hs[ty][tx + t][0]);
    const float4 h1 = *reinterpret_cast<const float4*>(&hs[ty][tx + t][4]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float w = win.w[i][t];
      acc[i][0] = fmaf(w, h0.x, acc[i][0]);
      acc[i][1] = fmaf(w, h0.y, acc[i][1]);
      acc[i][2] = fmaf(w, h0.z, acc[i][2]);
      acc[i][3] = fmaf(w, h0.w, acc[i][3]);
      acc[i][4] = fmaf(w, h1.x, acc[i][4]);
      acc[i][5] = fmaf(w, h1.y, acc[i][5]);
      acc[i][6] = fmaf(w, h1.z, acc[i][6]);
      acc[i][7] = fmaf(w, h1.w, acc[i][7]);
    }
  }
  float4* out = reinterpret_cast<float4*>(A + ((size_t)y * W + x) * 32);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
    out[2 * i + 1] = make_float4(acc[i][4], acc[i][5], acc[i][6], acc[i][7]);
  }
}

// ---------------------------------------------------------------- pass 2: filter along y, normalise
// 8 lanes per pixel, 32 pixels per workgroup: lane q owns elements 4q..4q+3
// of the 32 per cell row, for the 4 cell rows j (descriptor element
// j * 32 + i * 8 + o = (4 j + i) 8 + o).  Rows outside the image add nothing.
__global__ __launch_bounds__(256) void k_sift_desc(const float* __restrict__ A, int W, int H, SiftWin win,
                                                   float* __restrict__ D) {
  const int q = threadIdx.x & 7;
  const int pix = blockIdx.x * 32 + (threadIdx.x >> 3);
  const bool ok = pix < W * H;
  const int p = ok ? pix : 0;
  const int x = p % W, y = p / W;
  float acc[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[j][e] = 0.0f;
#pragma unroll
  for (int t = 0; t < kSiftTaps; ++t) {
    const int yy = y + t - kSiftReach;
    if (yy < 0 || yy >= H) continue;
    const float4 a = *reinterpret_cast<const float4*>(A + ((size_t)yy * W + x) * 32 + 4 * q);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float w = win.w[j][t];
      acc[j][0] = fmaf(w, a.x, acc[j][0]);
      acc[j][1] = fmaf(w, a.y, acc[j][1]);
      acc[j][2] = fmaf(w, a.z, acc[j][2]);
      acc[j][3] = fmaf(w, a.w, acc[j][3]);
    }
  }
  float nn = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) nn = fmaf(acc[j][e], acc[j][e], nn);
  nn += __shfl_xor(nn, 1);
  nn += __shfl_xor(nn, 2);
  nn += __shfl_xor(nn, 4);
  if (nn > 0.0f) {
    const float s = 1.0f / sqrtf(nn);
    float n2 = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[j][e] = fminf(acc[j][e] * s, 0.2f);
        n2 = fmaf(acc[j][e], acc[j][e], n2);
      }
    n2 += __shfl_xor(n2, 1);
    n2 += __shfl_xor(n2, 2);
    n2 += __shfl_xor(n2, 4);
    const float s2 = 1.0f / sqrtf(n2);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[j][e] *= s2;
  }
  if (!ok) return;
  float4* out = reinterpret_cast<float4*>(D + (size_t)pix * kSiftDim);
#pragma unroll
  for (int j = 0; j < 4; ++j) out[j * 8 + q] = make_float4(acc[j][0], acc[j][1], acc[j][2], acc[j][3]);
}

// ---------------------------------------------------------------- PCA: fp64 Gram partials
// Rows r0..r1 of the two images' vectors stacked (image 1 first).  Thread
// (bi, bj) of the 16 x 16 grid owns the 8 x 8 block of sum d d^T; threads
// 0..127 also sum element t.  Rows are staged 32 at a time in LDS.
// part: per workgroup 128 * 128 + 128 doubles.
constexpr int kGramRows = 32;
constexpr int kPartDoubles = kSiftDim * kSiftDim + kSiftDim;

__global__ __launch_bounds__(256) void k_sift_gram(const float* __restrict__ D1, int N1, const float* __restrict__ D2,
                                                   int N2, int rows_per_wg, double* __restrict__ part) {
  __shared__ float tile[kGramRows][kSiftDim + 4];
  const int bi = threadIdx.x >> 4, bj = threadIdx.x & 15;
  double acc[8][8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int l = 0; l < 8; ++l) acc[k][l] = 0.0;
  double msum = 0.0;
  const int N = N1 + N2;
  const int r0 = blockIdx.x * rows_per_wg, r1 = min(N, r0 + rows_per_wg);
  for (int rb = r0; rb < r1; rb += kGramRows) {
    for (int e = threadIdx.x; e < kGramRows * 32; e += 256) {
      const int rr = e >> 5, cq = e & 31;
      const int row = rb + rr;
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (row < r1) {
        const float* src = row < N1 ? D1 + (size_t)row * kSiftDim : D2 + (size_t)(row - N1) * kSiftDim;
        v = *reinterpret_cast<const float4*>(src + 4 * cq);
      }
      *reinterpret_cast<float4*>(&tile[rr][4 * cq]) = v;
    }
    __syncthreads();
    for (int rr = 0; rr < kGramRows; ++rr) {
      double a[8], b[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        a[k] = (double)tile[rr][8 * bi + k];
        b[k] = (double)tile[rr][8 * bj + k];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int l = 0; l < 8; ++l) acc[k][l] = fma(a[k], b[l], acc[k][l]);
      if (threadIdx.x < kSiftDim) msum += (double)tile[rr][threadIdx.x];
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * kPartDoubles;
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int l = 0; l < 8; ++l) out[(8 * bi + k) * kSiftDim + 8 * bj + l] = acc[k][l];
  if (threadIdx.x < kSiftDim) out[kSiftDim * kSiftDim + threadIdx.x] = msum;
}

// fixed-order sum of the partials, divided by N: E[d d^T] then the mean
__global__ void k_sift_gram_reduce(const double* __restrict__ part, int nparts, int N, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPartDoubles) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * kPartDoubles + e];
  out[e] = s / (double)N;
}

// ---------------------------------------------------------------- PCA: one-sided Jacobi eigen-solver
// The covariance C (128 x 128, positive semi-definite) is orthogonalised by
// one-sided (Hestenes) Jacobi rotations of its columns, M <- M J with M = C
// at the start: a pair of columns (p, q) with norms a = |m_p|^2, b = |m_q|^2
// and product g = m_p . m_q is rotated by the angle that makes them
// orthogonal (zeta = (b - a) / (2 g), t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = t c).  At convergence M = C V
// with orthogonal columns, so C^2 is diagonal in V and column i is
// lambda_i v_i: the eigenvalues are the column norms and the eigenvectors
// the normalised columns -- no rotation product is accumulated, and the
// whole matrix stays in LDS.  A sweep is 127 rounds of the round-robin
// tournament, 64 disjoint pairs per round, 16 lanes per pair (dot products
// by DPP row sums, one barrier per round).  Pairs whose columns are already
// orthogonal to 1e-13 of their norms, or whose rotation angle is below
// 1e-15 (no change beyond rounding), are left alone; sweeps stop when none is
// rotated (or after 30).  Eigenvalues are then ranked descending (ties by
// index), each eigenvector's largest-magnitude component (the first on
// ties) is made positive, and out receives mean (128), eigenvalues (128) and
// the basis (128 x 128, element [k][s] = component k of eigenvector s).
constexpr int kMP = kSiftDim + 2;   // LDS row pitch (doubles): the 4 pairs of a wavefront in different banks
constexpr int kJacobiSweeps = 30;
constexpr double kOrthTol = 1e-13;
constexpr double kMinAngle = 1e-15;

__device__ __forceinline__ void tourney(int round, int k, int& p, int& q) {
  // circle method: player 0 fixed, players 1..127 rotate
  auto pos = [&](int i) { return 1 + (i + round) % 127; };
  if (k == 0) {
    p = 0;
    q = pos(0);
  } else {
    p = pos(k);
    q = pos(127 - k);
  }
}

__global__ __launch_bounds__(1024) void k_sift_eig(const double* __restrict__ raw, double* __restrict__ out) {
  __shared__ double Mt[kSiftDim * kMP];   // row i = column i of M
  __shared__ int s_rot[16];
  __shared__ double s_norm[kSiftDim];
  __shared__ int s_rank[kSiftDim];
  const int t = threadIdx.x;
  const double* mean = raw + kSiftDim * kSiftDim;
  for (int e = t; e < kSiftDim * kSiftDim; e += 1024) {
    const int i = e >> 7, j = e & 127;
    Mt[i * kMP + j] = raw[e] - mean[i] * mean[j];
  }
  __syncthreads();
  const int g = t >> 4, l = t & 15;
  for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
    int rotated = 0;
    for (int round = 0; round < 127; ++round) {
      int p, q;
      tourney(round, g, p, q);
      double* mp = Mt + p * kMP;
      double* mq = Mt + q * kMP;
      double x[8], y[8];
      double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        x[i] = mp[l + 16 * i];
        y[i] = mq[l + 16 * i];
        a = fma(x[i], x[i], a);
        b = fma(y[i], y[i], b);
        c = fma(x[i], y[i], c);
      }
      a = row16_sum_f64(a);   // the pair's 16 lanes are one DPP row
      b = row16_sum_f64(b);
      c = row16_sum_f64(c);
      if (fabs(c) > kOrthTol * sqrt(a * b)) {   // the same in all 16 lanes of the pair
        const double zeta = (b - a) / (2.0 * c);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        // a rotation by less than the rounding of the columns changes
        // nothing (pairs with a column at rounding level stay there)
        if (fabs(tt) > kMinAngle) {
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = tt * cs;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            mp[l + 16 * i] = cs * x[i] - sn * y[i];
            mq[l + 16 * i] = sn * x[i] + cs * y[i];
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    // any rotation in this sweep?
    const int any = __any(rotated) ? 1 : 0;
    if ((t & 63) == 0) s_rot[t >> 6] = any;
    __syncthreads();
    int tot = 0;
    for (int w = 0; w < 16; ++w) tot |= s_rot[w];
    __syncthreads();
    if (!tot) break;
  }
  if (t < kSiftDim) {
    double nn = 0.0;
    for (int k = 0; k < kSiftDim; ++k) nn = fma(Mt[t * kMP + k], Mt[t * kMP + k], nn);
    s_norm[t] = sqrt(nn);
  }
  __syncthreads();
  if (t < kSiftDim) {
    const double li = s_norm[t];
    int rank = 0;
    for (int j = 0; j < kSiftDim; ++j) {
      const double lj = s_norm[j];
      rank += (lj > li || (lj == li && j < t)) ? 1 : 0;
    }
    s_rank[t] = rank;
    out[t] = mean[t];
    out[kSiftDim + rank] = li;
  }
  __syncthreads();
  if (t < kSiftDim) {
    // column t of M becomes basis column s_rank[t]
    const double* v = Mt + t * kMP;
    int m = 0;
    double best = fabs(v[0]);
    for (int k = 1; k < kSiftDim; ++k)
      if (fabs(v[k]) > best) {
        best = fabs(v[k]);
        m = k;
      }
    const double inv = s_norm[t] > 0.0 ? (v[m] < 0.0 ? -1.0 : 1.0) / s_norm[t] : 0.0;
    const int s = s_rank[t];
    for (int k = 0; k < kSiftDim; ++k) out[2 * kSiftDim + k * kSiftDim + s] = v[k] * inv;
  }
}

// ---------------------------------------------------------------- projection to codes
// One thread per pixel accumulates all S (<= SM) projections in fp64,
// walking its vector 4 elements at a time; the first S basis columns and the
// mean sit in LDS.  Codes round-half-even(1024 c) clamped to +-2047, H x W x S
// int16.
template <int SM>
__global__ __launch_bounds__(256) void k_sift_project(const float* __restrict__ D, int N, const double* __restrict__ pca,
                                                      int S, int16_t* __restrict__ codes) {
  __shared__ double basis[kSiftDim * SM];
  __shared__ double mu[kSiftDim];
  for (int e = threadIdx.x; e < kSiftDim * SM; e += 256) {
    const int k = e / SM, s = e % SM;
    basis[e] = s < S ? pca[2 * kSiftDim + k * kSiftDim + s] : 0.0;
  }
  if (threadIdx.x < kSiftDim) mu[threadIdx.x] = pca[threadIdx.x];
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  double acc[SM];
#pragma unroll
  for (int s = 0; s < SM; ++s) acc[s] = 0.0;
  const float4* src = reinterpret_cast<const float4*>(D + (size_t)p * kSiftDim);
#pragma unroll 1
  for (int k4 = 0; k4 < kSiftDim / 4; ++k4) {
    const float4 v = src[k4];
    const float dv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * k4 + u;
      const double x = (double)dv[u] - mu[k];
#pragma unroll
      for (int s = 0; s < SM; ++s) acc[s] = fma(x, basis[k * SM + s], acc[s]);
    }
  }
  int16_t* out = codes + (size_t)p * S;
#pragma unroll
  for (int s = 0; s < SM; ++s)
    if (s < S) {
      const double v = rint(acc[s] * kCodeScale);
      out[s] = (int16_t)(v > kCodeMax ? kCodeMax : (v < -kCodeMax ? -kCodeMax : (int)v));
    }
}

static void enqueue_project(const float* D, int N, const double* pca, int S, int16_t* codes, hipStream_t stream) {
  const unsigned g = (unsigned)((N + 255) / 256);
  if (S <= 8)
    k_sift_project<8><<<g, 256, 0, stream>>>(D, N, pca, S, codes);
  else if (S <= 16)
    k_sift_project<16><<<g, 256, 0, stream>>>(D, N, pca, S, codes);
  else if (S <= 24)
    k_sift_project<24><<<g, 256, 0, stream>>>(D, N, pca, S, codes);
  else
    k_sift_project<32><<<g, 256, 0, stream>>>(D, N, pca, S, codes);
}

// ---------------------------------------------------------------- colour-stage layout
struct SiftColorLayout {
  size_t off_A, off_D1, off_D2, off_part, off_raw, off_pca;
  int nparts, rows_per_wg;
  size_t bytes;
};

static SiftColorLayout sift_color_layout(int w1, int h1, int w2, int h2) {
  SiftColorLayout L{};
  const size_t N1 = (size_t)w1 * h1, N2 = (size_t)w2 * h2, Nm = std::max(N1, N2);
  const size_t N = N1 + N2;
  L.rows_per_wg = 1024;
  L.nparts = (int)std::min<size_t>((N + L.rows_per_wg - 1) / L.rows_per_wg, 1024);
  L.rows_per_wg = (int)((N + L.nparts - 1) / L.nparts);
  L.rows_per_wg = (L.rows_per_wg + kGramRows - 1) / kGramRows * kGramRows;
  size_t off = 0;
  L.off_A = off;
  off = align_up(off + Nm * 32 * 4, 256);
  L.off_D1 = off;
  off = align_up(off + N1 * kSiftDim * 4, 256);
  L.off_D2 = off;
  off = align_up(off + N2 * kSiftDim * 4, 256);
  L.off_part = off;
  off = align_up(off + (size_t)L.nparts * kPartDoubles * 8, 256);
  L.off_raw = off;
  off = align_up(off + (size_t)kPartDoubles * 8, 256);
  L.off_pca = off;
  off = align_up(off + (size_t)(2 * kSiftDim + kSiftDim * kSiftDim) * 8, 256);
  L.bytes = off;
  return L;
}

static void enqueue_dense_sift(const uint8_t* L, int W, int H, const SiftWin& win, float* A, float* D,
                               hipStream_t stream) {
  k_sift_hist<<<dim3((W + kHistTW - 1) / kHistTW, (H + kHistTH - 1) / kHistTH), 256, 0, stream>>>(L, W, H, win, A);
  k_sift_desc<<<(unsigned)(((size_t)W * H + 31) / 32), 256, 0, stream>>>(A, W, H, win, D);
}

static bool sift_dims_ok(int w, int h) { return w >= 1 && h >= 1 && w <= kMaxDim && h <= kMaxDim && (int64_t)w * h <= kMaxPoints; }

}  // namespace ff

using namespace ff;

extern "C" {

int32_t ff_sift_pitch(int32_t S) { return S < 1 || S > kSiftMaxS ? 0 : (S + 3) / 4 * 4; }

size_t ff_sift_workspace_bytes(int32_t w1, int32_t h1, int32_t w2, int32_t h2) {
  if (!sift_dims_ok(w1, h1) || !sift_dims_ok(w2, h2)) return 0;
  const size_t colors = sift_color_layout(w1, h1, w2, h2).bytes;
  const size_t levels = std::max(sift_levels_scratch_bytes(w1, h1, kSiftMaxS), sift_levels_scratch_bytes(w2, h2, kSiftMaxS));
  return std::max(colors, align_up(levels, 256));
}

ff_status ff_dense_sift(const uint8_t* L, int32_t width, int32_t height, float* desc, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
  if (!L || !desc || !workspace) return FF_ERR_ARG;
  if (width < 1 || height < 1) return FF_ERR_ARG;
  if (!sift_dims_ok(width, height)) return FF_ERR_SIZE;
  if (workspace_bytes < (size_t)width * height * 32 * 4) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  static const SiftWin win = sift_window();
  prof_mark(FF_PROF_SIFT_COLORS, stream, true);
  enqueue_dense_sift(L, width, height, win, static_cast<float*>(workspace), desc, stream);
  prof_mark(FF_PROF_SIFT_COLORS, stream, false);
  return launch_status();
}

ff_status ff_sift_colors(const uint8_t* L1, int32_t w1, int32_t h1, const uint8_t* L2, int32_t w2, int32_t h2,
                         int32_t S, int16_t* codes1, int16_t* codes2, double* pca, float* desc1, float* desc2,
                         void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!L1 || !L2 || !codes1 || !codes2 || !workspace) return FF_ERR_ARG;
  if (w1 < 1 || h1 < 1 || w2 < 1 || h2 < 1 || S < 1 || S > kSiftMaxS) return FF_ERR_ARG;
  if (!sift_dims_ok(w1, h1) || !sift_dims_ok(w2, h2)) return FF_ERR_SIZE;
  const SiftColorLayout Lo = sift_color_layout(w1, h1, w2, h2);
  if (workspace_bytes < Lo.bytes) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  static const SiftWin win = sift_window();
  char* ws = static_cast<char*>(workspace);
  float* A = reinterpret_cast<float*>(ws + Lo.off_A);
  float* D1 = desc1 ? desc1 : reinterpret_cast<float*>(ws + Lo.off_D1);
  float* D2 = desc2 ? desc2 : reinterpret_cast<float*>(ws + Lo.off_D2);
  double* part = reinterpret_cast<double*>(ws + Lo.off_part);
  double* raw = reinterpret_cast<double*>(ws + Lo.off_raw);
  double* P = pca ? pca : reinterpret_cast<double*>(ws + Lo.off_pca);
  const int N1 = w1 * h1, N2 = w2 * h2;
  prof_mark(FF_PROF_SIFT_COLORS, stream, true);
  enqueue_dense_sift(L1, w1, h1, win, A, D1, stream);
  enqueue_dense_sift(L2, w2, h2, win, A, D2, stream);
  prof_mark(FF_PROF_SIFT_PCA, stream, true);
  k_sift_gram<<<Lo.nparts, 256, 0, stream>>>(D1, N1, D2, N2, Lo.rows_per_wg, part);
  k_sift_gram_reduce<<<(kPartDoubles + 255) / 256, 256, 0, stream>>>(part, Lo.nparts, N1 + N2, raw);
  k_sift_eig<<<1, 1024, 0, stream>>>(raw, P);
  prof_mark(FF_PROF_SIFT_PCA, stream, false);
  enqueue_project(D1, N1, P, S, codes1, stream);
  enqueue_project(D2, N2, P, S, codes2, stream);
  prof_mark(FF_PROF_SIFT_COLORS, stream, false);
  return launch_status();
}

ff_status ff_sift_levels(const int16_t* codes, int32_t width, int32_t height, int32_t S, int32_t k, int16_t* levels,
                         void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!codes || !levels || !workspace) return FF_ERR_ARG;
  if (width < 1 || height < 1 || S < 1 || S > kSiftMaxS || k < 0 || k > 4) return FF_ERR_ARG;
  if (!sift_dims_ok(width, height)) return FF_ERR_SIZE;
  if (workspace_bytes < sift_levels_scratch_bytes(width, height, S)) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  prof_mark(FF_PROF_SIFT_LEVELS, stream, true);
  enqueue_sift_levels(codes, width, height, S, ff_sift_pitch(S), k, levels, static_cast<int32_t*>(workspace), stream);
  prof_mark(FF_PROF_SIFT_LEVELS, stream, false);
  return launch_status();
}

}  // extern "C"
