// Eq. 5 (section 3.4): two-way forward/backward consistency check.  Keep p
// iff the nearest target pixel m = round-half-up(p + F(p)) lies in the second
// image and, for every backward field B_j, B_j(m) is set and
// |F(p) + B_j(m)|^2 < eps^2 (all in 1/Q px).  One thread per pixel.
#include "ff_internal.h"

namespace ff {

struct BwdPtrs {
  const int32_t* p[4];
};

__global__ void k_consistency(const int32_t* __restrict__ F, int W1, int H1, BwdPtrs B, int nb, int W2, int H2, int qshift,
                              int64_t lim, uint8_t* __restrict__ keep, int32_t* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W1) return;
  const size_t i = (size_t)y * W1 + x;
  const int32_t f = F[i];
  bool ok = f != kEmpty;
  if (ok) {
    const int fx = fx_of(f), fy = fy_of(f);
    const int half = (1 << qshift) >> 1;
    const int mx = ((x << qshift) + fx + half) >> qshift;
    const int my = ((y << qshift) + fy + half) >> qshift;
    ok = mx >= 0 && my >= 0 && mx < W2 && my < H2;
    for (int j = 0; ok && j < nb; ++j) {
      const int32_t b = B.p[j][(size_t)my * W2 + mx];
      if (b == kEmpty) {
        ok = false;
      } else {
        const int64_t ex = fx + fx_of(b), ey = fy + fy_of(b);
        ok = ex * ex + ey * ey < lim;
      }
    }
  }
  keep[i] = ok ? 1 : 0;
  out[i] = ok ? f : kEmpty;
}

// ---------------------------------------------------------------- region filter
// Section 3.4, second paragraph: the partly filtered field (pixels the check
// kept, flow set) is segmented into regions: 4-neighbours join when their
// flows differ by less than 3 px (dx^2 + dy^2 < 9 Q^2 in 1/Q px).  A region
// of fewer than s pixels is removed whole if a deleted outlier (a pixel the
// check did not keep, flow set) 4-adjacent to one of its pixels could join it
// by the same rule.  Regions are named by their smallest pixel index.
//
// Connected components by union-find whose roots are always the smallest
// index of their set (a link always hangs the larger root under the smaller,
// by atomicMin), so the final root is the region's name:
//   k_rf_local: per 64x16 tile with a one-pixel halo in LDS: union-find in
//     LDS over the tile's own pixels, per local component its size and
//     whether a deleted outlier could join it; writes each pixel's local root
//     (as a global index) and, at local roots, size | joinable << 31;
//   k_rf_merge: unions across tile borders on the global forest;
//   k_rf_count: each local root adds its size and flag to its global root
//     and points straight at it;
//   k_rf_final: mask, field and names.
constexpr int kRfTW = 64, kRfTH = 16;          // tile: 1024 pixels, 4 per thread
constexpr int kRfHW = kRfTW + 2, kRfHH = kRfTH + 2;
constexpr uint32_t kRfJoin = 0x80000000u;
constexpr uint32_t kRfSize = 0x7FFFFFFFu;

__device__ __forceinline__ bool rf_similar(int32_t f, int32_t g, int64_t lim) {
  const int64_t dx = fx_of(f) - fx_of(g), dy = fy_of(f) - fy_of(g);
  return dx * dx + dy * dy < lim;
}

// LDS union-find: parent values only decrease and always name a member of
// the same set with a smaller index
__device__ __forceinline__ int rf_find_lds(int32_t* L, int x) {
  for (;;) {
    const int p = __hip_atomic_load(&L[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    x = p;
  }
}
__device__ __forceinline__ void rf_unite_lds(int32_t* L, int a, int b) {
  for (;;) {
    a = rf_find_lds(L, a);
    b = rf_find_lds(L, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    // hang root b under a; if b stopped being a root meanwhile, unite a with
    // what b hangs under now
    const int old = __hip_atomic_fetch_min(&L[b], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (old == b) return;
    b = old;
  }
}
// the same on the global forest: workgroups of one launch may sit on
// different XCDs, so every access is a device-scope atomic
__device__ __forceinline__ int rf_find_g(int32_t* P, int x) {
  for (;;) {
    const int p = __hip_atomic_load(&P[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    x = p;
  }
}
__device__ __forceinline__ void rf_unite_g(int32_t* P, int a, int b) {
  for (;;) {
    a = rf_find_g(P, a);
    b = rf_find_g(P, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = __hip_atomic_fetch_min(&P[b], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == b) return;
    b = old;
  }
}

// grid: (ceil(W / 64), ceil(H / 16)), 256 threads
__global__ __launch_bounds__(256) void k_rf_local(const int32_t* __restrict__ F, const uint8_t* __restrict__ keep, int W,
                                                  int H, int64_t lim, int32_t* __restrict__ parent,
                                                  uint32_t* __restrict__ info) {
  __shared__ int32_t sF[kRfHH * kRfHW];   // flows of the tile and its halo (EMPTY outside the image)
  __shared__ uint8_t sK[kRfHH * kRfHW];   // 1: in the field, 2: deleted outlier, 0: neither
  __shared__ int32_t L[kRfTH * kRfTW];    // local forest over tile indices ly * 64 + lx
  __shared__ uint32_t S[kRfTH * kRfTW];   // per local root: size | joinable
  const int x0 = blockIdx.x * kRfTW, y0 = blockIdx.y * kRfTH;
  const int tid = threadIdx.x;
  for (int i = tid; i < kRfHH * kRfHW; i += 256) {
    const int hy = i / kRfHW, hx = i - hy * kRfHW;
    const int x = x0 + hx - 1, y = y0 + hy - 1;
    int32_t f = kEmpty;
    uint8_t k = 0;
    if (x >= 0 && y >= 0 && x < W && y < H) {
      const size_t g = (size_t)y * W + x;
      f = F[g];
      if (f != kEmpty) k = keep[g] != 0 ? 1 : 2;
    }
    sF[i] = f;
    sK[i] = k;
  }
  for (int li = tid; li < kRfTH * kRfTW; li += 256) {
    L[li] = li;
    S[li] = 0;
  }
  __syncthreads();
  for (int li = tid; li < kRfTH * kRfTW; li += 256) {
    const int lx = li & (kRfTW - 1), ly = li / kRfTW;
    const int h = (ly + 1) * kRfHW + lx + 1;
    if (sK[h] != 1) continue;
    if (lx + 1 < kRfTW && sK[h + 1] == 1 && rf_similar(sF[h], sF[h + 1], lim)) rf_unite_lds(L, li, li + 1);
    if (ly + 1 < kRfTH && sK[h + kRfHW] == 1 && rf_similar(sF[h], sF[h + kRfHW], lim))
      rf_unite_lds(L, li, li + kRfTW);
  }
  __syncthreads();
  for (int li = tid; li < kRfTH * kRfTW; li += 256) {
    const int lx = li & (kRfTW - 1), ly = li / kRfTW;
    const int h = (ly + 1) * kRfHW + lx + 1;
    if (sK[h] != 1) continue;
    const int r = rf_find_lds(L, li);
    // a deleted outlier 4-adjacent and similar (the halo holds the tile's
    // outer neighbours)
    const int32_t f = sF[h];
    const bool join = (sK[h - 1] == 2 && rf_similar(f, sF[h - 1], lim)) ||
                      (sK[h + 1] == 2 && rf_similar(f, sF[h + 1], lim)) ||
                      (sK[h - kRfHW] == 2 && rf_similar(f, sF[h - kRfHW], lim)) ||
                      (sK[h + kRfHW] == 2 && rf_similar(f, sF[h + kRfHW], lim));
    atomicAdd(&S[r], 1u);
    if (join) atomicOr(&S[r], kRfJoin);
  }
  __syncthreads();
  for (int li = tid; li < kRfTH * kRfTW; li += 256) {
    const int lx = li & (kRfTW - 1), ly = li / kRfTW;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= W || y >= H) continue;
    const size_t g = (size_t)y * W + x;
    const int h = (ly + 1) * kRfHW + lx + 1;
    int32_t pg = -1;
    uint32_t v = 0;
    if (sK[h] == 1) {
      const int r = rf_find_lds(L, li);
      pg = (y0 + r / kRfTW) * W + x0 + (r & (kRfTW - 1));
      if (r == li) v = S[li];   // a local root: size (>= 1) | joinable
    }
    parent[g] = pg;
    info[g] = v;
  }
}

// Unions across tile borders: one thread per pair of 4-neighbours that lie
// in different tiles (vertical borders first, then horizontal ones).
__global__ __launch_bounds__(256) void k_rf_merge(const int32_t* __restrict__ F, const uint8_t* __restrict__ keep, int W,
                                                  int H, int64_t lim, int32_t* parent) {
  const int tx = (W + kRfTW - 1) / kRfTW, ty = (H + kRfTH - 1) / kRfTH;
  const int nv = (tx - 1) * H;           // pairs across vertical borders
  const int nh = (ty - 1) * W;           // pairs across horizontal borders
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a, b;
  if (i < nv) {
    const int y = i / (tx - 1), x = (i - y * (tx - 1) + 1) * kRfTW;
    a = y * W + x - 1;
    b = a + 1;
  } else if (i < nv + nh) {
    const int j = i - nv;
    const int bi = j / W, x = j - bi * W;
    const int y = (bi + 1) * kRfTH;
    b = y * W + x;
    a = b - W;
  } else {
    return;
  }
  const int32_t fa = F[a], fb = F[b];
  if (fa == kEmpty || fb == kEmpty || keep[a] == 0 || keep[b] == 0 || !rf_similar(fa, fb, lim)) return;
  rf_unite_g(parent, a, b);
}

// Local roots carry their size and flag to their global root and point at
// it.  After k_rf_merge the forest no longer changes but for these pointer
// shortcuts, each to a member's own root.
__global__ __launch_bounds__(256) void k_rf_count(int N, int32_t* parent, uint32_t* info) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const uint32_t v = info[g];
  if (v == 0) return;                 // not a local root
  const int r = rf_find_g(parent, g);
  if (r == g) return;
  __hip_atomic_store(&parent[g], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  atomicAdd(&info[r], v & kRfSize);
  if (v & kRfJoin) atomicOr(&info[r], kRfJoin);
}

__global__ __launch_bounds__(256) void k_rf_final(const int32_t* __restrict__ F, int N, int s,
                                                  const int32_t* __restrict__ parent,
                                                  const uint32_t* __restrict__ info, int32_t* __restrict__ label,
                                                  uint8_t* __restrict__ keep_out, int32_t* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int lr = parent[g];
  int r = -1;
  bool kept = false;
  if (lr >= 0) {
    r = parent[lr];                   // a local root points at its region's root
    const uint32_t v = info[r];
    kept = !((int64_t)(v & kRfSize) < s && (v & kRfJoin));
  }
  if (label) label[g] = r;
  keep_out[g] = kept ? 1 : 0;
  out[g] = kept ? F[g] : kEmpty;
}

// ---------------------------------------------------------------- sparsification
// Section 3.5: one sample per 3x3 region of the outlier-filtered field that
// still holds at least e samples -- the sample whose summed consistency
// errors |F(p) + B_j(m)| (m the nearest pixel of p + F(p), as in Eq. 5) are
// smallest, first in raster order on ties.  Each error is measured in fixed
// point, floor(2^14 |e_j|) with |e_j| in 1/Q px, by an exact integer square
// root, so the choice is integer arithmetic; a lookup outside the second
// image or at an empty backward flow counts as the largest error.  Regions
// tile the image from (0,0) and are clipped at the borders.

// floor(sqrt(v)) for v < 2^62: a floating-point estimate made exact by
// integer tests (the estimate is within one of the result)
__device__ __forceinline__ uint64_t isqrt_u64(uint64_t v) {
  uint64_t r = (uint64_t)__builtin_sqrt((double)v);
  if (r > (1ull << 31)) r = 1ull << 31;
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// one thread per 3x3 region; grid: (ceil(ceil(W1 / 3) / 256), ceil(H1 / 3))
__global__ __launch_bounds__(256) void k_sparsify(const int32_t* __restrict__ F, int W1, int H1, BwdPtrs B, int nb,
                                                  int W2, int H2, int qshift, int e, int32_t* __restrict__ pick,
                                                  int32_t* __restrict__ sparse) {
  const int Bw = (W1 + 2) / 3;
  const int bx = blockIdx.x * blockDim.x + threadIdx.x, by = blockIdx.y;
  if (bx >= Bw) return;
  const uint64_t kNone = ~0ull;
  const int half = (1 << qshift) >> 1;
  const int x0 = 3 * bx, y0 = 3 * by;
  const int x1 = min(x0 + 3, W1), y1 = min(y0 + 3, H1);
  int count = 0, best = -1;
  uint64_t bestErr = 0;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      const int i = y * W1 + x;
      const int32_t f = F[i];
      if (f == kEmpty) continue;
      ++count;
      const int fx = fx_of(f), fy = fy_of(f);
      const int mx = ((x << qshift) + fx + half) >> qshift;
      const int my = ((y << qshift) + fy + half) >> qshift;
      uint64_t err = 0;
      const bool inside = mx >= 0 && my >= 0 && mx < W2 && my < H2;
      for (int j = 0; j < nb; ++j) {
        const int32_t b = inside ? B.p[j][my * W2 + mx] : kEmpty;
        if (b == kEmpty) {
          err = kNone;
          break;
        }
        const int64_t ex = fx + fx_of(b), ey = fy + fy_of(b);
        err += isqrt_u64((uint64_t)(ex * ex + ey * ey) << 28);
      }
      if (best < 0 || err < bestErr) {
        best = i;
        bestErr = err;
      }
    }
  const int32_t chosen = count >= e ? best : -1;
  pick[by * Bw + bx] = chosen;
  if (sparse)
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) {
        const int i = y * W1 + x;
        sparse[i] = i == chosen ? F[i] : kEmpty;
      }
}

}  // namespace ff

using namespace ff;

extern "C" ff_status ff_consistency_filter(const int32_t* flow_fwd, int32_t w1, int32_t h1,
                                           const int32_t* const* flow_bwd, int32_t n_bwd, int32_t w2, int32_t h2,
                                           int32_t subpel, int32_t eps_q, uint8_t* keep, int32_t* flow_filtered,
                                           hipStream_t stream) {
  if (!flow_fwd || !flow_bwd || !keep || !flow_filtered) return FF_ERR_ARG;
  if (w1 < 1 || h1 < 1 || w2 < 1 || h2 < 1 || n_bwd < 1 || n_bwd > 4 || eps_q < 0) return FF_ERR_ARG;
  if (subpel != 1 && subpel != 2 && subpel != 4 && subpel != 8) return FF_ERR_ARG;
  if (w1 > kMaxDim || h1 > kMaxDim || w2 > kMaxDim || h2 > kMaxDim) return FF_ERR_SIZE;
  BwdPtrs B{};
  for (int j = 0; j < n_bwd; ++j) {
    if (!flow_bwd[j]) return FF_ERR_ARG;
    B.p[j] = flow_bwd[j];
  }
  prof_mark(FF_PROF_FILTER, stream, true);
  k_consistency<<<dim3((w1 + 255) / 256, h1), 256, 0, stream>>>(flow_fwd, w1, h1, B, n_bwd, w2, h2, ilog2i(subpel),
                                                               (int64_t)eps_q * eps_q, keep, flow_filtered);
  prof_mark(FF_PROF_FILTER, stream, false);
  return launch_status();
}

extern "C" size_t ff_region_filter_workspace_bytes(int32_t width, int32_t height) {
  if (width < 1 || height < 1 || width > kMaxDim || height > kMaxDim || (int64_t)width * height > kMaxPoints) return 0;
  const size_t N = (size_t)width * height;
  return align_up(N * 4, 256) + align_up(N * 4, 256);
}

extern "C" ff_status ff_region_filter(const int32_t* flow, const uint8_t* keep, int32_t width, int32_t height,
                                      int32_t subpel, int32_t min_region, int32_t* label, uint8_t* keep_out,
                                      int32_t* flow_out, void* workspace, size_t workspace_bytes,
                                      hipStream_t stream) {
  if (!flow || !keep || !keep_out || !flow_out || !workspace) return FF_ERR_ARG;
  if (width < 1 || height < 1 || min_region < 0) return FF_ERR_ARG;
  if (subpel != 1 && subpel != 2 && subpel != 4 && subpel != 8) return FF_ERR_ARG;
  if (width > kMaxDim || height > kMaxDim || (int64_t)width * height > kMaxPoints) return FF_ERR_SIZE;
  if (workspace_bytes < ff_region_filter_workspace_bytes(width, height)) return FF_ERR_WORKSPACE;
  const int N = width * height;
  int32_t* parent = static_cast<int32_t*>(workspace);
  uint32_t* info = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) + align_up((size_t)N * 4, 256));
  const int64_t lim = 9LL * subpel * subpel;
  const int tx = (width + kRfTW - 1) / kRfTW, ty = (height + kRfTH - 1) / kRfTH;
  const int pairs = (tx - 1) * height + (ty - 1) * width;
  prof_mark(FF_PROF_REGION, stream, true);
  k_rf_local<<<dim3(tx, ty), 256, 0, stream>>>(flow, keep, width, height, lim, parent, info);
  if (pairs > 0) k_rf_merge<<<(pairs + 255) / 256, 256, 0, stream>>>(flow, keep, width, height, lim, parent);
  k_rf_count<<<(N + 255) / 256, 256, 0, stream>>>(N, parent, info);
  k_rf_final<<<(N + 255) / 256, 256, 0, stream>>>(flow, N, min_region, parent, info, label, keep_out, flow_out);
  prof_mark(FF_PROF_REGION, stream, false);
  return launch_status();
}

extern "C" ff_status ff_sparsify(const int32_t* flow, int32_t w1, int32_t h1, const int32_t* const* flow_bwd,
                                 int32_t n_bwd, int32_t w2, int32_t h2, int32_t subpel, int32_t min_samples,
                                 int32_t* pick, int32_t* flow_sparse, hipStream_t stream) {
  if (!flow || !flow_bwd || !pick) return FF_ERR_ARG;
  if (w1 < 1 || h1 < 1 || w2 < 1 || h2 < 1 || n_bwd < 1 || n_bwd > 4) return FF_ERR_ARG;
  if (subpel != 1 && subpel != 2 && subpel != 4 && subpel != 8) return FF_ERR_ARG;
  if (w1 > kMaxDim || h1 > kMaxDim || w2 > kMaxDim || h2 > kMaxDim || (int64_t)w1 * h1 > kMaxPoints ||
      (int64_t)w2 * h2 > kMaxPoints)
    return FF_ERR_SIZE;
  BwdPtrs B{};
  for (int j = 0; j < n_bwd; ++j) {
    if (!flow_bwd[j]) return FF_ERR_ARG;
    B.p[j] = flow_bwd[j];
  }
  const int Bw = (w1 + 2) / 3, Bh = (h1 + 2) / 3;
  prof_mark(FF_PROF_SPARSIFY, stream, true);
  k_sparsify<<<dim3((Bw + 255) / 256, Bh), 256, 0, stream>>>(flow, w1, h1, B, n_bwd, w2, h2, ilog2i(subpel),
                                                              min_samples, pick, flow_sparse);
  prof_mark(FF_PROF_SPARSIFY, stream, false);
  return launch_status();
}
