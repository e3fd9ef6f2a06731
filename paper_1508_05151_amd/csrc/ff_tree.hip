// kd-tree over the WHT vectors of every target pixel (section 3.1): split
// while a node holds more than l points, on the dimension of maximal spread,
// at the median of (key, pixel index).
//
// GPU design.  The tree is perfectly balanced by construction (left child =
// first floor(cnt/2) points), so every node's range in the permutation array
// is a function of its heap index alone.  Only the *membership* of each child
// matters (leaves are finally sorted by pixel index), so the order inside a
// node is free.
//  * Top levels (nodes larger than kTreeLds points): level-synchronous passes
//    over all nodes of a level at once (down to kNodeMax points per node;
//    below that, one workgroup per node does a level in one launch) --
//      minmax    per-node per-dimension min/max (order-free atomics), a pass
//                of its own for the root only,
//      hist x4   MSD radix select of the rank floor(cnt/2) element of the
//                44-bit key ((key - min) << 22 | pixel), 11 bits per pass,
//      partition strict-less-than-pivot to the left, others right; each
//                workgroup then reduces the two children's min/max over its
//                chunk for the next level.
//  * Below: one workgroup per subtree of <= kTreeLds points finishes every
//    remaining level in LDS with a bitonic sort of (segment, key, pixel).
#include "ff_internal.h"
#include "ff_device.h"

namespace ff {

constexpr int kChunk = 2048;     // elements per workgroup in the global passes (more workgroups:
                                 // the passes are latency-bound, 4096 measured 12 % slower)
constexpr int kTpb = 256;

// The tree's launches are short, latency-bound chains on every field's
// critical path; beside them the census planes are built with time to spare.
// Their waves therefore go first in the SIMD arbitration (the census waves
// keep the default): measured 1.32 -> 1.28 ms per tree and 10.14 -> 10.12 ms
// per pair with the three trees and both images' census at once.
__device__ __forceinline__ void tree_priority() { __builtin_amdgcn_s_setprio(2); }

int tree_depth_of(int N, int leaf) {
  int d = 0;
  while (((int64_t)N + (1LL << d) - 1) / (1LL << d) > leaf) ++d;
  return d;
}

TreeLayout tree_layout(int N, int leaf, size_t base) {
  TreeLayout L{};
  L.N = N;
  L.depth = tree_depth_of(N, leaf);
  L.nodes = (2 << L.depth) - 1;
  int top = 0;
  while (((int64_t)N + (1LL << top) - 1) / (1LL << top) > kTreeLds) ++top;
  L.top = top;
  const size_t topnodes = ((size_t)1 << top) - 1;
  size_t off = align_up(base, 256);
  L.off_dim = off;   off = align_up(off + (size_t)L.nodes * 4, 256);
  L.off_split = off; off = align_up(off + (size_t)L.nodes * 4, 256);
  L.off_perm = off;  off = align_up(off + (size_t)N * 4, 256);
  L.off_perm2 = off; off = align_up(off + (size_t)N * 4, 256);
  L.off_minmax = off; off = align_up(off + topnodes * 64 * 4, 256);
  L.off_hist = off;  off = align_up(off + topnodes * kSelPasses * kSelBins * 4, 256);
  L.off_cnt = off;   off = align_up(off + topnodes * 2 * 4, 256);
  L.off_key = off;   off = align_up(off + (size_t)N * 4, 256);
  L.bytes = off - base;
  return L;
}

// range [start, start+cnt) of node j at depth d (j's bits from the top are
// the left/right decisions)
__device__ __forceinline__ void node_range(int d, int j, int N, int& start, int& cnt) {
  start = 0;
  cnt = N;
  for (int b = d - 1; b >= 0; --b) {
    const int h = cnt >> 1;
    if ((j >> b) & 1) { start += h; cnt -= h; }
    else cnt = h;
  }
}

// per-field views of the tree arrays
struct TreeView {
  const int32_t* V;
  int N, D, stride, top, nodes;
  int32_t *dim, *split, *perm, *perm2, *mm, *hist, *cnt;
  uint32_t* key;   // per position: value on the node's split dimension - node minimum
};

__device__ __forceinline__ TreeView tree_view(const FieldRec& f) {
  TreeView t;
  t.V = f.Vdst;
  t.N = f.Wd * f.Hd;
  t.D = f.D;
  t.stride = f.vstride;
  t.top = f.t_top;
  t.nodes = f.t_nodes;
  t.dim = reinterpret_cast<int32_t*>(f.ws + f.o_dim);
  t.split = reinterpret_cast<int32_t*>(f.ws + f.o_split);
  t.perm = reinterpret_cast<int32_t*>(f.ws + f.o_perm);
  t.perm2 = reinterpret_cast<int32_t*>(f.ws + f.o_perm2);
  t.mm = reinterpret_cast<int32_t*>(f.ws + f.o_mm);
  t.hist = reinterpret_cast<int32_t*>(f.ws + f.o_hist);
  t.cnt = reinterpret_cast<int32_t*>(f.ws + f.o_cnt);
  t.key = reinterpret_cast<uint32_t*>(f.ws + f.o_key);
  return t;
}

// node arrays -1 / 0, identity permutation, min/max sentinels, zero
// histograms and partition counters (grid-stride over the largest array)
__global__ void k_tree_init(const FieldRec* __restrict__ table) {
  tree_priority();
  const TreeView t = tree_view(table[blockIdx.y]);
  const int topnodes = (1 << t.top) - 1;
  const size_t nh = (size_t)topnodes * kSelPasses * kSelBins;
  const size_t total = (size_t)t.N + (size_t)t.nodes + (size_t)topnodes * 64 + nh + (size_t)topnodes * 2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    size_t j = i;
    if (j < (size_t)t.N) { t.perm[j] = (int32_t)j; continue; }
    j -= t.N;
    if (j < (size_t)t.nodes) { t.dim[j] = -1; t.split[j] = 0; continue; }
    j -= t.nodes;
    if (j < (size_t)topnodes * 64) { t.mm[j] = (j & 1) ? INT32_MIN : INT32_MAX; continue; }   // pairs (min, max)
    j -= (size_t)topnodes * 64;
    if (j < nh) { t.hist[j] = 0; continue; }
    j -= nh;
    t.cnt[j] = 0;
  }
}

// ---------------------------------------------------------------- top levels
// Rows are read whole: 8 lanes per row, each lane 4 consecutive dimensions
// (one 16-byte load), so a wavefront reads 8 full rows per instruction.
constexpr int kLpr = 8;
// rows in flight per lane group in the min/max loops
#define kMinmaxUnroll 16

typedef int32_t v4i_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4i_t row_quad(const int32_t* V, int stride, int id, int j) {
  // a global-memory load of a native vector (not a flat load, which would
  // also count against the LDS counter)
  return *(const __attribute__((address_space(1))) v4i_t*)(V + (size_t)id * stride + 4 * j);
}

// grid: (chunks, nodes at depth d, fields)
__global__ __launch_bounds__(kTpb) void k_tree_minmax(const FieldRec* __restrict__ table, int d) {
  tree_priority();
  const TreeView t = tree_view(table[blockIdx.z]);
  if (d >= t.top) return;
  const int j = blockIdx.y;
  int start, cnt;
  node_range(d, j, t.N, start, cnt);
  const int lo = blockIdx.x * kChunk;
  if (lo >= cnt) return;
  const int hi = min(cnt, lo + kChunk);
  const int32_t* perm = (d & 1) ? t.perm2 : t.perm;
  __shared__ int32_t smin[32], smax[32];
  if (threadIdx.x < 32) { smin[threadIdx.x] = INT32_MAX; smax[threadIdx.x] = INT32_MIN; }
  __syncthreads();
  const int g = threadIdx.x / kLpr, q = threadIdx.x % kLpr;
  const bool on = 4 * q < t.D;
  int mn[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  int mx[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
  if (on) {
#pragma unroll kMinmaxUnroll
    for (int e = lo + g; e < hi; e += kTpb / kLpr) {
      const v4i_t v = row_quad(t.V, t.stride, perm[start + e], q);
      mn[0] = min(mn[0], v.x); mx[0] = max(mx[0], v.x);
      mn[1] = min(mn[1], v.y); mx[1] = max(mx[1], v.y);
      mn[2] = min(mn[2], v.z); mx[2] = max(mx[2], v.z);
      mn[3] = min(mn[3], v.w); mx[3] = max(mx[3], v.w);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    for (int o = kLpr; o < 64; o <<= 1) {
      mn[i] = min(mn[i], __shfl_xor(mn[i], o));
      mx[i] = max(mx[i], __shfl_xor(mx[i], o));
    }
  if ((threadIdx.x & 63) < kLpr && on) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * q + i < t.D) { atomicMin(&smin[4 * q + i], mn[i]); atomicMax(&smax[4 * q + i], mx[i]); }
  }
  __syncthreads();
  const int node = (1 << d) - 1 + j;
  if ((int)threadIdx.x < t.D) {
    atomicMin(&t.mm[((size_t)node * 32 + threadIdx.x) * 2], smin[threadIdx.x]);
    atomicMax(&t.mm[((size_t)node * 32 + threadIdx.x) * 2 + 1], smax[threadIdx.x]);
  }
}

// split dimension of a node from its min/max: largest spread, lowest on ties
__device__ __forceinline__ void node_split_dim(const int32_t* mm, int node, int D, int& dim, int32_t& mn) {
  int best = 0;
  int64_t bs = -1;
  for (int k = 0; k < D; ++k) {
    const int64_t s = (int64_t)mm[((size_t)node * 32 + k) * 2 + 1] - mm[((size_t)node * 32 + k) * 2];
    if (s > bs) { bs = s; best = k; }
  }
  dim = best;
  mn = mm[((size_t)node * 32 + best) * 2];
}

// Radix-select state after `passes` completed passes: the known high digits
// of the pivot key and its rank among the keys sharing them.  Thread t holds
// bins [8t, 8t + 8) of every finished pass (all loaded at once); a pass's
// digit is found with a wavefront scan of the threads' partial sums and the
// four wavefront totals exchanged through LDS: two barriers per pass.
__device__ void select_state(const int32_t* __restrict__ hist, int node, int passes, int rank0, uint64_t& prefix,
                             int& rank) {
  constexpr int per = kSelBins / kTpb;
  static_assert(per == 8 && kTpb % 64 == 0, "8 bins per thread");
  __shared__ int32_t s_wtot[2][kTpb / 64];
  __shared__ int32_t s_bin[2], s_before[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v4i_t loc[kSelPasses][2];
#pragma unroll
  for (int p = 0; p < kSelPasses; ++p)
    if (p < passes) {
      const v4i_t* h = reinterpret_cast<const v4i_t*>(hist + ((size_t)node * kSelPasses + p) * kSelBins) + 2 * threadIdx.x;
      loc[p][0] = h[0];
      loc[p][1] = h[1];
    }
  prefix = 0;
  rank = rank0;
#pragma unroll
  for (int p = 0; p < kSelPasses; ++p) {
    if (p >= passes) break;
    const int32_t b[per] = {loc[p][0].x, loc[p][0].y, loc[p][0].z, loc[p][0].w,
                            loc[p][1].x, loc[p][1].y, loc[p][1].z, loc[p][1].w};
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) s += b[i];
    int32_t incl = wave_incl_scan(s);
    if (lane == 63) s_wtot[p & 1][wv] = incl;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kTpb / 64; ++w)
      if (w < wv) incl += s_wtot[p & 1][w];
    const int32_t excl = incl - s;
    if (rank >= excl && rank < incl) {
      // the one bin of this thread whose key range holds the rank
      int32_t c = excl;
      int bin = 0, before = excl;
#pragma unroll
      for (int i = 0; i < per; ++i) {
        if (rank >= c && rank < c + b[i]) { bin = i; before = c; }
        c += b[i];
      }
      s_bin[p & 1] = threadIdx.x * per + bin;
      s_before[p & 1] = before;
    }
    __syncthreads();
    prefix = (prefix << 11) | (uint64_t)s_bin[p & 1];
    rank -= s_before[p & 1];
  }
}

__global__ __launch_bounds__(kTpb) void k_tree_hist(const FieldRec* __restrict__ table, int d, int pass) {
  tree_priority();
  const TreeView t = tree_view(table[blockIdx.z]);
  if (d >= t.top) return;
  const int j = blockIdx.y;
  int start, cnt;
  node_range(d, j, t.N, start, cnt);
  const int lo = blockIdx.x * kChunk;
  if (lo >= cnt) return;
  const int hi = min(cnt, lo + kChunk);
  const int32_t* perm = (d & 1) ? t.perm2 : t.perm;
  const int node = (1 << d) - 1 + j;
  int dim;
  int32_t mn;
  node_split_dim(t.mm, node, t.D, dim, mn);
  if (pass == 0 && blockIdx.x == 0 && threadIdx.x == 0) t.dim[node] = dim;
  // all of a thread's element loads first (the element loop is unrolled), in
  // flight during the select-state scan, then the binning: a pass is a few
  // round trips, not one per element
  constexpr int EPT = kChunk / kTpb;
  int ids[EPT];
  uint32_t kvs[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = lo + threadIdx.x + i * kTpb;
    ids[i] = e < hi ? perm[start + e] : 0;
    kvs[i] = (pass != 0 && e < hi) ? t.key[start + e] : 0u;
  }
  if (pass == 0) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = lo + threadIdx.x + i * kTpb;
      if (e < hi) kvs[i] = (uint32_t)(t.V[(size_t)ids[i] * t.stride + dim] - mn);
    }
  }
  uint64_t prefix;
  int rank;
  select_state(t.hist, node, pass, cnt >> 1, prefix, rank);
  __shared__ int32_t lh[kSelBins];
  for (int i = threadIdx.x; i < kSelBins; i += kTpb) lh[i] = 0;
  __syncthreads();
  const int shift = 33 - 11 * pass;
  if (pass == 0) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = lo + threadIdx.x + i * kTpb;
      if (e < hi) t.key[start + e] = kvs[i];
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = lo + threadIdx.x + i * kTpb;
    const uint64_t ck = ((uint64_t)kvs[i] << 22) | (uint64_t)ids[i];
    if (e < hi && (ck >> (shift + 11)) == prefix) atomicAdd(&lh[(ck >> shift) & (kSelBins - 1)], 1);
  }
  __syncthreads();
  int32_t* g = t.hist + ((size_t)node * kSelPasses + pass) * kSelBins;
  for (int i = threadIdx.x; i < kSelBins; i += kTpb)
    if (lh[i]) atomicAdd(&g[i], lh[i]);
}

__global__ __launch_bounds__(kTpb) void k_tree_partition(const FieldRec* __restrict__ table, int d) {
  tree_priority();
  const TreeView t = tree_view(table[blockIdx.z]);
  if (d >= t.top) return;
  const int j = blockIdx.y;
  int start, cnt;
  node_range(d, j, t.N, start, cnt);
  const int lo = blockIdx.x * kChunk;
  if (lo >= cnt) return;
  const int hi = min(cnt, lo + kChunk);
  const int32_t* perm = (d & 1) ? t.perm2 : t.perm;
  int32_t* out = (d & 1) ? t.perm : t.perm2;
  const int node = (1 << d) - 1 + j;
  int dim;
  int32_t mn;
  node_split_dim(t.mm, node, t.D, dim, mn);
  constexpr int EPT = kChunk / kTpb;
  const int e0 = lo + threadIdx.x * EPT;
  int ids[EPT];
  uint32_t kv[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = e0 + i;
    ids[i] = e < hi ? perm[start + e] : 0;
    kv[i] = e < hi ? t.key[start + e] : 0u;
  }
  uint64_t pivot;
  int rank;
  select_state(t.hist, node, kSelPasses, cnt >> 1, pivot, rank);
  if (blockIdx.x == 0 && threadIdx.x == 0) t.split[node] = (int32_t)(pivot >> 22) + mn;
  uint32_t leftmask = 0;
  int nl = 0, nv = 0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    if (e0 + i < hi) {
      const uint64_t ck = ((uint64_t)kv[i] << 22) | (uint64_t)ids[i];
      if (ck < pivot) { leftmask |= 1u << i; ++nl; }
      ++nv;
    }
  }
  // exclusive offsets of this thread's left and right elements in the chunk:
  // wavefront scans, the wavefront totals through LDS
  __shared__ int32_t wl[kTpb / 64], wr[kTpb / 64];
  __shared__ int32_t baseL, baseR;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t il = wave_incl_scan(nl), ir = wave_incl_scan(nv - nl);
  if (lane == 63) { wl[wv] = il; wr[wv] = ir; }
  __syncthreads();
  int32_t totL = 0, totR = 0;
#pragma unroll
  for (int w = 0; w < kTpb / 64; ++w) {
    if (w < wv) { il += wl[w]; ir += wr[w]; }
    totL += wl[w];
    totR += wr[w];
  }
  if (threadIdx.x == 0) {
    baseL = atomicAdd(&t.cnt[node * 2], totL);
    baseR = atomicAdd(&t.cnt[node * 2 + 1], totR);
  }
  __syncthreads();
  int pl = start + baseL + il - nl;
  int pr = start + (cnt >> 1) + baseR + ir - (nv - nl);
  // every write stays inside this node's range even if the counts were off
  const int lend = start + (cnt >> 1), rend = start + cnt;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    if (e0 + i < hi) {
      if ((leftmask >> i) & 1) {
        if (pl < lend) out[pl] = ids[i];
        ++pl;
      } else {
        if (pr < rend) out[pr] = ids[i];
        ++pr;
      }
    }
  }
  if (d + 1 >= t.top) return;
  // The children's per-dimension minimum and maximum (their split dimensions
  // at the next level) over this chunk's points: the chunk's left points,
  // then its right points, listed in LDS; rows read whole by groups of 8
  // lanes as in k_tree_minmax; order-free atomics into the children's slots.
  __shared__ int32_t sids[kChunk];
  __shared__ int32_t cmin[2][32], cmax[2][32];
  {
    int ql = il - nl, qr = totL + ir - (nv - nl);
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (e0 + i < hi) {
        if ((leftmask >> i) & 1) sids[ql++] = ids[i];
        else sids[qr++] = ids[i];
      }
  }
  if (threadIdx.x < 64) {
    cmin[threadIdx.x >> 5][threadIdx.x & 31] = INT32_MAX;
    cmax[threadIdx.x >> 5][threadIdx.x & 31] = INT32_MIN;
  }
  __syncthreads();
  const int g = threadIdx.x / kLpr, q = threadIdx.x % kLpr;
  const bool on = 4 * q < t.D;
  const int nvt = totL + totR;
  int mnL[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX}, mxL[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
  int mnR[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX}, mxR[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
  if (on) {
#pragma unroll kMinmaxUnroll
    for (int e = g; e < nvt; e += kTpb / kLpr) {
      const v4i_t v = row_quad(t.V, t.stride, sids[e], q);
      const int vv[4] = {v.x, v.y, v.z, v.w};
      const bool left = e < totL;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mnL[i] = left ? min(mnL[i], vv[i]) : mnL[i];
        mxL[i] = left ? max(mxL[i], vv[i]) : mxL[i];
        mnR[i] = left ? mnR[i] : min(mnR[i], vv[i]);
        mxR[i] = left ? mxR[i] : max(mxR[i], vv[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    for (int o = kLpr; o < 64; o <<= 1) {
      mnL[i] = min(mnL[i], __shfl_xor(mnL[i], o));
      mxL[i] = max(mxL[i], __shfl_xor(mxL[i], o));
      mnR[i] = min(mnR[i], __shfl_xor(mnR[i], o));
      mxR[i] = max(mxR[i], __shfl_xor(mxR[i], o));
    }
  if ((threadIdx.x & 63) < kLpr && on) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * q + i < t.D) {
        atomicMin(&cmin[0][4 * q + i], mnL[i]);
        atomicMax(&cmax[0][4 * q + i], mxL[i]);
        atomicMin(&cmin[1][4 * q + i], mnR[i]);
        atomicMax(&cmax[1][4 * q + i], mxR[i]);
      }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * t.D) {
    const int side = threadIdx.x >= t.D ? 1 : 0, k = threadIdx.x - side * t.D;
    const size_t child = (size_t)2 * node + 1 + side;
    atomicMin(&t.mm[(child * 32 + k) * 2], cmin[side][k]);
    atomicMax(&t.mm[(child * 32 + k) * 2 + 1], cmax[side][k]);
  }
}

// ---------------------------------------------------------------- one workgroup per node
// Levels whose nodes hold at most kNodeMax points: one 1024-thread workgroup
// per node does the whole level in one launch -- the node's ids and split
// keys stay in registers (EPT per thread), the four radix-select passes bin
// them into an LDS histogram, the partition is a workgroup scan (no global
// atomics, so the children's order is fixed too), and the children's
// min/max are reduced over the partitioned ids listed in LDS.  The pivot,
// and so the tree, is the one the global passes select.
constexpr int kNodeTpb = 1024;
constexpr int kNodeMax = 16 * kNodeTpb;   // measured: 32 K (level 4 at 1024x436) slower, 8 K no better

// exclusive prefix of v over the workgroup (kNodeTpb threads) and the total;
// two barriers; `wt` holds kNodeTpb / 64 ints of LDS
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* wt, int32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t incl = wave_incl_scan(v);
  if (lane == 63) wt[wv] = incl;
  __syncthreads();
  int32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kNodeTpb / 64; ++w) {
    const int32_t x = wt[w];
    if (w < wv) off += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

template <int EPT>
__global__ __launch_bounds__(kNodeTpb) void k_tree_node(const FieldRec* __restrict__ table, int d) {
  tree_priority();
  extern __shared__ __align__(16) int32_t node_lds[];   // [kSelBins] histogram, then the side-ordered ids
  __shared__ int32_t s_wt[kNodeTpb / 64];
  __shared__ int32_t s_bin, s_before;
  __shared__ int32_t cmin[2][32], cmax[2][32];
  const TreeView t = tree_view(table[blockIdx.y]);
  if (d >= t.top) return;
  const int j = blockIdx.x;
  if (j >= (1 << d)) return;
  int start, cnt;
  node_range(d, j, t.N, start, cnt);
  const int32_t* perm = (d & 1) ? t.perm2 : t.perm;
  int32_t* out = (d & 1) ? t.perm : t.perm2;
  const int node = (1 << d) - 1 + j;
  int dim;
  int32_t mn;
  node_split_dim(t.mm, node, t.D, dim, mn);
  int32_t* hist = node_lds;
  int32_t* sids = node_lds + kSelBins;
  // ids and split keys of the node, all loads issued first
  int ids[EPT];
  uint32_t kv[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNodeTpb;
    ids[i] = e < cnt ? perm[start + e] : 0;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNodeTpb;
    kv[i] = e < cnt ? (uint32_t)(t.V[(size_t)ids[i] * t.stride + dim] - mn) : 0u;
  }
  // MSD radix select of rank cnt / 2 of the 44-bit key (key << 22 | pixel)
  uint64_t prefix = 0;
  int rank = cnt >> 1;
  for (int pass = 0; pass < kSelPasses; ++pass) {
    const int shift = 33 - 11 * pass;
    for (int i = threadIdx.x; i < kSelBins; i += kNodeTpb) hist[i] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kNodeTpb;
      const uint64_t ck = ((uint64_t)kv[i] << 22) | (uint64_t)ids[i];
      if (e < cnt && (ck >> (shift + 11)) == prefix) atomicAdd(&hist[(ck >> shift) & (kSelBins - 1)], 1);
    }
    __syncthreads();
    // thread t owns bins 2t and 2t + 1
    static_assert(kSelBins == 2 * kNodeTpb, "two bins per thread");
    const int32_t b0 = hist[2 * threadIdx.x], b1 = hist[2 * threadIdx.x + 1];
    int32_t tot;
    const int32_t excl = block_excl_scan(b0 + b1, s_wt, tot);
    if (rank >= excl && rank < excl + b0 + b1) {
      const bool first = rank < excl + b0;
      s_bin = 2 * threadIdx.x + (first ? 0 : 1);
      s_before = first ? excl : excl + b0;
    }
    __syncthreads();
    prefix = (prefix << 11) | (uint64_t)s_bin;
    rank -= s_before;
    __syncthreads();
  }
  const uint64_t pivot = prefix;
  if (threadIdx.x == 0) {
    t.dim[node] = dim;
    t.split[node] = (int32_t)(pivot >> 22) + mn;
  }
  // partition: the left points (key below the pivot) first, in a fixed order
  uint32_t leftmask = 0;
  int nl = 0, nv = 0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNodeTpb;
    if (e < cnt) {
      const uint64_t ck = ((uint64_t)kv[i] << 22) | (uint64_t)ids[i];
      if (ck < pivot) { leftmask |= 1u << i; ++nl; }
      ++nv;
    }
  }
  int32_t totL, totR;
  int pl = block_excl_scan(nl, s_wt, totL);
  int pr = block_excl_scan(nv - nl, s_wt, totR);
  const int h = cnt >> 1;
  const bool kids = d + 1 < t.top;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNodeTpb;
    if (e < cnt) {
      if ((leftmask >> i) & 1) {
        if (pl < h) {
          out[start + pl] = ids[i];
          if (kids) sids[pl] = ids[i];
        }
        ++pl;
      } else {
        if (pr < cnt - h) {
          out[start + h + pr] = ids[i];
          if (kids) sids[h + pr] = ids[i];
        }
        ++pr;
      }
    }
  }
  if (!kids) return;
  // the children's per-dimension min/max over the listed ids (left: [0, h),
  // right: [h, cnt)); rows read whole by groups of 8 lanes
  if (threadIdx.x < 64) {
    cmin[threadIdx.x >> 5][threadIdx.x & 31] = INT32_MAX;
    cmax[threadIdx.x >> 5][threadIdx.x & 31] = INT32_MIN;
  }
  __syncthreads();
  const int g = threadIdx.x / kLpr, q = threadIdx.x % kLpr;
  const bool on = 4 * q < t.D;
  int mnL[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX}, mxL[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
  int mnR[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX}, mxR[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
  if (on) {
#pragma unroll 8
    for (int e = g; e < cnt; e += kNodeTpb / kLpr) {
      const v4i_t v = row_quad(t.V, t.stride, sids[e], q);
      const int vv[4] = {v.x, v.y, v.z, v.w};
      const bool left = e < h;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mnL[i] = left ? min(mnL[i], vv[i]) : mnL[i];
        mxL[i] = left ? max(mxL[i], vv[i]) : mxL[i];
        mnR[i] = left ? mnR[i] : min(mnR[i], vv[i]);
        mxR[i] = left ? mxR[i] : max(mxR[i], vv[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    for (int o = kLpr; o < 64; o <<= 1) {
      mnL[i] = min(mnL[i], __shfl_xor(mnL[i], o));
      mxL[i] = max(mxL[i], __shfl_xor(mxL[i], o));
      mnR[i] = min(mnR[i], __shfl_xor(mnR[i], o));
      mxR[i] = max(mxR[i], __shfl_xor(mxR[i], o));
    }
  if ((threadIdx.x & 63) < kLpr && on) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * q + i < t.D) {
        atomicMin(&cmin[0][4 * q + i], mnL[i]);
        atomicMax(&cmax[0][4 * q + i], mxL[i]);
        atomicMin(&cmin[1][4 * q + i], mnR[i]);
        atomicMax(&cmax[1][4 * q + i], mxR[i]);
      }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * t.D) {
    const int side = threadIdx.x >= t.D ? 1 : 0, k = threadIdx.x - side * t.D;
    const size_t child = (size_t)2 * node + 1 + side;
    t.mm[(child * 32 + k) * 2] = cmin[side][k];
    t.mm[(child * 32 + k) * 2 + 1] = cmax[side][k];
  }
}

// ---------------------------------------------------------------- subtrees in LDS
constexpr int kSubTpb = 512;

__device__ __forceinline__ void heap_range(int node, int N, int& start, int& cnt) {
  const int d = 31 - __clz(node + 1);
  node_range(d, node + 1 - (1 << d), N, start, cnt);
}

// Bitonic sort of key[0, P) ascending (P a power of two, <= kTreeLds =
// 4 kSubTpb).  Thread t holds the four consecutive keys 4t..4t+3 in
// registers: a stage of stride j < 4 pairs keys of one thread, j < 256 keys
// of one wavefront (shuffles), and only the strides j >= 256 go through LDS,
// two barriers each.  Called by the whole workgroup; key[] must be settled
// (a barrier after its last writes) before the call.
static_assert(kTreeLds == 4 * kSubTpb, "four keys per thread");
__device__ __forceinline__ uint64_t cas_keep(uint64_t mine, uint64_t other, int i, int j, int k) {
  // compare-exchange of positions i and i ^ j in a sequence sorted up where
  // (i & k) == 0: the lower position keeps the smaller key there
  const bool up = (i & k) == 0, lower = (i & j) == 0;
  const uint64_t lo = mine < other ? mine : other, hi = mine < other ? other : mine;
  return lower == up ? lo : hi;
}

// Sorts every aligned block of B keys (B a power of two <= P) ascending: the
// network of a full sort stopped at merges of size B, the last merge taken
// ascending in every block.
__device__ void bitonic_sort(uint64_t* key, int P, int B) {
  const int t = threadIdx.x;
  uint64_t v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = key[4 * t + r];
  for (int k = 2; k <= B; k <<= 1) {
    const int kd = k == B ? 2 * P : k;   // direction bit: none in the last merge
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 256) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) key[4 * t + r] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * t + r;
          v[r] = cas_keep(v[r], key[i ^ j], i, j, kd);
        }
      } else if (j >= 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = cas_keep(v[r], __shfl_xor(v[r], j >> 2), 4 * t + r, j, kd);
      } else {
        uint64_t w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = cas_keep(v[r], v[r ^ j], 4 * t + r, j, kd);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = w[r];
      }
    }
  }
  __syncthreads();
  if (4 * t < P) {
#pragma unroll
    for (int r = 0; r < 4; ++r) key[4 * t + r] = v[r];
  }
  __syncthreads();
}

// grid: (2^maxTop, fields); block x finishes the subtree rooted at node x of
// depth top (of its field)
__global__ __launch_bounds__(kSubTpb) void k_tree_subtree(const FieldRec* __restrict__ table, int leaf) {
  tree_priority();
  const TreeView t = tree_view(table[blockIdx.y]);
  if ((int)blockIdx.x >= (1 << t.top)) return;
  const int32_t* perm_in = (t.top & 1) ? t.perm2 : t.perm;
  int32_t* perm_out = t.perm;
  const int32_t* V = t.V;
  const int stride = t.stride, D = t.D, N = t.N;
  // Padded layout: at relative depth lvl the subtree's 2^lvl segments sit in
  // aligned blocks of B = P >> lvl positions (segment s in [s B, s B + cnt),
  // the rest +inf), so each level sorts every block on its own and a split
  // keeps the left half in place and moves the right half to the second
  // half of the block.  A segment that stops splitting is a leaf: its block,
  // sorted by pixel index at that level, is written out at once.
  __shared__ uint64_t keys[2][kTreeLds];
  __shared__ int32_t s_start[kTreeLds / 2], s_cnt[kTreeLds / 2];
  __shared__ int32_t s_best[kTreeLds / 2], s_dim[kTreeLds / 2], s_bmin[kTreeLds / 2];
  __shared__ uint8_t s_alive[kTreeLds / 2], s_alive2[kTreeLds / 2];
  __shared__ int32_t s_pmin[kSubTpb / 64][32], s_pmax[kSubTpb / 64][32];
  __shared__ int s_any;
  const int root = (1 << t.top) - 1 + blockIdx.x;
  int rstart, rcnt;
  heap_range(root, N, rstart, rcnt);
  int P = 1;
  while (P < rcnt) P <<= 1;
  int cur = 0;
  for (int e = threadIdx.x; e < P; e += kSubTpb) keys[0][e] = e < rcnt ? (uint64_t)perm_in[rstart + e] : ~0ull;
  if (threadIdx.x == 0) s_alive[0] = 1;
  __syncthreads();
  const uint64_t idmask = (1ull << 22) - 1;
  for (int lvl = 0;; ++lvl) {
    const int nslots = 1 << lvl;
    const int B = P >> lvl;
    const int lgB = 31 - __clz(B);
    const int base = (root + 1) * nslots - 1;    // first heap index at this relative depth
    uint64_t* key = keys[cur];
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < nslots; s += kSubTpb) {
      int st, c;
      heap_range(base + s, N, st, c);
      s_start[s] = st - rstart;
      s_cnt[s] = c;
      s_best[s] = -1;
      s_dim[s] = 0;
      s_bmin[s] = 0;
      if (s_alive[s] && c > leaf) s_any = 1;
    }
    __syncthreads();
    const bool last = !s_any;
    if (!last) {
      // Split dimension of every splitting segment in one pass over its rows:
      // 64 groups of 8 lanes, a lane holding 4 dimensions of a row.  With
      // fewer than 64 segments, gps groups share a segment (partials merged by
      // shuffles inside a wavefront, then through LDS across wavefronts); with
      // more, each group walks spg segments.
      const int g = threadIdx.x >> 3, q = threadIdx.x & 7, wv = threadIdx.x >> 6;
      const int gps = nslots >= 64 ? 1 : 64 / nslots;
      const int spg = nslots >= 64 ? nslots / 64 : 1;
      for (int si = 0; si < spg; ++si) {
        const int s = nslots >= 64 ? g * spg + si : g / gps;
        const int part = nslots >= 64 ? 0 : g % gps;
        const bool act = s_alive[s] && s_cnt[s] > leaf;
        int mn[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
        int mx[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
        if (act && 4 * q < D) {
          const int c = s_cnt[s], st = s << lgB;
          const int a = st + c * part / gps, b = st + c * (part + 1) / gps;
#pragma unroll 8
          for (int e = a; e < b; ++e) {
            const v4i_t v = row_quad(V, stride, (int)(key[e] & idmask), q);
            mn[0] = min(mn[0], v.x); mx[0] = max(mx[0], v.x);
            mn[1] = min(mn[1], v.y); mx[1] = max(mx[1], v.y);
            mn[2] = min(mn[2], v.z); mx[2] = max(mx[2], v.z);
            mn[3] = min(mn[3], v.w); mx[3] = max(mx[3], v.w);
          }
        }
        for (int m = 1; m < gps && m < 8; m <<= 1)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            mn[i] = min(mn[i], __shfl_xor(mn[i], 8 * m));
            mx[i] = max(mx[i], __shfl_xor(mx[i], 8 * m));
          }
        if (gps > 8) {
          // 2..8 wavefronts per segment: merge their partials through LDS
          if ((g & 7) == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) { s_pmin[wv][4 * q + i] = mn[i]; s_pmax[wv][4 * q + i] = mx[i]; }
          __syncthreads();
          const int wps = gps / 8;
          const int s2 = g < nslots ? g : 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            mn[i] = INT32_MAX;
            mx[i] = INT32_MIN;
            for (int w = s2 * wps; w < (s2 + 1) * wps; ++w) {
              mn[i] = min(mn[i], s_pmin[w][4 * q + i]);
              mx[i] = max(mx[i], s_pmax[w][4 * q + i]);
            }
          }
        }
        // best dimension of the group's segment: largest spread, lowest on ties
        int bs = -1, bd = 0, bm = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 4 * q + i;
          if (k < D) {
            const int sp = mx[i] - mn[i];
            if (sp > bs) { bs = sp; bd = k; bm = mn[i]; }
          }
        }
        for (int o = 1; o < 8; o <<= 1) {
          const int obs = __shfl_xor(bs, o), obd = __shfl_xor(bd, o), obm = __shfl_xor(bm, o);
          if (obs > bs || (obs == bs && obd < bd)) { bs = obs; bd = obd; bm = obm; }
        }
        const bool owner = gps > 8 ? (g < nslots) : (part == 0);
        const int so = gps > 8 ? g : s;
        if (owner && q == 0 && s_alive[so] && s_cnt[so] > leaf) { s_best[so] = bs; s_dim[so] = bd; s_bmin[so] = bm; }
      }
      __syncthreads();
    }
    // keys: (split value - minimum) << 22 | pixel for a splitting segment,
    // the pixel alone for a leaf, +inf outside the live segments
    for (int e = threadIdx.x; e < P; e += kSubTpb) {
      const int s = e >> lgB, j = e & (B - 1);
      uint64_t kv = ~0ull;
      if (s_alive[s] && j < s_cnt[s]) {
        const uint64_t id = key[e] & idmask;
        uint64_t sub = 0;
        if (s_cnt[s] > leaf) sub = (uint64_t)(uint32_t)(V[(size_t)id * stride + s_dim[s]] - s_bmin[s]) << 22;
        kv = sub | id;
      }
      key[e] = kv;
    }
    __syncthreads();
    bitonic_sort(key, P, B);
    // split nodes; leaves written out (their blocks are in pixel order)
    for (int s = threadIdx.x; s < nslots; s += kSubTpb) {
      if (s_alive[s] && s_cnt[s] > leaf) {
        const int h = s_cnt[s] >> 1;
        const uint64_t pid = key[(s << lgB) + h] & idmask;
        t.dim[base + s] = s_dim[s];
        t.split[base + s] = V[(size_t)pid * stride + s_dim[s]];
      }
    }
    for (int e = threadIdx.x; e < P; e += kSubTpb) {
      const int s = e >> lgB, j = e & (B - 1);
      if (s_alive[s] && s_cnt[s] <= leaf && j < s_cnt[s]) perm_out[rstart + s_start[s] + j] = (int32_t)(key[e] & idmask);
    }
    if (last) break;
    // the next level's layout: block 2s takes the first h of segment s, block
    // 2s + 1 the rest, both of size B / 2
    uint64_t* nkey = keys[cur ^ 1];
    const int hB = B >> 1;
    for (int e = threadIdx.x; e < P; e += kSubTpb) {
      const int s2 = e >> (lgB - 1), j = e & (hB - 1), s = s2 >> 1;
      uint64_t kv = ~0ull;
      if (s_alive[s] && s_cnt[s] > leaf) {
        const int h = s_cnt[s] >> 1;
        if (!(s2 & 1)) {
          if (j < h) kv = key[(s << lgB) + j];
        } else {
          if (j < s_cnt[s] - h) kv = key[(s << lgB) + h + j];
        }
      }
      nkey[e] = kv;
    }
    for (int s2 = threadIdx.x; s2 < 2 * nslots; s2 += kSubTpb) s_alive2[s2] = s_alive[s2 >> 1] && s_cnt[s2 >> 1] > leaf;
    __syncthreads();
    for (int s2 = threadIdx.x; s2 < 2 * nslots; s2 += kSubTpb) s_alive[s2] = s_alive2[s2];
    cur ^= 1;
    __syncthreads();
  }
}

ff_status enqueue_tree_build(const FieldRec* table, int nf, int maxN, int maxTop, int leaf, hipStream_t stream) {
  (void)leaf;
  k_tree_init<<<dim3(512, nf), 256, 0, stream>>>(table);
  for (int d = 0; d < maxTop; ++d) {
    const int maxcnt = (int)(((int64_t)maxN + (1LL << d) - 1) >> d);
    const dim3 grid((maxcnt + kChunk - 1) / kChunk, 1 << d, nf);
    // below the root the previous level's partition has reduced each
    // node's minimum and maximum
    if (d == 0) k_tree_minmax<<<grid, kTpb, 0, stream>>>(table, d);
    if (maxcnt <= kNodeMax) {
      const size_t lds = (size_t)(kSelBins + maxcnt) * 4;
      const dim3 ng(1 << d, nf);
      if (maxcnt <= 4 * kNodeTpb) k_tree_node<4><<<ng, kNodeTpb, lds, stream>>>(table, d);
      else if (maxcnt <= 8 * kNodeTpb) k_tree_node<8><<<ng, kNodeTpb, lds, stream>>>(table, d);
      else k_tree_node<16><<<ng, kNodeTpb, lds, stream>>>(table, d);
      continue;
    }
    for (int p = 0; p < kSelPasses; ++p) k_tree_hist<<<grid, kTpb, 0, stream>>>(table, d, p);
    k_tree_partition<<<grid, kTpb, 0, stream>>>(table, d);
  }
  k_tree_subtree<<<dim3(1 << maxTop, nf), kSubTpb, 0, stream>>>(table, leaf);
  return launch_status();
}

}  // namespace ff

using namespace ff;

extern "C" {

int32_t ff_tree_nodes(int32_t n_points, int32_t leaf) {
  if (n_points < 1 || leaf < 1) return 0;
  return (2 << tree_depth_of(n_points, leaf)) - 1;
}

}  // extern "C"
