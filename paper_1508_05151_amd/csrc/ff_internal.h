// Internal declarations shared by the translation units of libff (HIP for
// gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ff.h"

namespace ff {

constexpr int32_t kEmpty = FF_EMPTY;
constexpr int32_t kInf = FF_COST_INF;
constexpr int kMaxPoints = 1 << 22;   // pixel index fits 22 bits
constexpr int kMaxDim = 8191;         // packed int16 flows at Q = 4 (|f| <= 32767)
constexpr int kMaxRadius = 15;
constexpr int kMaxLeaf = 64;

// ---------------------------------------------------------------- helpers
__host__ __device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__host__ __device__ inline int fx_of(int32_t f) { return (int)(int16_t)(uint16_t)((uint32_t)f & 0xFFFFu); }
__host__ __device__ inline int fy_of(int32_t f) { return (int)(int16_t)(uint16_t)((uint32_t)f >> 16); }
__host__ __device__ inline int32_t packf(int dx, int dy) {
  return (int32_t)(((uint32_t)(uint16_t)(int16_t)dy << 16) | (uint32_t)(uint16_t)(int16_t)dx);
}
__host__ __device__ inline int ilog2i(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------- kd-tree
// Levels whose nodes hold more than kTreeLds points are split by global
// radix-select passes; below that, one workgroup finishes each subtree in LDS.
constexpr int kTreeLds = 2048;
constexpr int kSelBins = 2048;        // 11-bit digits, 4 passes over 44 bits
constexpr int kSelPasses = 4;

struct TreeLayout {
  int N, depth, nodes;   // nodes = (2 << depth) - 1
  int top;               // levels handled by the global passes
  size_t off_dim, off_split, off_perm, off_perm2, off_minmax, off_hist, off_cnt, off_key;
  size_t bytes;
};
TreeLayout tree_layout(int N, int leaf, size_t base);
int tree_depth_of(int N, int leaf);

// Device record of one field of a match call (src -> dst, patch radius r).
// Kernels of every stage read it, so one launch serves all fields of a batch.
struct FieldRec {
  const uint32_t* src;   // source census planes (level 0, phase 0); level l at + l Q^2 pws
  const uint32_t* srcT;  // the same, transposed
  const uint32_t* dst;   // target census planes
  const uint32_t* dstT;
  const int32_t* Vsrc;   // WHT vectors of this radius (tree queries / tree keys)
  const int32_t* Vdst;
  const int32_t* proposal;
  int32_t* flow;         // outputs (also the level-1 grid)
  int32_t* cost;
  char* ws;              // this field's workspace region
  uint32_t pws, pwd;     // plane words of source / target
  int32_t Ws, Hs, Wd, Hd;
  int32_t r, D, vstride, pad0;
  uint32_t k0, k1, c3, pad1;
  // kd-tree over the target (offsets into ws)
  int32_t t_nodes, t_top, pad2, pad3;
  uint32_t o_dim, o_split, o_perm, o_perm2, o_mm, o_hist, o_cnt, o_key;
  // level grids n = 2..2^k (flow then cost), the band handoff words of the
  // first and of the second sweep of a launch, and the column-progress words
  // of a pipelined sweep pair (two arrays)
  uint32_t o_grid[5];
  uint32_t o_xch;
  uint32_t o_xch2, o_prog;
};

// Enqueue the kd-tree builds of `nf` fields whose records are in `table`
// (device).  maxN / maxTop bound the launch geometry.
ff_status enqueue_tree_build(const FieldRec* table, int nf, int maxN, int maxTop, int leaf, hipStream_t stream);

// ---------------------------------------------------------------- descriptors
inline const uint32_t* census_plane(const ff_desc* d, const void* blob, int lev, int a, int b) {
  return reinterpret_cast<const uint32_t*>(static_cast<const char*>(blob) + d->off_census +
                                           d->plane_bytes * ((size_t)lev * d->subpel * d->subpel + b * d->subpel + a));
}
inline const uint32_t* census_plane_t(const ff_desc* d, const void* blob, int lev, int a, int b) {
  return reinterpret_cast<const uint32_t*>(static_cast<const char*>(blob) + d->off_census_t +
                                           d->plane_bytes * ((size_t)lev * d->subpel * d->subpel + b * d->subpel + a));
}
inline const int32_t* wht_block(const ff_desc* d, const void* blob, int radius) {
  for (int i = 0; i < d->n_radii; ++i)
    if (d->radii[i] == radius)
      return reinterpret_cast<const int32_t*>(static_cast<const char*>(blob) + d->off_wht +
                                              (size_t)i * d->width * d->height * d->wht_stride * 4);
  return nullptr;
}

// SIFT colour levels (section 3.3 smoothed as section 3.2): scratch bytes
// and the enqueue (ff_desc.hip holds the Lanczos table)
size_t sift_levels_scratch_bytes(int W, int H, int S);
void enqueue_sift_levels(const int16_t* codes, int W, int H, int S, int P, int k, int16_t* levels, int32_t* scratch,
                         hipStream_t stream);

ff_status ensure_init();
ff_status launch_status();   // maps hipGetLastError to FF_ERR_HIP

// fill a device int32 buffer with a value (graph-safe: a kernel, no memset)
void fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t s);

// device address of the current device's no-allocation scratch array
// (looked up once per device; out may be null to only do the lookup)
ff_status noalloc_scratch(char** out);

}  // namespace ff

namespace ff {
// Profiling hook: when a kernel class is armed with ff_profile_begin, each
// launch (or launch sequence) of that class is bracketed by two events on its
// stream.  prof_mark is a no-op otherwise.
void prof_mark(int kernel_class, hipStream_t stream, bool start);
}  // namespace ff
