// The Flow Field search of one field (sections 3.1, 3.2): kd-tree seeds on
// the coarsest grid, then per level the alternating propagation sweeps and
// random searches, coarse flows seeding the next level.
//
// Data term E^n_r(p, f) (Eq. 1/3/4 with the census of section 3.3): the sum
// over the (2r+1)^2 samples at stride n of popcount(D1 ^ D2), D1 from the
// source's phase-(0,0) plane of level n at p + n d, D2 from the target's
// plane of the subpixel phase of m = pQ + f at floor(m/Q) + n d; lookups
// clamp to the image; f is invalid ("infinite") unless m lies in the image.
//
// Propagation (Eq. 2) keeps the raster-order dependencies exactly with an
// anti-diagonal wavefront: a workgroup owns a band of BH grid rows and steps
// along its own anti-diagonals; row 0 of a band waits on the band above's
// progress counter.  Bands are claimed with a ticket, so a band only ever
// waits on a band that started before it.  Propagated candidates are costed
// with sliding windows: E(p, F(q)) = C(q) - (row or column leaving the patch)
// + (row or column entering it), 2(2r+1) terms instead of (2r+1)^2, exact
// because every sample lookup clamps per coordinate.
#include "ff_internal.h"

namespace ff {

constexpr int kBandRows = 16;     // BH: grid rows per propagation workgroup
constexpr int kLanesProp = 16;    // lanes per point in the propagation sweep
constexpr int kLanesPt = 16;      // lanes per point in recost / random search
constexpr int kStatusBytes = 256;

// ---------------------------------------------------------------- layout
struct MatchLayout {
  TreeLayout tree;
  bool has_tree;
  size_t off_grid[5];     // per level 1..k: flow then cost (level 0 = outputs)
  size_t off_sync;        // per propagation launch: ticket + progress per band
  int sync_stride;        // ints per launch
  int launches;
  size_t bytes;
};

static MatchLayout match_layout(const ff_desc* src, const ff_desc* dst, const ff_match_params* p) {
  MatchLayout M{};
  size_t off = kStatusBytes;
  M.has_tree = p->use_kdtree != 0;
  if (M.has_tree) {
    M.tree = tree_layout(dst->width * dst->height, p->leaf, off);
    off += M.tree.bytes;
  }
  for (int lev = 1; lev <= p->k; ++lev) {
    const int n = 1 << lev;
    const size_t G = (size_t)((src->width + n - 1) / n) * ((src->height + n - 1) / n);
    off = align_up(off, 256);
    M.off_grid[lev] = off;
    off += G * 8;
  }
  off = align_up(off, 256);
  M.off_sync = off;
  M.sync_stride = 1 + (src->height + kBandRows - 1) / kBandRows + 1;
  M.launches = (p->k + 1) * p->n_prop;
  off += (size_t)M.sync_stride * M.launches * 4;
  M.bytes = align_up(off, 256);
  return M;
}

// ---------------------------------------------------------------- device helpers
struct CostCtx {
  const uint32_t* src;   // source plane, level n, phase (0,0)
  const uint32_t* dst;   // target planes of level n (phase i at dst + i * pw)
  size_t pw;
  int Ws, Hs, Wd, Hd;
  int qshift, qmask, Q;
  int n, r;
};

// Philox4x32-10 (Salmon et al., SC 2011): 10 rounds of the two multiplier
// S-boxes with Weyl-sequence key schedule.  Returns the first two words.
__device__ __forceinline__ void philox2(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                        uint32_t& o0, uint32_t& o1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  o0 = c0;
  o1 = c1;
}

__device__ __forceinline__ bool centre_valid(const CostCtx& c, int px, int py, int fx, int fy) {
  const int mx = px * c.Q + fx, my = py * c.Q + fy;
  return mx >= 0 && my >= 0 && mx <= (c.Wd - 1) * c.Q && my <= (c.Hd - 1) * c.Q;
}

// partial patch sum over this lane's share (terms lane, lane+L, ...)
__device__ __forceinline__ int32_t patch_partial(const CostCtx& c, int px, int py, int fx, int fy, int lane, int L) {
  const int mx = px * c.Q + fx, my = py * c.Q + fy;
  const int Mx = mx >> c.qshift, My = my >> c.qshift;
  const uint32_t* D2 = c.dst + c.pw * (size_t)(((my & c.qmask) << c.qshift) + (mx & c.qmask));
  const int S = 2 * c.r + 1;
  int dy = lane / S, dx = lane - dy * S;
  const int stepy = L / S, stepx = L - stepy * S;
  int32_t sum = 0;
  for (int t = lane; t < S * S; t += L) {
    const int oy = (dy - c.r) * c.n, ox = (dx - c.r) * c.n;
    const uint32_t a = c.src[(size_t)clampi(py + oy, 0, c.Hs - 1) * c.Ws + clampi(px + ox, 0, c.Ws - 1)];
    const uint32_t b = D2[(size_t)clampi(My + oy, 0, c.Hd - 1) * c.Wd + clampi(Mx + ox, 0, c.Wd - 1)];
    sum += __popc(a ^ b);
    dx += stepx;
    dy += stepy;
    if (dx >= S) { dx -= S; ++dy; }
  }
  return sum;
}

template <int L>
__device__ __forceinline__ int32_t group_sum(int32_t v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
  return v;
}

// ---------------------------------------------------------------- seeds (Eq. 1 / Eq. 4)
// One wavefront per coarse grid point: descend the kd-tree with the source
// patch's WHT vector, then re-rank the leaf (ascending pixel index) and the
// optional proposal by the data term; the first minimum wins.
__global__ __launch_bounds__(256) void k_seed(CostCtx c, int Gw, int Gh, const int32_t* __restrict__ Vsrc, int vstride,
                                              const int32_t* __restrict__ node_dim, const int32_t* __restrict__ node_split,
                                              const int32_t* __restrict__ perm, int Nd, int n_nodes, int use_tree,
                                              const int32_t* __restrict__ proposal, int32_t* __restrict__ F,
                                              int32_t* __restrict__ C) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= Gw * Gh) return;
  const int gx = wave % Gw, gy = wave / Gw;
  const int px = gx * c.n, py = gy * c.n;
  int32_t bestF = kEmpty, bestC = kInf;
  if (use_tree) {
    const int32_t* q = Vsrc + ((size_t)py * c.Ws + px) * vstride;
    int node = 0, start = 0, cnt = Nd;
    for (;;) {
      const int dim = node_dim[node];
      if (dim < 0 || 2 * node + 2 >= n_nodes) break;
      const int h = cnt >> 1;
      if (q[dim] >= node_split[node]) { node = 2 * node + 2; start += h; cnt -= h; }
      else { node = 2 * node + 1; cnt = h; }
    }
    for (int i = 0; i < cnt && start + i < Nd; ++i) {
      const int id = perm[start + i];
      const int fx = (id % c.Wd - px) * c.Q, fy = (id / c.Wd - py) * c.Q;
      const int32_t e = group_sum<64>(patch_partial(c, px, py, fx, fy, lane, 64));
      if (e < bestC) { bestC = e; bestF = packf(fx, fy); }
    }
  }
  if (proposal) {
    const int32_t fp = proposal[(size_t)gy * Gw + gx];
    if (fp != kEmpty && centre_valid(c, px, py, fx_of(fp), fy_of(fp))) {
      const int32_t e = group_sum<64>(patch_partial(c, px, py, fx_of(fp), fy_of(fp), lane, 64));
      if (e < bestC) { bestC = e; bestF = fp; }
    }
  }
  if (lane == 0) {
    F[(size_t)gy * Gw + gx] = bestF;
    C[(size_t)gy * Gw + gx] = bestC;
  }
}

// ---------------------------------------------------------------- level entry
// Section 3.2: points of the coarser grid keep their flow and are re-costed
// with this level's patch; new points start empty.
template <int L>
__global__ __launch_bounds__(256) void k_level_entry(CostCtx c, int Gw, int Gh, const int32_t* __restrict__ Fc,
                                                     int Gwc, int32_t* __restrict__ F, int32_t* __restrict__ C) {
  const int pid = (blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int lane = threadIdx.x % L;
  if (pid >= Gw * Gh) return;
  const int gx = pid % Gw, gy = pid / Gw;
  int32_t f = kEmpty, e = kInf;
  if (!(gx & 1) && !(gy & 1)) {
    f = Fc[(size_t)(gy >> 1) * Gwc + (gx >> 1)];
    if (f != kEmpty) e = group_sum<L>(patch_partial(c, gx * c.n, gy * c.n, fx_of(f), fy_of(f), lane, L));
  }
  if (lane == 0) {
    F[pid] = f;
    C[pid] = e;
  }
}

// ---------------------------------------------------------------- random search
// Section 3.1 / 3.2: one uniform offset per point, per axis an integer in
// [-nRQ, nRQ] 1/Q px, from Philox keyed by the seed with counter (pixel, level,
// step, field | pair << 2); replace only on a strictly lower cost.
template <int L>
__global__ __launch_bounds__(256) void k_random_search(CostCtx c, int Gw, int Gh, int lev, int step, int rad,
                                                       uint32_t c3, uint32_t k0, uint32_t k1, int32_t* __restrict__ F,
                                                       int32_t* __restrict__ C) {
  const int pid = (blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int lane = threadIdx.x % L;
  if (pid >= Gw * Gh) return;
  const int32_t f = F[pid];
  if (f == kEmpty) return;
  const int gx = pid % Gw, gy = pid / Gw;
  const int px = gx * c.n, py = gy * c.n;
  uint32_t u0, u1;
  philox2((uint32_t)(py * c.Ws + px), (uint32_t)lev, (uint32_t)step, c3, k0, k1, u0, u1);
  const uint64_t span = (uint64_t)(2 * rad + 1);
  const int ox = (int)((u0 * span) >> 32) - rad;
  const int oy = (int)((u1 * span) >> 32) - rad;
  const int fx = fx_of(f) + ox, fy = fy_of(f) + oy;
  if (!centre_valid(c, px, py, fx, fy)) return;
  const int32_t e = group_sum<L>(patch_partial(c, px, py, fx, fy, lane, L));
  if (lane == 0 && e < C[pid]) {
    F[pid] = packf(fx, fy);
    C[pid] = e;
  }
}

// ---------------------------------------------------------------- propagation (Eq. 2)
// Sweep direction (sx, sy): 1: (+,+), 2: (-,-), 3: (-,+), 4: (+,-); the
// predecessors of a point lie at -sx (horizontal) and -sy (vertical).  In
// the transformed coordinates u = sx > 0 ? gx : Gw-1-gx (same for v) every
// sweep runs right and down.
__device__ __forceinline__ uint64_t rt_clock() { return __builtin_amdgcn_s_memrealtime(); }

__global__ __launch_bounds__(kBandRows * kLanesProp) void k_propagate(CostCtx c, int Gw, int Gh, int sx, int sy,
                                                                      int32_t* __restrict__ F, int32_t* __restrict__ C,
                                                                      int32_t* __restrict__ sync, int32_t* __restrict__ status,
                                                                      uint64_t timeout_ticks) {
  constexpr int BH = kBandRows, L = kLanesProp;
  __shared__ int32_t s_band;
  __shared__ int32_t bufF[2][BH], bufC[2][BH];
  const int row = threadIdx.x / L, lane = threadIdx.x % L;
  if (threadIdx.x == 0) s_band = atomicAdd(&sync[0], 1);
  __syncthreads();
  const int band = s_band;
  const int v0 = band * BH;
  if (v0 >= Gh) return;
  const int rows = min(BH, Gh - v0);
  int32_t* progress = sync + 1;
  const int nsteps = Gw + rows - 1;
  const int S = 2 * c.r + 1;
  const int Q = c.Q;
  const int vv = v0 + row;
  const int gy = sy > 0 ? vv : Gh - 1 - vv;
  const int py = gy * c.n;
  // term assignment of this lane: groups 0/1 = row leaving / entering for the
  // vertical candidate, 2/3 = column leaving / entering for the horizontal
  const int crv = -sy * (c.r + 1), cav = sy * c.r;
  const int crh = -sx * (c.r + 1), cah = sx * c.r;
  int32_t prevF = kEmpty, prevC = kInf;   // this row's result at u-1
  bool abandoned = false;
  for (int t = 0; t < nsteps; ++t) {
    const int u = t - row;
    const bool active = row < rows && u >= 0 && u < Gw;
    if (active) {
      const int gx = sx > 0 ? u : Gw - 1 - u;
      const int px = gx * c.n;
      const size_t pidx = (size_t)gy * Gw + gx;
      int32_t curF = F[pidx], curC = C[pidx];
      // vertical predecessor
      int32_t vF = kEmpty, vC = kInf;
      if (row > 0) {
        vF = bufF[(t - 1) & 1][row - 1];
        vC = bufC[(t - 1) & 1][row - 1];
      } else if (v0 > 0) {
        const int need = t + BH;
        int32_t got = __hip_atomic_load(&progress[band - 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (got < need && !abandoned) {
          const uint64_t t0 = rt_clock();
          while (got < need) {
            __builtin_amdgcn_s_sleep(1);
            got = __hip_atomic_load(&progress[band - 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (rt_clock() - t0 > timeout_ticks) {
              __hip_atomic_store(status, (int32_t)FF_ERR_DEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              abandoned = true;
              break;
            }
          }
        }
        const int gyq = sy > 0 ? v0 - 1 : Gh - v0;
        const size_t qidx = (size_t)gyq * Gw + gx;
        vF = __hip_atomic_load(&F[qidx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        vC = __hip_atomic_load(&C[qidx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const int32_t hF = u > 0 ? prevF : kEmpty, hC = u > 0 ? prevC : kInf;
      const bool useV = vF != kEmpty && vF != curF && centre_valid(c, px, py, fx_of(vF), fy_of(vF));
      const bool useH = hF != kEmpty && hF != curF && centre_valid(c, px, py, fx_of(hF), fy_of(hF));
      int32_t dv = 0, dh = 0;
      if (useV || useH) {
        // target positions and phase planes of both candidates
        const int mxv = px * Q + fx_of(vF), myv = py * Q + fy_of(vF);
        const int mxh = px * Q + fx_of(hF), myh = py * Q + fy_of(hF);
        const uint32_t* D2v = c.dst + c.pw * (size_t)(((myv & c.qmask) << c.qshift) + (mxv & c.qmask));
        const uint32_t* D2h = c.dst + c.pw * (size_t)(((myh & c.qmask) << c.qshift) + (mxh & c.qmask));
        const int Mxv = mxv >> c.qshift, Myv = myv >> c.qshift;
        const int Mxh = mxh >> c.qshift, Myh = myh >> c.qshift;
        for (int tt = lane; tt < 4 * S; tt += L) {
          const int g = tt / S;
          const int o = (tt - g * S - c.r) * c.n;
          if (g < 2) {
            if (!useV) continue;
            const int cy = (g == 0 ? crv : cav) * c.n;
            const uint32_t a = c.src[(size_t)clampi(py + cy, 0, c.Hs - 1) * c.Ws + clampi(px + o, 0, c.Ws - 1)];
            const uint32_t b = D2v[(size_t)clampi(Myv + cy, 0, c.Hd - 1) * c.Wd + clampi(Mxv + o, 0, c.Wd - 1)];
            const int32_t pc = __popc(a ^ b);
            dv += g == 0 ? -pc : pc;
          } else {
            if (!useH) continue;
            const int cx = (g == 2 ? crh : cah) * c.n;
            const uint32_t a = c.src[(size_t)clampi(py + o, 0, c.Hs - 1) * c.Ws + clampi(px + cx, 0, c.Ws - 1)];
            const uint32_t b = D2h[(size_t)clampi(Myh + o, 0, c.Hd - 1) * c.Wd + clampi(Mxh + cx, 0, c.Wd - 1)];
            const int32_t pc = __popc(a ^ b);
            dh += g == 2 ? -pc : pc;
          }
        }
      }
      dv = group_sum<L>(dv);
      dh = group_sum<L>(dh);
      // candidate order of Eq. 2: current, vertical, horizontal; strict <
      if (useV && vC + dv < curC) { curF = vF; curC = vC + dv; }
      if (useH && hC + dh < curC) { curF = hF; curC = hC + dh; }
      prevF = curF;
      prevC = curC;
      if (lane == 0) {
        bufF[t & 1][row] = curF;
        bufC[t & 1][row] = curC;
        if (row == rows - 1 && v0 + rows < Gh) {
          // the band below reads this row: agent-coherent stores, then publish
          __hip_atomic_store(&F[pidx], curF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&C[pidx], curC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&progress[band], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          F[pidx] = curF;
          C[pidx] = curC;
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_write_grid(const int32_t* __restrict__ Fg, const int32_t* __restrict__ Cg, int Gw, int n, int W, int H,
                             int32_t* __restrict__ F, int32_t* __restrict__ C) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  const size_t o = (size_t)y * W + x;
  if ((x % n) == 0 && (y % n) == 0) {
    F[o] = Fg[(size_t)(y / n) * Gw + x / n];
    C[o] = Cg[(size_t)(y / n) * Gw + x / n];
  } else {
    F[o] = kEmpty;
    C[o] = kInf;
  }
}

static ff_status check_params(const ff_desc* src, const ff_desc* dst, int radius, const ff_match_params* p) {
  if (!src || !dst || !p) return FF_ERR_ARG;
  if (src->channels != dst->channels || src->subpel != dst->subpel) return FF_ERR_ARG;
  if (p->k < 0 || p->k > src->k || p->k > dst->k) return FF_ERR_ARG;
  if (radius < 1 || radius > kMaxRadius) return FF_ERR_ARG;
  if (p->R < 0 || p->R > 64 || p->n_prop < 0 || p->n_prop > 64 || p->n_rs < 0 || p->n_rs > p->n_prop) return FF_ERR_ARG;
  if (p->field_id > 3) return FF_ERR_ARG;
  if (p->use_kdtree) {
    if (p->leaf < 2 || p->leaf > kMaxLeaf) return FF_ERR_ARG;
    bool hs = false, hd = false;
    for (int i = 0; i < src->n_radii; ++i) hs |= src->radii[i] == radius;
    for (int i = 0; i < dst->n_radii; ++i) hd |= dst->radii[i] == radius;
    if (!hs || !hd) return FF_ERR_ARG;
  }
  return FF_OK;
}

static CostCtx make_ctx(const ff_desc* src, const void* sb, const ff_desc* dst, const void* db, int lev, int r) {
  CostCtx c;
  c.src = census_plane(src, sb, lev, 0, 0);
  c.dst = census_plane(dst, db, lev, 0, 0);
  c.pw = (size_t)dst->width * dst->height;
  c.Ws = src->width;
  c.Hs = src->height;
  c.Wd = dst->width;
  c.Hd = dst->height;
  c.Q = dst->subpel;
  c.qshift = ilog2i(dst->subpel);
  c.qmask = dst->subpel - 1;
  c.n = 1 << lev;
  c.r = r;
  return c;
}

}  // namespace ff

using namespace ff;

extern "C" {

void ff_default_params(ff_match_params* p) {
  if (!p) return;
  *p = ff_match_params{};
  p->k = 3;
  p->R = 1;
  p->leaf = 8;
  p->n_prop = 4;
  p->n_rs = 3;
  p->use_kdtree = 1;
  p->max_steps = -1;
}

size_t ff_match_workspace_bytes(const ff_desc* src, const ff_desc* dst, int32_t radius, const ff_match_params* p) {
  if (check_params(src, dst, radius, p) != FF_OK) return 0;
  return match_layout(src, dst, p).bytes;
}

ff_status ff_read_status(const void* workspace, int32_t* status_host) {
  if (!workspace || !status_host) return FF_ERR_ARG;
  if (hipMemcpy(status_host, workspace, 4, hipMemcpyDeviceToHost) != hipSuccess) return FF_ERR_HIP;
  return FF_OK;
}

ff_status ff_build_kdtree(const ff_desc* d, const void* blob, int32_t radius, int32_t leaf, int32_t* node_dim,
                          int32_t* node_split, int32_t* perm, void* workspace, size_t workspace_bytes,
                          hipStream_t stream) {
  if (!d || !blob || !node_dim || !node_split || !perm || !workspace) return FF_ERR_ARG;
  if (leaf < 2 || leaf > kMaxLeaf) return FF_ERR_ARG;
  const int32_t* V = wht_block(d, blob, radius);
  if (!V) return FF_ERR_ARG;
  const int N = d->width * d->height;
  TreeLayout L = tree_layout(N, leaf, kStatusBytes);
  if (workspace_bytes < kStatusBytes + L.bytes) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  char* ws = static_cast<char*>(workspace);
  st = enqueue_tree_build(V, N, d->wht_dims, d->wht_stride, leaf, L, ws, stream);
  if (st != FF_OK) return st;
  if (hipMemcpyAsync(node_dim, ws + L.off_dim, (size_t)L.nodes * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(node_split, ws + L.off_split, (size_t)L.nodes * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(perm, ws + L.off_perm, (size_t)N * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return FF_ERR_HIP;
  return FF_OK;
}

ff_status ff_match_field(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                         int32_t radius, const ff_match_params* p, const int32_t* proposal, int32_t* flow,
                         int32_t* cost, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  ff_status st = check_params(src, dst, radius, p);
  if (st != FF_OK) return st;
  if (!src_blob || !dst_blob || !flow || !cost || !workspace) return FF_ERR_ARG;
  if (!p->use_kdtree && !proposal) return FF_ERR_ARG;
  const MatchLayout M = match_layout(src, dst, p);
  if (workspace_bytes < M.bytes) return FF_ERR_WORKSPACE;
  st = ensure_init();
  if (st != FF_OK) return st;
  char* ws = static_cast<char*>(workspace);
  int32_t* status = reinterpret_cast<int32_t*>(ws);
  int32_t* sync = reinterpret_cast<int32_t*>(ws + M.off_sync);
  fill_i32(status, 1, 0, stream);
  fill_i32(sync, (size_t)M.sync_stride * M.launches, 0, stream);
  const int Ws = src->width, Hs = src->height;
  const int k = p->k;
  if (M.has_tree) {
    st = enqueue_tree_build(wht_block(dst, dst_blob, radius), dst->width * dst->height, dst->wht_dims, dst->wht_stride,
                            p->leaf, M.tree, ws, stream);
    if (st != FF_OK) return st;
  }
  auto gridF = [&](int lev) -> int32_t* {
    return lev == 0 ? flow : reinterpret_cast<int32_t*>(ws + M.off_grid[lev]);
  };
  auto gridC = [&](int lev) -> int32_t* {
    if (lev == 0) return cost;
    const int n = 1 << lev;
    const size_t G = (size_t)((Ws + n - 1) / n) * ((Hs + n - 1) / n);
    return reinterpret_cast<int32_t*>(ws + M.off_grid[lev]) + G;
  };
  int steps = 0;
  int cur_lev = k;
  auto stop = [&]() { return p->max_steps >= 0 && steps >= p->max_steps; };
  auto finish = [&]() -> ff_status {
    if (cur_lev > 0) {
      const int n = 1 << cur_lev;
      k_write_grid<<<dim3((Ws + 255) / 256, Hs), 256, 0, stream>>>(gridF(cur_lev), gridC(cur_lev), (Ws + n - 1) / n, n,
                                                                   Ws, Hs, flow, cost);
    }
    return launch_status();
  };
  {
    const CostCtx c = make_ctx(src, src_blob, dst, dst_blob, k, radius);
    const int n = 1 << k;
    const int Gw = (Ws + n - 1) / n, Gh = (Hs + n - 1) / n;
    const int32_t* Vs = M.has_tree ? wht_block(src, src_blob, radius) : nullptr;
    const int32_t* nd = M.has_tree ? reinterpret_cast<const int32_t*>(ws + M.tree.off_dim) : nullptr;
    const int32_t* ns = M.has_tree ? reinterpret_cast<const int32_t*>(ws + M.tree.off_split) : nullptr;
    const int32_t* pm = M.has_tree ? reinterpret_cast<const int32_t*>(ws + M.tree.off_perm) : nullptr;
    const int waves = Gw * Gh;
    k_seed<<<(waves + 3) / 4, 256, 0, stream>>>(c, Gw, Gh, Vs, src->wht_stride, nd, ns, pm, dst->width * dst->height,
                                                 M.has_tree ? M.tree.nodes : 0, M.has_tree ? 1 : 0, proposal,
                                                 gridF(k), gridC(k));
  }
  ++steps;
  if (stop()) return finish();
  const uint32_t c3base = p->field_id | (p->pair_id << 2);
  const uint32_t k0 = (uint32_t)(p->seed & 0xFFFFFFFFu), k1 = (uint32_t)(p->seed >> 32);
  // watchdog for the propagation's inter-band waits: 2 s of the 100 MHz
  // constant clock
  const uint64_t timeout = 200000000ull;
  int launch = 0;
  for (int lev = k; lev >= 0; --lev) {
    cur_lev = lev;
    const int n = 1 << lev;
    const int Gw = (Ws + n - 1) / n, Gh = (Hs + n - 1) / n;
    const CostCtx c = make_ctx(src, src_blob, dst, dst_blob, lev, radius);
    int32_t* F = gridF(lev);
    int32_t* C = gridC(lev);
    const int G = Gw * Gh;
    if (lev < k) {
      const int nc = n * 2;
      k_level_entry<kLanesPt><<<(G * kLanesPt + 255) / 256, 256, 0, stream>>>(c, Gw, Gh, gridF(lev + 1),
                                                                             (Ws + nc - 1) / nc, F, C);
      ++steps;
      if (stop()) return finish();
    }
    for (int i = 0; i < p->n_prop; ++i) {
      const int dir = i & 3;
      const int sx = (dir == 0 || dir == 3) ? 1 : -1;
      const int sy = (dir == 0 || dir == 2) ? 1 : -1;
      const int bands = (Gh + kBandRows - 1) / kBandRows;
      k_propagate<<<bands, kBandRows * kLanesProp, 0, stream>>>(c, Gw, Gh, sx, sy, F, C,
                                                               sync + (size_t)launch * M.sync_stride, status, timeout);
      ++launch;
      ++steps;
      if (stop()) return finish();
      if (i < p->n_rs) {
        k_random_search<kLanesPt><<<(G * kLanesPt + 255) / 256, 256, 0, stream>>>(
            c, Gw, Gh, lev, i, n * p->R * dst->subpel, c3base, k0, k1, F, C);
        ++steps;
        if (stop()) return finish();
      }
    }
  }
  cur_lev = 0;
  return finish();
}

}  // extern "C"
