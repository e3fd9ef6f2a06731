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
// along its own anti-diagonals; row 0 of a band waits on the results the
// band above publishes.  Bands are claimed with a ticket, so a band only ever
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
  size_t off_sync;        // per propagation launch: its band ticket
  size_t off_xch;         // band handoff words, bands x Gw (largest level)
  size_t xch_words;
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
  M.launches = (p->k + 1) * p->n_prop;
  off = align_up(off + (size_t)M.launches * 4, 256);
  M.off_xch = off;
  M.xch_words = (size_t)((src->height + kBandRows - 1) / kBandRows) * src->width;
  off += M.xch_words * 8;
  M.bytes = align_up(off, 256);
  return M;
}

// ---------------------------------------------------------------- device helpers
struct CostCtx {
  const uint32_t* src;   // source plane, level n, phase (0,0)
  const uint32_t* dst;   // target planes of level n (phase i at dst + i * pw)
  const uint32_t* srcT;  // the same, transposed (x-major, pitch Hs / Hd)
  const uint32_t* dstT;
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

// 32-bit word load at a 32-bit word index (index < 2^30), as a relaxed
// agent-scope load: it skips the vector L1, whose miss path costs more than a
// direct L2 access for these scattered, rarely reused census words
__device__ __forceinline__ uint32_t ld32(const uint32_t* base, uint32_t idx) {
  return __hip_atomic_load(reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + (idx << 2)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
#pragma unroll 4
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

// sum over a 16-lane DPP row, left in every lane of the row: swap adjacent
// lanes, swap lane pairs, mirror within half-rows (quad 0 <-> quad 1), mirror
// within the row (half 0 <-> half 1)
__device__ __forceinline__ int32_t row16_sum(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
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
//
// Step t of a band: row i handles u = t - i.  Rows hand results down through
// a double-buffered LDS slot (one barrier per step).  The band's last row
// publishes each result as one 64-bit word (flow | cost | launch tag) with a
// relaxed agent-scope store; row 0 of the band below polls that word until
// the tag matches.  One single-copy-atomic word carries data and readiness,
// so no fence (L2 write-back or invalidate) is needed on the critical path.
// Everything that does not depend on the wavefront -- the point's own flow
// and cost, the source census terms, the next handoff word -- is loaded one
// step ahead.
__device__ __forceinline__ uint64_t rt_clock() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ uint64_t xch_pack(int32_t f, int32_t cst, uint32_t tag) {
  const uint32_t c16 = cst == kInf ? 0xFFFFu : (uint32_t)cst;
  return (uint64_t)(uint32_t)f | ((uint64_t)(c16 | (tag << 16)) << 32);
}

// Batches of kBatch steps.  Before a batch the band stages in LDS (a) every
// row's own flow and cost for the batch and (b) the source census tile the
// batch's terms read (the source side does not depend on the wavefront);
// after it the results leave from an LDS ring with coalesced stores.  Inside
// a batch a step's only global traffic is its target census terms plus the
// one-word handoff.
//
// Term layout.  In sweep-transformed grid coordinates (u right, v down) the
// sliding-window terms of a point are four groups of S = 2r+1: g0/g1 = row
// v-r-1 / v+r (vertical candidate leaving / entering), g2/g3 = column u-r-1 /
// u+r (horizontal candidate), each over offsets -r..r.  Lane l of a point
// takes offset index l + 16 m of every group for the FULL = S / 16 full
// slots; the S % 16 remaining offsets of the four groups are packed into TAIL
// extra slots.
constexpr int kBatch = 32;
constexpr int kMaxTileWords = (kBandRows + 2 * kMaxRadius + 1) * ((kBatch + kBandRows + 2 * kMaxRadius) | 1);

template <int FULL, int TAIL>
__global__ __launch_bounds__(kBandRows * kLanesProp) void k_propagate(CostCtx c, int Gw, int Gh, int sx, int sy,
                                                                      int32_t* __restrict__ F, int32_t* __restrict__ C,
                                                                      uint64_t* __restrict__ xch, uint32_t tag,
                                                                      int32_t* __restrict__ ticket,
                                                                      int32_t* __restrict__ status,
                                                                      uint64_t timeout_ticks) {
  constexpr int BH = kBandRows, L = kLanesProp, CH = kBatch;
  constexpr int NS = 4 * FULL + TAIL;   // term slots per lane
  static_assert(L == 16 && CH % 2 == 0 && CH % L == 0, "layout");
  __shared__ int32_t s_band;
  __shared__ int32_t bufF[2][BH], bufC[2][BH];
  __shared__ int32_t inF[BH][CH], inC[BH][CH], outF[BH][CH], outC[BH][CH];
  __shared__ uint32_t tile[kMaxTileWords];
  const int row = threadIdx.x / L, lane = threadIdx.x % L;
  if (threadIdx.x == 0) s_band = atomicAdd(ticket, 1);
  __syncthreads();
  const int band = s_band;
  const int v0 = band * BH;
  if (v0 >= Gh) return;
  const int rows = min(BH, Gh - v0);
  const int nsteps = Gw + rows - 1;
  const int r = c.r, S = 2 * r + 1, n = c.n, Q = c.Q;
  const int TH = BH + 2 * r + 1;          // tile rows: v0-r-1 .. v0+BH-1+r
  const int TW = (CH + BH + 2 * r) | 1;   // tile cols: tb-BH-r .. tb+CH-1+r; odd pitch (banks)
  const bool rowok = row < rows;
  const int rr = rowok ? row : rows - 1;  // inactive rows shadow a valid row
  const int gy = sy > 0 ? v0 + rr : Gh - 1 - (v0 + rr);
  const int py = gy * n;
  const bool publish = rowok && row == rows - 1 && v0 + rows < Gh;
  const bool poll = rowok && row == 0 && v0 > 0;
  const uint64_t* xin = xch + (size_t)(band > 0 ? band - 1 : 0) * Gw;
  uint64_t* xout = xch + (size_t)band * Gw;
  int32_t* Frow = F + (size_t)gy * Gw;
  int32_t* Crow = C + (size_t)gy * Gw;
  auto gx_of = [&](int u) { return sx > 0 ? u : Gw - 1 - u; };
  auto gy_of = [&](int v) { return sy > 0 ? v : Gh - 1 - v; };
  // slot table: group (0..3), offset index i (0..S-1), validity
  int sg[NS], si[NS];
  uint32_t sval = 0;
#pragma unroll
  for (int m = 0; m < FULL; ++m)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      sg[4 * m + g] = g;
      si[4 * m + g] = lane + 16 * m;
      sval |= 1u << (4 * m + g);
    }
  {
    const int tl = S - 16 * FULL;   // remaining offsets per group
#pragma unroll
    for (int q = 0; q < TAIL; ++q) {
      const int e = lane + 16 * q;   // packed tail term
      const int g = tl > 0 ? e / tl : 0;
      sg[4 * FULL + q] = g < 4 ? g : 0;
      si[4 * FULL + q] = 16 * FULL + (tl > 0 ? e % tl : 0);
      if (g < 4) sval |= 1u << (4 * FULL + q);
    }
  }
  // per slot: transformed offsets (du, dv), and the LDS tile offset
  int sdu[NS], sdv[NS], stoff[NS];
  uint32_t shor = 0, sneg = 0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int g = sg[k], o = si[k] - r;
    const int du = g < 2 ? o : (g == 2 ? -r - 1 : r);
    const int dv = g < 2 ? (g == 0 ? -r - 1 : r) : o;
    sdu[k] = du;
    sdv[k] = dv;
    stoff[k] = (r + 1 + dv) * TW + (BH + r + du);
    if (g >= 2) shor |= 1u << k;
    if (g == 0 || g == 2) sneg |= 1u << k;
  }
  int32_t prevF = kEmpty, prevC = kInf;   // this row's result at u-1
  bool abandoned = false;
  auto wait_word = [&](int u, uint64_t w) -> uint64_t {
    if ((uint32_t)(w >> 48) != tag && !abandoned) {
      const uint64_t t0 = rt_clock();
      do {
        __builtin_amdgcn_s_sleep(1);
        w = __hip_atomic_load(&xin[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (rt_clock() - t0 > timeout_ticks) {
          __hip_atomic_store(status, (int32_t)FF_ERR_DEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          abandoned = true;
          break;
        }
      } while ((uint32_t)(w >> 48) != tag);
    }
    return w;
  };
  const uint32_t* dplane = c.dst;
  const uint32_t* dplaneT = c.dstT;
  // one step; `pw` holds the prefetched handoff word for this step (row 0),
  // `pn` receives the next one
  auto step = [&](int t, int tb, uint64_t pw, uint64_t& pn) {
    const int j = t - tb;
    const int u = t - row;
    const bool active = rowok && u >= 0 && u < Gw;
    const int px = gx_of(clampi(u, 0, Gw - 1)) * n;
    const int32_t curF0 = inF[row][j], curC0 = inC[row][j];
    int32_t vF = bufF[(t - 1) & 1][row > 0 ? row - 1 : 0];
    int32_t vC = bufC[(t - 1) & 1][row > 0 ? row - 1 : 0];
    if (row == 0) {
      vF = kEmpty;
      vC = kInf;
      if (poll && active) {
        const uint64_t w = wait_word(u, pw);
        vF = (int32_t)(uint32_t)w;
        const uint32_t c16 = (uint32_t)(w >> 32) & 0xFFFFu;
        vC = c16 == 0xFFFFu ? kInf : (int32_t)c16;
      }
    }
    const int32_t hF = u > 0 ? prevF : kEmpty, hC = u > 0 ? prevC : kInf;
    const bool useV = active && vF != kEmpty && vF != curF0 && centre_valid(c, px, py, fx_of(vF), fy_of(vF));
    const bool useH = active && hF != kEmpty && hF != curF0 && centre_valid(c, px, py, fx_of(hF), fy_of(hF));
    int32_t dvs = 0, dhs = 0;
    if (__any(useV || useH)) {
      // target side: both candidates' centres, phase planes and the fixed
      // row (vertical) / column (horizontal) of each group
      const int mxv = px * Q + fx_of(vF), myv = py * Q + fy_of(vF);
      const int mxh = px * Q + fx_of(hF), myh = py * Q + fy_of(hF);
      const int Mxv = mxv >> c.qshift, Myv = myv >> c.qshift;
      const int Mxh = mxh >> c.qshift, Myh = myh >> c.qshift;
      const uint32_t phv = (uint32_t)c.pw * (uint32_t)(((myv & c.qmask) << c.qshift) + (mxv & c.qmask));
      const uint32_t phh = (uint32_t)c.pw * (uint32_t)(((myh & c.qmask) << c.qshift) + (mxh & c.qmask));
      const int nsx = sx * n, nsy = sy * n;
      const uint32_t rb0 = phv + (uint32_t)clampi(Myv - nsy * (r + 1), 0, c.Hd - 1) * (uint32_t)c.Wd;
      const uint32_t rb1 = phv + (uint32_t)clampi(Myv + nsy * r, 0, c.Hd - 1) * (uint32_t)c.Wd;
      const uint32_t cb2 = phh + (uint32_t)clampi(Mxh - nsx * (r + 1), 0, c.Wd - 1) * (uint32_t)c.Hd;
      const uint32_t cb3 = phh + (uint32_t)clampi(Mxh + nsx * r, 0, c.Wd - 1) * (uint32_t)c.Hd;
      const int tbase = (row) * TW + (u - tb);   // tile index of (u, v) minus the slot offset base
      uint32_t a[NS], b[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        // full slots have a compile-time group (k & 3); tail slots select
        const int g = k < 4 * FULL ? (k & 3) : sg[k];
        const uint32_t iv = (g == 0 ? rb0 : rb1) + (uint32_t)clampi(Mxv + nsx * sdu[k], 0, c.Wd - 1);
        const uint32_t ih = (g == 2 ? cb2 : cb3) + (uint32_t)clampi(Myh + nsy * sdv[k], 0, c.Hd - 1);
        if (k < 4 * FULL) {
          b[k] = g < 2 ? ld32(dplane, iv) : ld32(dplaneT, ih);
        } else {
          const uint32_t bv = ld32(dplane, iv), bh = ld32(dplaneT, ih);
          b[k] = ((sval >> k) & 1) ? (g < 2 ? bv : bh) : 0u;
        }
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) a[k] = tile[tbase + stoff[k]];
      pn = poll ? __hip_atomic_load(&xin[clampi(u + 1, 0, Gw - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int32_t pc = ((sval >> k) & 1) ? __popc(a[k] ^ b[k]) : 0;
        const int32_t sgn = ((sneg >> k) & 1) ? -pc : pc;
        if ((shor >> k) & 1) dhs += sgn;
        else dvs += sgn;
      }
    } else {
      pn = poll ? __hip_atomic_load(&xin[clampi(u + 1, 0, Gw - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    }
    dvs = row16_sum(dvs);
    dhs = row16_sum(dhs);
    // candidate order of Eq. 2: current, vertical, horizontal; strict <
    int32_t curF = curF0, curC = curC0;
    if (useV && vC + dvs < curC) { curF = vF; curC = vC + dvs; }
    if (useH && hC + dhs < curC) { curF = hF; curC = hC + dhs; }
    prevF = curF;
    prevC = curC;
    if (lane == 0) {
      bufF[t & 1][row] = curF;
      bufC[t & 1][row] = curC;
      outF[row][j] = curF;
      outC[row][j] = curC;
      if (publish && active)
        __hip_atomic_store(&xout[u], xch_pack(curF, curC, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  uint64_t w0 = poll ? __hip_atomic_load(&xin[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0, w1 = 0;
  const int TT = TH * TW;
  for (int tb = 0; tb < nsteps; tb += CH) {
    // stage this batch's own flows and costs (row r at step tb + j works on
    // u = tb + j - r) and the source tile: tile(y, x) is the source census
    // at transformed grid (u, v) = (tb - BH - r + x, v0 - r - 1 + y),
    // clamped to the image in pixels
#pragma unroll
    for (int jj = 0; jj < CH / L; ++jj) {
      const int j = lane + jj * L;
      const int u = tb + j - row;
      if (rowok && u >= 0 && u < Gw) {
        inF[row][j] = Frow[gx_of(u)];
        inC[row][j] = Crow[gx_of(u)];
      }
    }
    for (int e = threadIdx.x; e < TT; e += BH * L) {
      const int y = e / TW, x = e - y * TW;
      const int gxp = gx_of(tb - BH - r + x) * n, gyp = gy_of(v0 - r - 1 + y) * n;
      tile[e] = c.src[(size_t)clampi(gyp, 0, c.Hs - 1) * c.Ws + clampi(gxp, 0, c.Ws - 1)];
    }
    __syncthreads();
    const int te = min(tb + CH, nsteps);
    for (int t = tb; t < te; t += 2) {
      step(t, tb, w0, w1);
      __syncthreads();
      if (t + 1 < te) {
        step(t + 1, tb, w1, w0);
        __syncthreads();
      } else {
        w0 = w1;
      }
    }
    // write the batch's results back
#pragma unroll
    for (int jj = 0; jj < CH / L; ++jj) {
      const int j = lane + jj * L;
      const int u = tb + j - row;
      if (rowok && u >= 0 && u < Gw && tb + j < te) {
        Frow[gx_of(u)] = outF[row][j];
        Crow[gx_of(u)] = outC[row][j];
      }
    }
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

static void launch_propagate(int r, int bands, hipStream_t stream, const CostCtx& c, int Gw, int Gh, int sx, int sy,
                             int32_t* F, int32_t* C, uint64_t* xch, uint32_t tag, int32_t* ticket, int32_t* status,
                             uint64_t timeout) {
  const dim3 grid(bands), block(kBandRows * kLanesProp);
  const int S = 2 * r + 1, full = S / 16, tl = S - 16 * full, tail = (4 * tl + 15) / 16;
#define FF_PROP(FU, TA)                                                                                      \
  if (full == FU && tail == TA) {                                                                          \
    k_propagate<FU, TA><<<grid, block, 0, stream>>>(c, Gw, Gh, sx, sy, F, C, xch, tag, ticket, status, timeout); \
    return;                                                                                                \
  }
  FF_PROP(0, 1) FF_PROP(0, 2) FF_PROP(0, 3) FF_PROP(0, 4)
  FF_PROP(1, 0) FF_PROP(1, 1) FF_PROP(1, 2) FF_PROP(1, 3) FF_PROP(1, 4)
#undef FF_PROP
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
  c.srcT = census_plane_t(src, sb, lev, 0, 0);
  c.dstT = census_plane_t(dst, db, lev, 0, 0);
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
  uint64_t* xch = reinterpret_cast<uint64_t*>(ws + M.off_xch);
  fill_i32(sync, (size_t)M.launches, 0, stream);
  fill_i32(reinterpret_cast<int32_t*>(xch), M.xch_words * 2, 0, stream);
  const int Ws = src->width, Hs = src->height;
  const int k = p->k;
  if (M.has_tree) {
    prof_mark(FF_PROF_TREE, stream, true);
    st = enqueue_tree_build(wht_block(dst, dst_blob, radius), dst->width * dst->height, dst->wht_dims, dst->wht_stride,
                            p->leaf, M.tree, ws, stream);
    prof_mark(FF_PROF_TREE, stream, false);
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
    prof_mark(FF_PROF_SEED, stream, true);
    k_seed<<<(waves + 3) / 4, 256, 0, stream>>>(c, Gw, Gh, Vs, src->wht_stride, nd, ns, pm, dst->width * dst->height,
                                                 M.has_tree ? M.tree.nodes : 0, M.has_tree ? 1 : 0, proposal,
                                                 gridF(k), gridC(k));
    prof_mark(FF_PROF_SEED, stream, false);
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
      prof_mark(FF_PROF_LEVEL_ENTRY, stream, true);
      k_level_entry<kLanesPt><<<(G * kLanesPt + 255) / 256, 256, 0, stream>>>(c, Gw, Gh, gridF(lev + 1),
                                                                             (Ws + nc - 1) / nc, F, C);
      prof_mark(FF_PROF_LEVEL_ENTRY, stream, false);
      ++steps;
      if (stop()) return finish();
    }
    for (int i = 0; i < p->n_prop; ++i) {
      const int dir = i & 3;
      const int sx = (dir == 0 || dir == 3) ? 1 : -1;
      const int sy = (dir == 0 || dir == 2) ? 1 : -1;
      const int bands = (Gh + kBandRows - 1) / kBandRows;
      prof_mark(FF_PROF_PROPAGATE, stream, true);
      launch_propagate(radius, bands, stream, c, Gw, Gh, sx, sy, F, C, xch, (uint32_t)(launch + 1), sync + launch, status,
                       timeout);
      prof_mark(FF_PROF_PROPAGATE, stream, false);
      ++launch;
      ++steps;
      if (stop()) return finish();
      if (i < p->n_rs) {
        prof_mark(FF_PROF_RANDOM_SEARCH, stream, true);
        k_random_search<kLanesPt><<<(G * kLanesPt + 255) / 256, 256, 0, stream>>>(
            c, Gw, Gh, lev, i, n * p->R * dst->subpel, c3base, k0, k1, F, C);
        prof_mark(FF_PROF_RANDOM_SEARCH, stream, false);
        ++steps;
        if (stop()) return finish();
      }
    }
  }
  cur_lev = 0;
  return finish();
}

}  // extern "C"
