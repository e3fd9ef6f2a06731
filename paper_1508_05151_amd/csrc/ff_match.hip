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
#include <algorithm>
#include <mutex>
#include <vector>

#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

constexpr int kLanesProp = 16;    // lanes per point in the propagation sweep
constexpr int kLanesPt = 16;      // lanes per point in recost / random search
constexpr int kStatusBytes = 256;
constexpr int kMinBandRows = 8;   // smallest band height (sizes the handoff buffer)
constexpr int kRecsPerWrite = 16; // table records per writer launch (kernel argument size)
// words per pipelined-progress array: covers ceil(Gh / BH) * BH / 4 random-
// search workgroups of any band height up to 32 at any level
__host__ __device__ __forceinline__ int prog_words(int Hs) { return (Hs + 31) / 4 + 8; }

// ---------------------------------------------------------------- per-field cost context
struct CostCtx {
  const uint32_t* src;   // source plane, level n, phase (0,0)
  const uint32_t* dst;   // target planes of level n (phase i at dst + i * pw)
  const uint32_t* srcT;  // the same, transposed (x-major, pitch Hs / Hd)
  const uint32_t* dstT;
  uint32_t pw;           // target plane words
  int Ws, Hs, Wd, Hd;
  int qshift, qmask, Q;
  int n, r;
};

__device__ __forceinline__ CostCtx ctx_of(const FieldRec& f, int lev, int qshift) {
  CostCtx c;
  const int Q = 1 << qshift;
  c.src = f.src + (size_t)lev * Q * Q * f.pws;
  c.srcT = f.srcT + (size_t)lev * Q * Q * f.pws;
  c.dst = f.dst + (size_t)lev * Q * Q * f.pwd;
  c.dstT = f.dstT + (size_t)lev * Q * Q * f.pwd;
  c.pw = f.pwd;
  c.Ws = f.Ws;
  c.Hs = f.Hs;
  c.Wd = f.Wd;
  c.Hd = f.Hd;
  c.Q = Q;
  c.qshift = qshift;
  c.qmask = Q - 1;
  c.n = 1 << lev;
  c.r = f.r;
  return c;
}

// level grids: n = 1 is the output pair itself
__device__ __forceinline__ int32_t* grid_flow(const FieldRec& f, int lev) {
  return lev == 0 ? f.flow : reinterpret_cast<int32_t*>(f.ws + f.o_grid[lev]);
}
__device__ __forceinline__ int32_t* grid_cost(const FieldRec& f, int lev, int G) {
  return lev == 0 ? f.cost : reinterpret_cast<int32_t*>(f.ws + f.o_grid[lev]) + G;
}

__device__ __forceinline__ bool centre_valid(const CostCtx& c, int px, int py, int fx, int fy) {
  const int mx = px * c.Q + fx, my = py * c.Q + fy;
  return mx >= 0 && my >= 0 && mx <= (c.Wd - 1) * c.Q && my <= (c.Hd - 1) * c.Q;
}

// partial patch sum over this lane's share (terms lane, lane+L, ...)
__device__ __forceinline__ int32_t patch_partial(const CostCtx& c, int px, int py, int fx, int fy, int lane, int L) {
  const int mx = px * c.Q + fx, my = py * c.Q + fy;
  const int Mx = mx >> c.qshift, My = my >> c.qshift;
  const uint32_t* D2 = c.dst + (size_t)c.pw * (size_t)(((my & c.qmask) << c.qshift) + (mx & c.qmask));
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

// Census distance of two S x S patches at stride 1 by a group of 16 lanes
// (partial sums, one per lane): lane l < min(S, 16) sums patch column l over
// all S rows, so each load of a wavefront reads 64 consecutive bytes per
// point rather than one row segment per lane; column 16 (S = 17) spreads its
// rows over the lanes.  Each side is given as the address of the patch's
// column 0 in plane row 0 (sb, tb), its row pitch in words and the plane row
// of patch row 0 (sy0, ty0); rows clamp to [0, ymax], columns are not
// clamped, so the caller guarantees that both S-word row segments lie inside
// their planes.  INSIDE: the source rows never clamp (sy0 = 0, symax = S - 1)
// and a patch whose target rows all lie inside skips the clamps (kept out of
// the sweep kernel, whose register count it would raise).
// Measured against one row per lane (16-byte loads): random search 55.6 ->
// 51.9 us per launch, pair 10.13 -> 10.02 ms.
typedef __attribute__((address_space(1))) const uint32_t g_u32;

template <int S, bool INSIDE, typename SP>
__device__ __forceinline__ int32_t cols_sum_n1(SP sb, int spw, int sy0, int symax, g_u32* tb, int tpw, int ty0,
                                               int tymax, int lane) {
  int32_t sum = 0;
  if (INSIDE && ty0 >= 0 && ty0 + S - 1 <= tymax) {
    g_u32* t0 = tb + ty0 * tpw;
    if (lane < S) {
#pragma unroll
      for (int row = 0; row < S; ++row) sum += __popc(sb[row * spw + lane] ^ t0[row * tpw + lane]);
    }
    for (int row = lane; S > 16 && row < S; row += 16) sum += __popc(sb[row * spw + 16] ^ t0[row * tpw + 16]);
    return sum;
  }
  if (lane < S) {
#pragma unroll
    for (int row = 0; row < S; ++row)
      sum += __popc(sb[clampi(sy0 + row, 0, symax) * spw + lane] ^ tb[clampi(ty0 + row, 0, tymax) * tpw + lane]);
  }
  for (int row = lane; S > 16 && row < S; row += 16)
    sum += __popc(sb[clampi(sy0 + row, 0, symax) * spw + 16] ^ tb[clampi(ty0 + row, 0, tymax) * tpw + 16]);
  return sum;
}

// ---------------------------------------------------------------- field table
struct RecChunk {
  FieldRec r[kRecsPerWrite];
};

__global__ void k_write_table(RecChunk chunk, int n, FieldRec* __restrict__ out) {
  if ((int)threadIdx.x < n) out[threadIdx.x] = chunk.r[threadIdx.x];
}

// zero every field's band handoff words and progress words (grid: chunks x
// fields)
__global__ void k_clear_xch(const FieldRec* __restrict__ table, int bands_rows) {
  const FieldRec& f = table[blockIdx.y];
  uint64_t* x = reinterpret_cast<uint64_t*>(f.ws + f.o_xch);
  uint64_t* x2 = reinterpret_cast<uint64_t*>(f.ws + f.o_xch2);
  int32_t* pg = reinterpret_cast<int32_t*>(f.ws + f.o_prog);
  const size_t nb = (size_t)((f.Hs + bands_rows - 1) / bands_rows);
  const size_t nw = nb * f.Ws;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) {
    x[i] = 0;
    x2[i] = 0;
  }
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * (size_t)prog_words(f.Hs);
       i += (size_t)gridDim.x * blockDim.x)
    pg[i] = 0;
}

// ---------------------------------------------------------------- seeds (Eq. 1 / Eq. 4)
// One wavefront per coarse grid point: descend the kd-tree with the source
// patch's WHT vector, then re-rank the leaf (ascending pixel index) and the
// optional proposal by the data term; the first minimum wins.
// grid: (points / 4, fields)
__global__ __launch_bounds__(256) void k_seed(const FieldRec* __restrict__ table, int lev, int qshift, int use_tree) {
  const FieldRec& f = table[blockIdx.y];
  const CostCtx c = ctx_of(f, lev, qshift);
  const int Gw = (f.Ws + c.n - 1) >> lev, Gh = (f.Hs + c.n - 1) >> lev;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= Gw * Gh) return;
  const int gx = wave % Gw, gy = wave / Gw;
  const int px = gx * c.n, py = gy * c.n;
  int32_t bestF = kEmpty, bestC = kInf;
  if (use_tree) {
    const int32_t* node_dim = reinterpret_cast<const int32_t*>(f.ws + f.o_dim);
    const int32_t* node_split = reinterpret_cast<const int32_t*>(f.ws + f.o_split);
    const int32_t* perm = reinterpret_cast<const int32_t*>(f.ws + f.o_perm);
    const int Nd = f.Wd * f.Hd;
    const int32_t* q = f.Vsrc + ((size_t)py * c.Ws + px) * f.vstride;
    int node = 0, start = 0, cnt = Nd;
    for (;;) {
      const int dim = node_dim[node];
      if (dim < 0 || 2 * node + 2 >= f.t_nodes) break;
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
  if (f.proposal) {
    const int32_t fp = f.proposal[(size_t)gy * Gw + gx];
    if (fp != kEmpty && centre_valid(c, px, py, fx_of(fp), fy_of(fp))) {
      const int32_t e = group_sum<64>(patch_partial(c, px, py, fx_of(fp), fy_of(fp), lane, 64));
      if (e < bestC) { bestC = e; bestF = fp; }
    }
  }
  if (lane == 0) {
    grid_flow(f, lev)[(size_t)gy * Gw + gx] = bestF;
    grid_cost(f, lev, Gw * Gh)[(size_t)gy * Gw + gx] = bestC;
  }
}

// ---------------------------------------------------------------- level entry
// Section 3.2: points of the coarser grid keep their flow and are re-costed
// with this level's patch; new points start empty.  One group of L lanes per
// coarse point (the fine points of even coordinates), which also writes the
// three new points it covers.  grid: (coarse pts L / 256, fields)
template <int L>
__global__ __launch_bounds__(256) void k_level_entry(const FieldRec* __restrict__ table, int lev, int qshift) {
  static_assert(L == 16, "the row path assumes 16 lanes per point");
  const FieldRec& f = table[blockIdx.y];
  const CostCtx c = ctx_of(f, lev, qshift);
  const int Gw = (f.Ws + c.n - 1) >> lev, Gh = (f.Hs + c.n - 1) >> lev;
  const int Gwc = (f.Ws + 2 * c.n - 1) >> (lev + 1), Ghc = (f.Hs + 2 * c.n - 1) >> (lev + 1);
  const int cid = (blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int lane = threadIdx.x % L;
  if (cid >= Gwc * Ghc) return;
  const int cx = cid % Gwc, cy = cid / Gwc;
  const int gx = 2 * cx, gy = 2 * cy;
  const int32_t fl = grid_flow(f, lev + 1)[cid];
  int32_t e = kInf;
  if (fl != kEmpty) {
    const int px = gx * c.n, py = gy * c.n, fx = fx_of(fl), fy = fy_of(fl);
    const int mx = px * c.Q + fx, my = py * c.Q + fy;
    const int Mx = mx >> c.qshift, My = my >> c.qshift;
    int32_t part;
    if (lev == 0 && (c.r == 8 || c.r == 6) && px >= c.r && px + c.r < c.Ws && Mx >= c.r && Mx + c.r < c.Wd) {
      // stride 1, no column clamp on either side: whole columns per lane
      const uint32_t* D2 = c.dst + (size_t)c.pw * (size_t)(((my & c.qmask) << c.qshift) + (mx & c.qmask));
      g_u32* sb = (g_u32*)(c.src + (px - c.r));
      g_u32* tb = (g_u32*)(D2 + (Mx - c.r));
      part = c.r == 8 ? cols_sum_n1<17, false>(sb, c.Ws, py - 8, c.Hs - 1, tb, c.Wd, My - 8, c.Hd - 1, lane)
                      : cols_sum_n1<13, false>(sb, c.Ws, py - 6, c.Hs - 1, tb, c.Wd, My - 6, c.Hd - 1, lane);
    } else {
      part = patch_partial(c, px, py, fx, fy, lane, L);
    }
    e = group_sum<L>(part);
  }
  int32_t* F = grid_flow(f, lev);
  int32_t* C = grid_cost(f, lev, Gw * Gh);
  if (lane < 4) {
    const int x = gx + (lane & 1), y = gy + (lane >> 1);
    if (x < Gw && y < Gh) {
      F[(size_t)y * Gw + x] = lane == 0 ? fl : kEmpty;
      C[(size_t)y * Gw + x] = lane == 0 ? e : kInf;
    }
  }
  (void)Ghc;
}

// ---------------------------------------------------------------- random search
// Section 3.1 / 3.2: one uniform offset per point, per axis an integer in
// [-nRQ, nRQ] 1/Q px, from Philox keyed by the seed with counter (pixel, level,
// step, field | pair << 2); replace only on a strictly lower cost.
// One workgroup = 256 / L consecutive points of one grid row.  Their source
// patches overlap: the union (S rows x S - 1 + 256 / L columns, grid-aligned
// samples clamped to the image) is staged in LDS once, so only the target
// side of each term is read from global memory.
template <int L>
__global__ __launch_bounds__(256) void k_random_search(const FieldRec* __restrict__ table, int lev, int qshift, int step,
                                                       int R) {
  constexpr int PTS = 256 / L;
  __shared__ uint32_t stile[(2 * kMaxRadius + 1) * (2 * kMaxRadius + PTS + 1)];
  const FieldRec& f = table[blockIdx.y];
  const CostCtx c = ctx_of(f, lev, qshift);
  const int Gw = (f.Ws + c.n - 1) >> lev, Gh = (f.Hs + c.n - 1) >> lev;
  const int tilesX = (Gw + PTS - 1) / PTS;
  const int gy = blockIdx.x / tilesX, gx0 = (blockIdx.x % tilesX) * PTS;
  if (gy >= Gh) return;   // whole workgroup
  // tile rows: S patch rows; pitch odd, so that the row-per-lane path's 16
  // lanes of a point fall in different banks
  const int S = 2 * c.r + 1, TWs = S - 1 + PTS, TP = TWs | 1;
  int32_t* F = grid_flow(f, lev);
  int32_t* C = grid_cost(f, lev, Gw * Gh);
  const int py = gy * c.n;
  // each point's flow and cost, loaded before the tile so that the two
  // round trips overlap
  const int gq = gx0 + (int)threadIdx.x;
  int32_t fl = kEmpty, cq = 0;
  if (threadIdx.x < PTS && gq < Gw) {
    fl = F[gy * Gw + gq];
    cq = C[gy * Gw + gq];
  }
  for (int e = threadIdx.x; e < S * TWs; e += 256) {
    const int yy = e / TWs, xx = e - yy * TWs;
    const int sy = clampi((gy + yy - c.r) * c.n, 0, c.Hs - 1), sx = clampi((gx0 + xx - c.r) * c.n, 0, c.Ws - 1);
    stile[yy * TP + xx] = c.src[(size_t)sy * c.Ws + sx];
  }
  // each point's candidate, once per point (one lane of the first wavefront
  // per point: the Philox rounds are quarter-rate multiplies)
  __shared__ int32_t s_fx[PTS], s_fy[PTS], s_c[PTS], s_ok[PTS];
  if (threadIdx.x < PTS) {
    int ok = 0, fxq = 0, fyq = 0;
    if (gq < Gw) {
      if (fl != kEmpty) {
        const int pxq = gq * c.n;
        const int rad = c.n * R * c.Q;
        uint32_t u0, u1;
        philox2((uint32_t)(py * c.Ws + pxq), (uint32_t)lev, (uint32_t)step, f.c3, f.k0, f.k1, u0, u1);
        const uint64_t span = (uint64_t)(2 * rad + 1);
        fxq = fx_of(fl) + (int)((u0 * span) >> 32) - rad;
        fyq = fy_of(fl) + (int)((u1 * span) >> 32) - rad;
        ok = centre_valid(c, pxq, py, fxq, fyq) ? 1 : 0;
      }
    }
    s_fx[threadIdx.x] = fxq;
    s_fy[threadIdx.x] = fyq;
    s_c[threadIdx.x] = cq;
    s_ok[threadIdx.x] = ok;
  }
  __syncthreads();
  const int i = threadIdx.x / L, lane = threadIdx.x % L;
  const int gx = gx0 + i;
  if (gx >= Gw || !s_ok[i]) return;
  const int pid = gy * Gw + gx;
  const int px = gx * c.n;
  const int fx = s_fx[i], fy = s_fy[i];
  // the patch sum, source terms from the tile
  const int mx = px * c.Q + fx, my = py * c.Q + fy;
  const int Mx = mx >> c.qshift, My = my >> c.qshift;
  const uint32_t* D2 = c.dst + (size_t)c.pw * (size_t)(((my & c.qmask) << c.qshift) + (mx & c.qmask));
  int32_t sum = 0;
  if (L == 16 && lev == 0 && (c.r == 8 || c.r == 6) && Mx >= c.r && Mx + c.r < c.Wd) {
    // stride 1 and no column clamp on the target side: whole columns per lane
    // (the tile's rows are already clamped)
    g_u32* tb = (g_u32*)(D2 + (Mx - c.r));
    const uint32_t* sb = stile + i;
    sum = c.r == 8 ? cols_sum_n1<17, true>(sb, TP, 0, S - 1, tb, c.Wd, My - 8, c.Hd - 1, lane)
                   : cols_sum_n1<13, true>(sb, TP, 0, S - 1, tb, c.Wd, My - 6, c.Hd - 1, lane);
  } else {
    int dy = lane / S, dx = lane - dy * S;
    const int stepy = L / S, stepx = L - stepy * S;
#pragma unroll 4
    for (int t = lane; t < S * S; t += L) {
      const uint32_t a = stile[dy * TP + i + dx];
      const uint32_t b = D2[(size_t)clampi(My + (dy - c.r) * c.n, 0, c.Hd - 1) * c.Wd +
                            clampi(Mx + (dx - c.r) * c.n, 0, c.Wd - 1)];
      sum += __popc(a ^ b);
      dx += stepx;
      dy += stepy;
      if (dx >= S) { dx -= S; ++dy; }
    }
  }
  const int32_t e = group_sum<L>(sum);
  if (lane == 0 && e < s_c[i]) {
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
// Step t of a band: row i handles u = t - s(i), s(i) = i + i / 4 (each
// wavefront of four rows one step behind the one above, so that every
// candidate of a step is known, and its target words loaded, at the end of
// the step before).  Rows hand results down inside a wavefront by DPP and
// across wavefronts through a double-buffered LDS slot (one barrier per
// step).  The band's last row
// publishes each result as one 64-bit word (flow | cost | launch tag) with a
// relaxed agent-scope store; row 0 of the band below polls that word until
// the tag matches.  One single-copy-atomic word carries data and readiness,
// so no fence (L2 write-back or invalidate) is needed on the critical path.
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
// u+r (horizontal candidate), each over offsets -r..r.  Slot g of lane l
// takes offset index l of group g (valid while l < S); for S > 16 the S - 16
// remaining offsets of the four groups are packed into TAIL extra slots whose
// group is a per-lane constant.
//
// A step is written for a short instruction stream (one wavefront per SIMD,
// so a step's latency is its instruction count plus what is left of one
// memory round trip after the barrier and the step's LDS reads):
// target words are read with 32-bit offsets from one scalar base (row-major
// and transposed planes of a level lie in one blob), tail groups are chosen
// with lane-constant masks, and the vertical and horizontal sums travel
// packed in one 32-bit word through the DPP reduction.
constexpr int kBatch = 32;

typedef __attribute__((address_space(1))) const char g_byte;


__device__ __forceinline__ int med3i(int v, int lo, int hi) { return min(max(v, lo), hi); }
// clamp to [0, hi] in one instruction (the compiler emits max then min when
// the upper bound is not a constant); hi is uniform
__device__ __forceinline__ uint32_t clamp0(int v, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(v), "s"(hi));
  return (uint32_t)r;
}
// target word at a 32-bit word offset from a uniform base: the byte offset is
// formed in 32 bits so the load takes the scalar-base + 32-bit-offset form
// (ff_desc_init refuses layouts whose largest offset would not fit)
__device__ __forceinline__ uint32_t tword(g_byte* base, uint32_t w) {
  return *reinterpret_cast<__attribute__((address_space(1))) const uint32_t*>(base + (w << 2));
}

// ---------------------------------------------------------------- pipelined sweep pairs
// Two consecutive sweeps that share the horizontal direction (and so run in
// opposite vertical directions) can overlap: a point's value after the first
// sweep and the random search between them is all the second one needs, so
// the second sweep may start on columns the first has finished.  Such a pair
// is one launch with three roles, claimed in this order by the launch's
// ticket: A (the first sweep, one workgroup per band), X (the random search
// after A, kXRows grid rows of the second sweep's bands per workgroup, run
// behind A's progress) and B (the second sweep, one workgroup per band,
// starting a batch once X has finished the columns it stages).  Every wait is
// on a workgroup with a lower ticket, which is already running.  The random
// search of a point depends on that point alone, so every result equals the
// one-launch-per-stage order.  Workgroups of one launch may sit on different
// XCDs, whose L2 caches are not coherent: flows and costs that cross roles
// are read and written with device-coherent (agent-scope) accesses, and A and
// X publish how many columns of a band are final in a progress word (launch
// tag << 20 | columns) after their stores have completed.
// The same holds across a level change: the last sweep of level 2n runs in
// the horizontal direction of the first sweep of level n, and only the level
// entry (coarse flows carried to the finer grid and re-costed, a per-point
// step like the random search) lies between them; such a cross-level pair has
// A on the coarse grid and X (the level entry) and B on the fine one.
constexpr int kRoleA = 0, kRoleX = 1, kRoleB = 2;
constexpr int kXRows = 4;
constexpr int kPairSame = 1, kPairCross = 2;

// global-address-space accesses throughout: a flat access also counts as an
// LDS operation and, while pending, turns a wait for some loads into a wait
// for all of them
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
__device__ __forceinline__ int32_t ld_coh(const int32_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(int32_t* p, int32_t v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t prog_word(uint32_t tag, int cols) {
  return (int32_t)(((tag & 0xFFFu) << 20) | (uint32_t)cols);
}
__device__ __forceinline__ int prog_cols(int32_t w, uint32_t tag) {
  return ((uint32_t)w >> 20) == (tag & 0xFFFu) ? (int)((uint32_t)w & 0xFFFFFu) : 0;
}
// one thread: wait until a progress word reaches `need` columns; on the
// watchdog the launch reports FF_ERR_DEVICE and the wait gives up, and once
// an error is reported no later wait of the call waits at all
__device__ bool wait_prog(const int32_t* w, uint32_t tag, int need, int32_t* status, uint64_t timeout) {
  if (prog_cols(ld_coh(w), tag) >= need) return true;
  const uint64_t t0 = rt_clock();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (prog_cols(ld_coh(w), tag) >= need) return true;
    if (ld_coh(status) != 0) return false;
    if (rt_clock() - t0 > timeout) {
      __hip_atomic_store(status, (int32_t)FF_ERR_DEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}
// all of this workgroup's global stores complete, then one word published
__device__ __forceinline__ void publish_prog(int32_t* w, uint32_t tag, int cols) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) st_coh(w, prog_word(tag, cols));
}

// Data term of candidate (fx, fy) at grid point (px, py) of level lev by a
// group of 16 lanes (the sum is left in every lane of the group): whole columns
// per lane at stride 1 when no column clamps, else the generic walk.
__device__ __forceinline__ int32_t cand_cost(const CostCtx& c, int lev, int px, int py, int fx, int fy, int lane) {
  const int mx = px * c.Q + fx, my = py * c.Q + fy;
  const int Mx = mx >> c.qshift, My = my >> c.qshift;
  int32_t part;
  if (lev == 0 && (c.r == 8 || c.r == 6) && px >= c.r && px + c.r < c.Ws && Mx >= c.r && Mx + c.r < c.Wd) {
    const uint32_t* D2 = c.dst + (size_t)c.pw * (size_t)(((my & c.qmask) << c.qshift) + (mx & c.qmask));
    g_u32* sb = (g_u32*)(c.src + (px - c.r));
    g_u32* tb = (g_u32*)(D2 + (Mx - c.r));
    part = c.r == 8 ? cols_sum_n1<17, false>(sb, c.Ws, py - 8, c.Hs - 1, tb, c.Wd, My - 8, c.Hd - 1, lane)
                    : cols_sum_n1<13, false>(sb, c.Ws, py - 6, c.Hs - 1, tb, c.Wd, My - 6, c.Hd - 1, lane);
  } else {
    part = patch_partial(c, px, py, fx, fy, lane, 16);
  }
  return group_sum<16>(part);
}

// An X workgroup: rows kXRows m .. kXRows m + kXRows - 1 of band k of the
// second sweep (level lev, direction syX), columns in chunks of 32 as the
// first sweep's bands (direction -syX, progress words progA) finish the
// columns they need; publishes its progress in progX[k * BH / kXRows + m].
// Same-level pair: random search step rs (< 0: none, progress is only passed
// on), as in k_random_search, the first sweep on the same grid.  Cross-level
// pair: the level entry, as in k_level_entry, the first sweep on the grid of
// level lev + 1.  A chunk's candidates are formed one point per thread (flow
// and cost loads, Philox) before the 16-lane groups cost them, so a point's
// chain holds one memory round trip.
template <int BH>
__device__ __forceinline__ void x_worker(const FieldRec& fr, const CostCtx& c, int lev, bool cross, int k, int m,
                                         int sx, int syX, const int32_t* progA, int32_t* progX, int rs, int R,
                                         uint32_t tag, int32_t* status, uint64_t timeout) {
  constexpr int CH = kBatch;
  __shared__ int32_t x_fx[kXRows * CH], x_fy[kXRows * CH], x_c[kXRows * CH], x_ok[kXRows * CH];
  const int n = c.n;
  const int Gw = (fr.Ws + n - 1) >> lev, Gh = (fr.Hs + n - 1) >> lev;
  int32_t* const F = grid_flow(fr, lev);
  int32_t* const C = grid_cost(fr, lev, Gw * Gh);
  // the first sweep's grid
  const int la = cross ? lev + 1 : lev;
  const int Gwa = (fr.Ws + (1 << la) - 1) >> la, Gha = (fr.Hs + (1 << la) - 1) >> la;
  const int32_t* const Fa = grid_flow(fr, la);
  const int b0 = k * BH;
  const int v0 = b0 + m * kXRows;
  const int rows = min(kXRows, min(BH, Gh - b0) - m * kXRows);
  int32_t* const pw = progX + k * (BH / kXRows) + m;
  if (rows <= 0) {
    publish_prog(pw, tag, Gw);
    return;
  }
  // the first sweep's bands holding these grid rows: grid rows gy (range
  // gya..gyb) lie in row gy >> cross of the first sweep's grid, which that
  // sweep (direction -syX) numbers Gha - 1 - (gy >> cross) if it runs upward
  const int gya = syX > 0 ? v0 : Gh - 1 - (v0 + rows - 1), gyb = syX > 0 ? v0 + rows - 1 : Gh - 1 - v0;
  const int sh = cross ? 1 : 0;
  const int blo = syX > 0 ? (Gha - 1 - (gyb >> sh)) / BH : (gya >> sh) / BH;
  const int bhi = syX > 0 ? (Gha - 1 - (gya >> sh)) / BH : (gyb >> sh) / BH;
  const int lane = threadIdx.x % 16, group = threadIdx.x / 16, ngroups = blockDim.x / 16;
  for (int c0 = 0; c0 < Gw; c0 += CH) {
    const int c1 = min(c0 + CH, Gw), cw = c1 - c0;
    // columns of the first sweep's grid that hold this chunk's points: the
    // last column of the chunk maps to the largest one
    const int gxl = sx > 0 ? c1 - 1 : Gw - c1;
    const int need = (sx > 0 ? (gxl >> sh) : Gwa - 1 - (gxl >> sh)) + 1;
    if (threadIdx.x == 0)
      for (int b = blo; b <= bhi; ++b) wait_prog(progA + b, tag, need, status, timeout);
    __syncthreads();
    if (cross || rs >= 0) {
      // candidates, one point per thread
      for (int q = threadIdx.x; q < rows * cw; q += blockDim.x) {
        const int v = v0 + q / cw, u = c0 + q % cw;
        const int gx = sx > 0 ? u : Gw - 1 - u, gy = syX > 0 ? v : Gh - 1 - v;
        const int px = gx * n, py = gy * n;
        int ok = 0, fxq = 0, fyq = 0, cq = 0;
        if (cross) {
          // carried points keep the coarse flow; every other point is new
          int32_t fl = kEmpty;
          if (!(gx & 1) && !(gy & 1)) fl = ld_coh(Fa + (size_t)(gy >> 1) * Gwa + (gx >> 1));
          if (fl != kEmpty) {
            ok = 1;
            fxq = fx_of(fl);
            fyq = fy_of(fl);
          } else {
            st_coh(F + (size_t)gy * Gw + gx, kEmpty);
            st_coh(C + (size_t)gy * Gw + gx, kInf);
          }
        } else {
          const int32_t fl = ld_coh(F + (size_t)gy * Gw + gx);
          if (fl != kEmpty) {
            const int rad = n * R * c.Q;
            uint32_t u0, u1;
            philox2((uint32_t)(py * c.Ws + px), (uint32_t)lev, (uint32_t)rs, fr.c3, fr.k0, fr.k1, u0, u1);
            const uint64_t span = (uint64_t)(2 * rad + 1);
            fxq = fx_of(fl) + (int)((u0 * span) >> 32) - rad;
            fyq = fy_of(fl) + (int)((u1 * span) >> 32) - rad;
            ok = centre_valid(c, px, py, fxq, fyq) ? 1 : 0;
            cq = ld_coh(C + (size_t)gy * Gw + gx);
          }
        }
        x_fx[q] = fxq;
        x_fy[q] = fyq;
        x_c[q] = cq;
        x_ok[q] = ok;
      }
      __syncthreads();
      // their data terms, one group of 16 lanes per point
      for (int i = group; i < rows * cw; i += ngroups) {
        if (!x_ok[i]) continue;
        const int v = v0 + i / cw, u = c0 + i % cw;
        const int gx = sx > 0 ? u : Gw - 1 - u, gy = syX > 0 ? v : Gh - 1 - v;
        const int fx = x_fx[i], fy = x_fy[i];
        const int32_t e = cand_cost(c, lev, gx * n, gy * n, fx, fy, lane);
        if (lane == 0) {
          if (cross) {
            // the level entry keeps the flow whatever its cost
            st_coh(F + (size_t)gy * Gw + gx, packf(fx, fy));
            st_coh(C + (size_t)gy * Gw + gx, e);
          } else if (e < x_c[i]) {
            st_coh(F + (size_t)gy * Gw + gx, packf(fx, fy));
            st_coh(C + (size_t)gy * Gw + gx, e);
          }
        }
      }
    }
    publish_prog(pw, tag, c1);
  }
}

// pair = 0: one sweep (sx, sy) at level lev, one workgroup per band;
// kPairSame: the sweep pair (sx, sy) then (sx, -sy) at level lev with the
// random search step rs (< 0: none) between them; kPairCross: the sweep
// (sx, sy) at level lev + 1, the level entry of level lev, then the sweep
// (sx, -sy) at level lev.  na: bands of level lev over the launch's fields;
// na_a: bands of the first sweep's level.
template <int TAIL, int BH>
__global__ __launch_bounds__(BH * kLanesProp + 64) void k_propagate(const FieldRec* __restrict__ table, int f0, int nf,
                                                               int lev, int qshift, int sx, int sy, uint32_t tag,
                                                               int32_t* __restrict__ ticket,
                                                               int32_t* __restrict__ status,
                                                               uint64_t timeout_ticks, int pair, int na, int na_a,
                                                               int rs, int R) {
  constexpr int L = kLanesProp, CH = kBatch;
  constexpr int NS = 4 + TAIL;   // term slots per lane
  static_assert(L == 16 && CH % 2 == 0 && CH % L == 0 && TAIL <= 4, "layout");
  // rows run skewed: row i works on u = t - s(i), s(i) = i + i / 4 (one more
  // step per wavefront), so the tile's left margin is BH + BH / 4 columns
  constexpr int M = BH + BH / 4;
  constexpr int kTileWords = (BH + 2 * kMaxRadius + 1) * ((kBatch + M + 2 * kMaxRadius) | 1);
  __shared__ int32_t s_band, s_field, s_role, s_sub;
  __shared__ int32_t bufF[2][BH], bufC[2][BH];
  __shared__ int32_t topF[2], topC[2];   // row 0's vertical candidate, by step parity
  __shared__ int32_t inF[BH][CH], inC[BH][CH], outF[BH][CH], outC[BH][CH];
  __shared__ uint32_t tile[kTileWords];
  // the band's rows run on BH / 4 wavefronts; one more wavefront waits for
  // the band above and hands row 0 its vertical candidate through LDS, one
  // step ahead, so that no compute wavefront polls global memory
  const bool pollWave = __builtin_amdgcn_readfirstlane(threadIdx.x) >= BH * L;
  const int row = pollWave ? 0 : threadIdx.x / L, lane = threadIdx.x % L;
  if (threadIdx.x == 0) {
    // tickets are handed out in launch order; role-major, then field-major,
    // band-minor; role sizes: A na_a, X na BH / kXRows, B na
    int tk = atomicAdd(ticket, 1), fi = f0;
    int role = -1, sub = 0;
    for (int rb = 0; rb < (pair ? 3 : 1); ++rb) {
      const int per = rb == kRoleX ? BH / kXRows : 1;
      const int cnt = (rb == kRoleA ? na_a : na) * per;
      if (tk < cnt) {
        role = rb;
        sub = tk % per;
        tk /= per;
        break;
      }
      tk -= cnt;
    }
    s_role = role;
    s_sub = sub;
    const int nr = 1 << (role == kRoleA && pair == kPairCross ? lev + 1 : lev);
    for (; fi < f0 + nf; ++fi) {
      const int gh = (table[fi].Hs + nr - 1) / nr;
      const int nb = (gh + BH - 1) / BH;
      if (tk < nb) break;
      tk -= nb;
    }
    s_band = tk;
    s_field = fi;
  }
  __syncthreads();
  if (s_field >= f0 + nf || s_role < 0) return;
  const int role = s_role;
  if (role == kRoleA && pair == kPairCross) ++lev;   // the first sweep runs on the coarser grid
  const int n = 1 << lev;
  const FieldRec& fr = table[s_field];
  const CostCtx c = ctx_of(fr, lev, qshift);
  const int Gw = (fr.Ws + n - 1) >> lev, Gh = (fr.Hs + n - 1) >> lev;
  int32_t* const F = grid_flow(fr, lev);
  int32_t* const C = grid_cost(fr, lev, Gw * Gh);
  // progress words: A's bands, then X's workgroups
  int32_t* const progA = reinterpret_cast<int32_t*>(fr.ws + fr.o_prog);
  int32_t* const progX = progA + prog_words(fr.Hs);
  if (role == kRoleX) {
    x_worker<BH>(fr, c, lev, pair == kPairCross, s_band, s_sub, sx, -sy, progA, progX, rs, R, tag, status,
                 timeout_ticks);
    return;
  }
  if (role == kRoleB) sy = -sy;
  // a band's step is a latency chain: its compute wavefronts go first in the
  // SIMD arbitration against co-resident workgroups (the X role's searches,
  // other launches); measured 10.20 -> 10.16 ms per pair
  if (!pollWave) __builtin_amdgcn_s_setprio(3);
  const bool coherent = pair != 0;   // flows/costs cross roles of this launch
  const int32_t* const waitProg = role == kRoleB ? progX : nullptr;
  int32_t* const pubProg = role == kRoleA && pair ? progA : nullptr;
  uint64_t* const xch = reinterpret_cast<uint64_t*>(fr.ws + (role == kRoleB ? fr.o_xch2 : fr.o_xch));
  const int band = s_band;
  const int v0 = band * BH;
  if (v0 >= Gh) return;
  const int rows = min(BH, Gh - v0);
  const int skew = row + (row >> 2);      // s(row): this row works on u = t - skew
  const int skewLast = (rows - 1) + ((rows - 1) >> 2);
  const int nsteps = Gw + skewLast;
  const int r = c.r, S = 2 * r + 1, Q = c.Q;
  const int TH = BH + 2 * r + 1;          // tile rows: v0-r-1 .. v0+BH-1+r
  const int TW = (CH + M + 2 * r) | 1;    // tile cols: tb-M-r .. tb+CH-1+r; odd pitch (banks)
  const bool rowok = !pollWave && row < rows;
  const int rr = rowok ? row : rows - 1;  // inactive rows shadow a valid row
  const int gy = sy > 0 ? v0 + rr : Gh - 1 - (v0 + rr);
  const int py = gy * n;
  const bool publish = rowok && row == rows - 1 && v0 + rows < Gh;
  const bool above = v0 > 0;              // a band above exists
  const uint64_t* xin = xch + (size_t)(band > 0 ? band - 1 : 0) * Gw;
  uint64_t* xout = xch + (size_t)band * Gw;
  int32_t* Frow = F + (size_t)gy * Gw;
  int32_t* Crow = C + (size_t)gy * Gw;
  auto gx_of = [&](int u) { return sx > 0 ? u : Gw - 1 - u; };
  auto gy_of = [&](int v) { return sy > 0 ? v : Gh - 1 - v; };
  // target words: one scalar base (level plane 0), 32-bit word offsets; the
  // transposed planes start dT words after the row-major ones
  g_byte* const tgt = (g_byte*)(c.dst);
  const uint32_t dT = (uint32_t)(c.dstT - c.dst);
  const int nsx = sx * n, nsy = sy * n;
  const int Wm = c.Wd - 1, Hm = c.Hd - 1;
  const uint32_t Wd = (uint32_t)c.Wd, Hd = (uint32_t)c.Hd;
  // lane constants: the full slots' offset along the group's free axis and
  // validity; per tail slot its group (as selection masks), validity, sign
  // and half of the packed sum; every slot's tile offset
  const int offFull = lane - r;
  const uint32_t fullMask = TAIL > 0 || lane < S ? ~0u : 0u;
  const int oxFull = nsx * offFull, oyFull = nsy * offFull;
  int tOff[TAIL > 0 ? TAIL : 1], tGrp[TAIL > 0 ? TAIL : 1];
  bool tG1[TAIL > 0 ? TAIL : 1], tG3[TAIL > 0 ? TAIL : 1], tH[TAIL > 0 ? TAIL : 1];
  int32_t tMul[TAIL > 0 ? TAIL : 1];
#pragma unroll
  for (int q = 0; q < TAIL; ++q) {
    const int tl = S - 16;                   // remaining offsets per group
    const int e = lane + 16 * q;             // packed tail term
    const int g0 = e / tl;
    const bool ok = g0 < 4;
    const int g = ok ? g0 : 0;
    tGrp[q] = g;
    tOff[q] = 16 + (ok ? e % tl : 0) - r;
    tG1[q] = g == 1;
    tG3[q] = g == 3;
    tH[q] = g >= 2;
    tMul[q] = ok ? ((g & 1) ? 1 : -1) * (g >= 2 ? 65536 : 1) : 0;
  }
  int stoff[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int g = k < 4 ? k : tGrp[k - 4 < TAIL ? k - 4 : 0];
    const int o = k < 4 ? offFull : tOff[k - 4 < TAIL ? k - 4 : 0];
    const int du = g < 2 ? o : (g == 2 ? -r - 1 : r);
    const int dv = g < 2 ? (g == 0 ? -r - 1 : r) : o;
    stoff[k] = (r + 1 + dv) * TW + (M + r + du);
  }
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
  const uint32_t maxMx = (uint32_t)(Wm * Q), maxMy = (uint32_t)(Hm * Q);
  // the polling wavefront: before the barrier that ends step col - 2, the
  // band above's result at column col for row 0 (EMPTY without a band
  // above or past the row's end); `pw` holds the prefetched word for col
  uint64_t pw = above ? __hip_atomic_load(&xin[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  auto provide = [&](int col) {
    int32_t f = kEmpty, cst = kInf;
    if (above && col < Gw) {
      const uint64_t w = wait_word(col, pw);
      f = (int32_t)(uint32_t)w;
      const uint32_t c16 = (uint32_t)(w >> 32) & 0xFFFFu;
      cst = c16 == 0xFFFFu ? kInf : (int32_t)c16;
      pw = __hip_atomic_load(&xin[med3i(col + 1, 0, Gw - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if ((threadIdx.x & 63) == 0) {
      topF[col & 1] = f;
      topC[col & 1] = cst;
    }
  };
  // Both candidates of the next step are known at the end of a step: the
  // horizontal one is the row's own result, the vertical one the result of
  // the row above -- in this wavefront (moved down one 16-lane row by DPP),
  // or, for a wavefront's first row, written to LDS by the wavefront above
  // two steps earlier (the skew), or for row 0 handed over by the polling
  // wavefront two steps ahead.  So every target word of the next step is
  // loaded at the end of the step before and is in flight across the
  // barrier (which waits for LDS operations only).
  int32_t hFn = kEmpty, hCn = kInf, vFn = kEmpty, vCn = kInf;
  int mxh = 0, myh = 0, mxv = 0, myv = 0;
  uint32_t nb[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) nb[k] = 0;
  // pxq: the next column's x in 1/Q px (computed ahead, off the chain from
  // a step's result to its successor's loads); hok: that column has a
  // horizontal predecessor
  const int nQshift = lev + c.qshift;   // n Q = 2^(lev + qshift)
  auto pxq_of = [&](int un) { return gx_of(med3i(un, 0, Gw - 1)) << nQshift; };
  auto prep = [&](int pxq, bool hok, int32_t f, int32_t cst, int32_t vf, int32_t vc) {
    hFn = hok ? f : kEmpty;
    hCn = hok ? cst : kInf;
    vFn = vf;
    vCn = vc;
    mxh = pxq + fx_of(hFn);
    myh = py * Q + fy_of(hFn);
    mxv = pxq + fx_of(vFn);
    myv = py * Q + fy_of(vFn);
    const int Mxh = mxh >> c.qshift, Myh = myh >> c.qshift;
    const int Mxv = mxv >> c.qshift, Myv = myv >> c.qshift;
    // every product has both factors below 2^24 (plane words <= 2^22, phase
    // < 64, coordinates and pitches < 8192): full-rate 24-bit multiplies
    const uint32_t phh = dT + __umul24(c.pw, (uint32_t)(((myh & c.qmask) << c.qshift) + (mxh & c.qmask)));
    const uint32_t base2 = phh + __umul24(clamp0(Mxh - nsx * (r + 1), Wm), Hd);
    const uint32_t base3 = phh + __umul24(clamp0(Mxh + nsx * r, Wm), Hd);
    const uint32_t phv = __umul24(c.pw, (uint32_t)(((myv & c.qmask) << c.qshift) + (mxv & c.qmask)));
    const uint32_t base0 = phv + __umul24(clamp0(Myv - nsy * (r + 1), Hm), Wd);
    const uint32_t base1 = phv + __umul24(clamp0(Myv + nsy * r, Hm), Wd);
    const uint32_t xv = clamp0(Mxv + oxFull, Wm);
    const uint32_t yh = clamp0(Myh + oyFull, Hm);
    nb[0] = tword(tgt, base0 + xv);
    nb[1] = tword(tgt, base1 + xv);
    nb[2] = tword(tgt, base2 + yh);
    nb[3] = tword(tgt, base3 + yh);
#pragma unroll
    for (int q = 0; q < TAIL; ++q) {
      // the lane's group (a per-lane constant) picks the base and the free
      // coordinate
      const uint32_t xq = clamp0(Mxv + nsx * tOff[q], Wm);
      const uint32_t yq = clamp0(Myh + nsy * tOff[q], Hm);
      const uint32_t bv = tG1[q] ? base1 : base0, bh = tG3[q] ? base3 : base2;
      nb[4 + q] = tword(tgt, (tH[q] ? bh : bv) + (tH[q] ? yq : xq));
    }
  };
  const bool waveFirst = (row & 3) == 0;
  auto step = [&](int t, int tb) {
    const int j = t - tb;
    const int u = t - skew;
    const bool active = rowok && u >= 0 && u < Gw;
    const int pxq1 = pxq_of(u + 1);
    const int32_t curF0 = inF[row][j], curC0 = inC[row][j];
    // the next step's vertical candidate of a wavefront's first row: row 0
    // from the polling wavefront, else the row above's result of step t - 1
    const int32_t lvF = row == 0 ? topF[(t + 1) & 1] : bufF[(t - 1) & 1][row > 0 ? row - 1 : 0];
    const int32_t lvC = row == 0 ? topC[(t + 1) & 1] : bufC[(t - 1) & 1][row > 0 ? row - 1 : 0];
    const int32_t vF = vFn, vC = vCn, hF = hFn, hC = hCn;
    // candidate centres in 1/Q px; EMPTY (-32768, -32768) always falls
    // outside, so the validity test also rejects empty candidates
    const bool useV = active && vF != curF0 && (uint32_t)mxv <= maxMx && (uint32_t)myv <= maxMy;
    const bool useH = active && hF != curF0 && (uint32_t)mxh <= maxMx && (uint32_t)myh <= maxMy;
    const int tbase = row * TW + (u - tb);
    uint32_t aw[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) aw[k] = tile[tbase + stoff[k]];
    // entering minus leaving terms, vertical in the low half, horizontal in
    // the high half of one word (|sums| < 2^15)
    int32_t packed = (int32_t)__popc((aw[1] ^ nb[1]) & fullMask) - (int32_t)__popc((aw[0] ^ nb[0]) & fullMask);
    packed += (int32_t)((uint32_t)((int32_t)__popc((aw[3] ^ nb[3]) & fullMask) -
                                   (int32_t)__popc((aw[2] ^ nb[2]) & fullMask)) << 16);
#pragma unroll
    for (int q = 0; q < TAIL; ++q) {
      packed += __mul24((int32_t)__popc(aw[4 + q] ^ nb[4 + q]), tMul[q]);
    }
    const int32_t sum = row16_sum(packed);
    const int32_t dvs = (int32_t)(int16_t)(uint16_t)((uint32_t)sum & 0xFFFFu);
    const int32_t dhs = (sum - dvs) >> 16;
    // candidate order of Eq. 2: current, vertical, horizontal; strict <
    int32_t curF = curF0, curC = curC0;
    if (useV && vC + dvs < curC) { curF = vF; curC = vC + dvs; }
    if (useH && hC + dhs < curC) { curF = hF; curC = hC + dhs; }
    // the next step's candidates: the row above's result moved down one row
    // of 16 lanes (rows 1..3 of the wavefront), or the LDS value
    const int32_t dF = __builtin_amdgcn_update_dpp(0, curF, 0x142, 0xE, 0xF, false);   // row_bcast:15
    const int32_t dC = __builtin_amdgcn_update_dpp(0, curC, 0x142, 0xE, 0xF, false);
    prep(pxq1, u >= 0, curF, curC, waveFirst ? lvF : dF, waveFirst ? lvC : dC);
    if (lane == 0) {
      bufF[t & 1][row] = curF;
      bufC[t & 1][row] = curC;
      outF[row][j] = curF;
      outC[row][j] = curC;
      if (publish && active)
        __hip_atomic_store(gp(xout + u), xch_pack(curF, curC, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  const int TT = TH * TW;
  constexpr int KPT = (kTileWords + BH * L - 1) / (BH * L);   // tile words per thread
  for (int tb = 0; tb < nsteps; tb += CH) {
    // a trailing sweep starts a batch once the columns it stages are final
    if (waitProg) {
      if (threadIdx.x == 0)
        for (int m = 0; m < BH / kXRows; ++m)
          wait_prog(waitProg + band * (BH / kXRows) + m, tag, min(tb + CH, Gw), status, timeout_ticks);
      __syncthreads();
    }
    // stage this batch's own flows and costs (row r at step tb + j works on
    // u = tb + j - s(r)) and the source tile: tile(y, x) is the source
    // census at transformed grid (u, v) = (tb - M - r + x, v0 - r - 1 + y),
    // clamped to the image in pixels
#pragma unroll
    for (int jj = 0; jj < CH / L; ++jj) {
      const int j = lane + jj * L;
      const int u = tb + j - skew;
      if (rowok && u >= 0 && u < Gw) {
        if (coherent) {
          inF[row][j] = ld_coh(Frow + gx_of(u));
          inC[row][j] = ld_coh(Crow + gx_of(u));
        } else {
          inF[row][j] = Frow[gx_of(u)];
          inC[row][j] = Crow[gx_of(u)];
        }
      }
    }
    if (!pollWave) {
      // all of a thread's tile loads are issued before its first LDS write
      uint32_t tv[KPT];
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const int e = min((int)threadIdx.x + k * BH * L, TT - 1);
        const int y = e / TW, x = e - y * TW;
        const int gxp = gx_of(tb - M - r + x) * n, gyp = gy_of(v0 - r - 1 + y) * n;
        tv[k] = c.src[(size_t)clampi(gyp, 0, c.Hs - 1) * c.Ws + clampi(gxp, 0, c.Ws - 1)];
      }
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const int e = (int)threadIdx.x + k * BH * L;
        if (e < TT) tile[e] = tv[k];
      }
    } else if (tb == 0) {
      provide(0);
      provide(1);
    }
    __syncthreads();
    if (tb == 0) {
      // step 0's candidates (row 0's vertical one from the polling wavefront);
      // a barrier before the polling wavefront reuses that LDS slot
      if (!pollWave) prep(pxq_of(0), false, kEmpty, kInf, row == 0 ? topF[0] : kEmpty, row == 0 ? topC[0] : kInf);
      lds_barrier();
    }
    const int te = min(tb + CH, nsteps);
    for (int t = tb; t < te; ++t) {
      if (pollWave) provide(t + 2);
      else step(t, tb);
      lds_barrier();
    }
    // write the batch's results back
#pragma unroll
    for (int jj = 0; jj < CH / L; ++jj) {
      const int j = lane + jj * L;
      const int u = tb + j - skew;
      if (rowok && u >= 0 && u < Gw && tb + j < te) {
        if (coherent) {
          st_coh(Frow + gx_of(u), outF[row][j]);
          st_coh(Crow + gx_of(u), outC[row][j]);
        } else {
          Frow[gx_of(u)] = outF[row][j];
          Crow[gx_of(u)] = outC[row][j];
        }
      }
    }
    // after steps < te every row has finished columns u <= te - 1 - s(rows - 1)
    if (pubProg) publish_prog(pubProg + band, tag, min(max(te - skewLast, 0), Gw));
  }
}

// write the grid of level lev into the full-resolution outputs (inspection
// stops); grid: (W / 256, H, fields)
__global__ void k_write_grid(const FieldRec* __restrict__ table, int lev) {
  const FieldRec& f = table[blockIdx.z];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= f.Ws || y >= f.Hs) return;
  const int n = 1 << lev;
  const int Gw = (f.Ws + n - 1) >> lev, Gh = (f.Hs + n - 1) >> lev;
  const size_t o = (size_t)y * f.Ws + x;
  if ((x % n) == 0 && (y % n) == 0) {
    f.flow[o] = grid_flow(f, lev)[(size_t)(y / n) * Gw + x / n];
    f.cost[o] = grid_cost(f, lev, Gw * Gh)[(size_t)(y / n) * Gw + x / n];
  } else {
    f.flow[o] = kEmpty;
    f.cost[o] = kInf;
  }
}

// One propagation launch: a sweep, or a sweep pair (A, X, B workgroups);
// lev is the level of the (second) sweep.
struct PropLaunch {
  int lev, qshift, sx, sy;
  uint32_t tag;
  int32_t* ticket;
  int32_t* status;
  uint64_t timeout;
  int pair, rs, R;
};

template <int BH>
static void launch_propagate_bh(int r, int bands, int bands_a, hipStream_t stream, const FieldRec* table, int f0,
                                int nf, const PropLaunch& L) {
  const dim3 grid(L.pair ? bands_a + bands * (1 + BH / kXRows) : bands), block(BH * kLanesProp + 64);
  const int S = 2 * r + 1, tail = S > 16 ? (4 * (S - 16) + 15) / 16 : 0;
#define FF_PROP(TA)                                                                                                \
  if (tail == TA) {                                                                                                \
    k_propagate<TA, BH><<<grid, block, 0, stream>>>(table, f0, nf, L.lev, L.qshift, L.sx, L.sy, L.tag, L.ticket,    \
                                                    L.status, L.timeout, L.pair, bands, bands_a, L.rs, L.R);       \
    return;                                                                                                        \
  }
  FF_PROP(0) FF_PROP(1) FF_PROP(2) FF_PROP(3) FF_PROP(4)
#undef FF_PROP
}

static void launch_propagate(int bh, int r, int bands, int bands_a, hipStream_t stream, const FieldRec* table, int f0,
                             int nf, const PropLaunch& L) {
  if (bh == 8)
    launch_propagate_bh<8>(r, bands, bands_a, stream, table, f0, nf, L);
  else if (bh == 32)
    launch_propagate_bh<32>(r, bands, bands_a, stream, table, f0, nf, L);
  else
    launch_propagate_bh<16>(r, bands, bands_a, stream, table, f0, nf, L);
}

// ---------------------------------------------------------------- host plans
struct FieldPlan {
  bool has_tree;
  TreeLayout tree;        // offsets relative to the field region
  size_t off_grid[5];
  size_t off_xch, off_xch2, off_prog;
  size_t bytes;
};

static FieldPlan field_plan(const ff_desc* src, const ff_desc* dst, const ff_match_params* p) {
  FieldPlan P{};
  size_t off = 0;
  P.has_tree = p->use_kdtree != 0;
  if (P.has_tree) {
    P.tree = tree_layout(dst->width * dst->height, p->leaf, 0);
    off = P.tree.bytes;
  }
  for (int lev = 1; lev <= p->k; ++lev) {
    const int n = 1 << lev;
    const size_t G = (size_t)((src->width + n - 1) / n) * ((src->height + n - 1) / n);
    off = align_up(off, 256);
    P.off_grid[lev] = off;
    off += G * 8;
  }
  const size_t nb = (size_t)((src->height + kMinBandRows - 1) / kMinBandRows);
  off = align_up(off, 256);
  P.off_xch = off;
  off = align_up(off + nb * src->width * 8, 256);
  P.off_xch2 = off;
  off = align_up(off + nb * src->width * 8, 256);
  P.off_prog = off;
  off += 2 * (size_t)prog_words(src->height) * 4;
  P.bytes = align_up(off, 256);
  return P;
}

static int band_rows_of(const ff_match_params* p) { return p->band_rows == 0 ? 16 : p->band_rows; }

static ff_status check_params(const ff_desc* src, const ff_desc* dst, int radius, const ff_match_params* p) {
  if (!src || !dst || !p) return FF_ERR_ARG;
  if (src->channels != dst->channels || src->subpel != dst->subpel) return FF_ERR_ARG;
  if (p->k < 0 || p->k > src->k || p->k > dst->k) return FF_ERR_ARG;
  if (radius < 1 || radius > kMaxRadius) return FF_ERR_ARG;
  if (p->R < 0 || p->R > 64 || p->n_prop < 0 || p->n_prop > 64 || p->n_rs < 0 || p->n_rs > p->n_prop) return FF_ERR_ARG;
  if (p->field_id > 3) return FF_ERR_ARG;
  if (p->band_rows != 0 && p->band_rows != 8 && p->band_rows != 16 && p->band_rows != 32) return FF_ERR_ARG;
  if (p->pipeline != 0 && p->pipeline != 1) return FF_ERR_ARG;
  if (p->watchdog_us < 0) return FF_ERR_ARG;
  if (p->use_kdtree < 0 || p->use_kdtree > 2) return FF_ERR_ARG;
  if (p->use_kdtree) {
    if (p->leaf < 2 || p->leaf > kMaxLeaf) return FF_ERR_ARG;
    bool hs = false, hd = false;
    for (int i = 0; i < src->n_radii; ++i) hs |= src->radii[i] == radius;
    for (int i = 0; i < dst->n_radii; ++i) hd |= dst->radii[i] == radius;
    if (!hs || !hd) return FF_ERR_ARG;
  }
  return FF_OK;
}

static ff_status check_job(const ff_field_job& j, const ff_match_params* p) {
  ff_match_params q = *p;
  q.field_id = j.field_id;
  ff_status st = check_params(j.src, j.dst, j.radius, &q);
  if (st != FF_OK) return st;
  if (!j.src_blob || !j.dst_blob || !j.flow || !j.cost) return FF_ERR_ARG;
  if (!p->use_kdtree && !j.proposal) return FF_ERR_ARG;
  return FF_OK;
}

// Per-job host arrays of a call: held inline for a single job (so that the
// single-field entry points touch no host heap either), on the heap for more.
template <class T>
struct JobArray {
  T one{};
  std::vector<T> many;
  int n = 0;
  void resize(int k) {
    n = k;
    if (k > 1) many.assign((size_t)k, T{});
  }
  T& operator[](int i) { return n > 1 ? many[(size_t)i] : one; }
  const T& operator[](int i) const { return n > 1 ? many[(size_t)i] : one; }
};

struct BatchLayout {
  size_t off_tickets, off_table;
  int launches;
  JobArray<size_t> off_field;   // per table entry
  JobArray<int> order;          // table entry -> job index (grouped by radius)
  size_t bytes;
};

static BatchLayout batch_layout(const ff_field_job* jobs, int n, const ff_match_params* p) {
  BatchLayout B;
  B.order.resize(n);
  for (int i = 0; i < n; ++i) B.order[i] = i;
  if (n > 1)
    std::stable_sort(B.order.many.begin(), B.order.many.end(),
                     [&](int a, int b) { return jobs[a].radius > jobs[b].radius; });
  int groups = 0;
  for (int i = 0; i < n; ++i)
    if (i == 0 || jobs[B.order[i]].radius != jobs[B.order[i - 1]].radius) ++groups;
  size_t off = kStatusBytes;
  B.off_tickets = off;
  B.launches = (p->k + 1) * p->n_prop * groups;
  off = align_up(off + (size_t)B.launches * 4, 256);
  B.off_table = off;
  off = align_up(off + (size_t)n * sizeof(FieldRec), 256);
  B.off_field.resize(n);
  for (int i = 0; i < n; ++i) {
    const ff_field_job& j = jobs[B.order[i]];
    B.off_field[i] = off;
    off = align_up(off + field_plan(j.src, j.dst, p).bytes, 256);
  }
  B.bytes = off;
  return B;
}

static FieldRec make_rec(const ff_field_job& j, const ff_match_params* p, char* fws) {
  const ff_desc* s = j.src;
  const ff_desc* d = j.dst;
  const FieldPlan P = field_plan(s, d, p);
  FieldRec r{};
  r.src = census_plane(s, j.src_blob, 0, 0, 0);
  r.srcT = census_plane_t(s, j.src_blob, 0, 0, 0);
  r.dst = census_plane(d, j.dst_blob, 0, 0, 0);
  r.dstT = census_plane_t(d, j.dst_blob, 0, 0, 0);
  r.Vsrc = p->use_kdtree ? wht_block(s, j.src_blob, j.radius) : nullptr;
  r.Vdst = p->use_kdtree ? wht_block(d, j.dst_blob, j.radius) : nullptr;
  r.proposal = j.proposal;
  r.flow = j.flow;
  r.cost = j.cost;
  r.ws = fws;
  r.pws = (uint32_t)(s->width * s->height);
  r.pwd = (uint32_t)(d->width * d->height);
  r.Ws = s->width;
  r.Hs = s->height;
  r.Wd = d->width;
  r.Hd = d->height;
  r.r = j.radius;
  r.D = d->wht_dims;
  r.vstride = d->wht_stride;
  r.k0 = (uint32_t)(j.seed & 0xFFFFFFFFu);
  r.k1 = (uint32_t)(j.seed >> 32);
  r.c3 = j.field_id | (j.pair_id << 2);
  if (P.has_tree) {
    r.t_nodes = P.tree.nodes;
    r.t_top = P.tree.top;
    r.o_dim = (uint32_t)P.tree.off_dim;
    r.o_split = (uint32_t)P.tree.off_split;
    r.o_perm = (uint32_t)P.tree.off_perm;
    r.o_perm2 = (uint32_t)P.tree.off_perm2;
    r.o_mm = (uint32_t)P.tree.off_minmax;
    r.o_hist = (uint32_t)P.tree.off_hist;
    r.o_cnt = (uint32_t)P.tree.off_cnt;
    r.o_key = (uint32_t)P.tree.off_key;
  }
  for (int l = 0; l < 5; ++l) r.o_grid[l] = (uint32_t)P.off_grid[l];
  r.o_xch = (uint32_t)P.off_xch;
  r.o_xch2 = (uint32_t)P.off_xch2;
  r.o_prog = (uint32_t)P.off_prog;
  return r;
}

static void write_table(const JobArray<FieldRec>& recs, int nrec, FieldRec* dev, hipStream_t stream) {
  for (int i = 0; i < nrec; i += kRecsPerWrite) {
    RecChunk ch{};
    const int n = std::min(kRecsPerWrite, nrec - i);
    for (int k = 0; k < n; ++k) ch.r[k] = recs[i + k];
    k_write_table<<<1, kRecsPerWrite, 0, stream>>>(ch, n, dev + i);
  }
}

// The whole search for a batch of fields.  Every stage is one launch over
// all fields (propagation: one launch per patch radius).
// tree_only: the call's set-up and the kd-tree build, nothing after (the
// tree stays in the workspace for a later call with use_kdtree = 2)
static ff_status run_batch(const ff_field_job* jobs, int n, const ff_match_params* p, char* ws, const BatchLayout& B,
                           hipStream_t stream, bool tree_only = false) {
  int32_t* status = reinterpret_cast<int32_t*>(ws);
  int32_t* tickets = reinterpret_cast<int32_t*>(ws + B.off_tickets);
  FieldRec* table = reinterpret_cast<FieldRec*>(ws + B.off_table);
  JobArray<FieldRec> recs;
  recs.resize(n);
  int maxW = 0, maxH = 0, maxN = 0, maxTop = 0, maxG = 0;
  for (int i = 0; i < n; ++i) {
    const ff_field_job& j = jobs[B.order[i]];
    recs[i] = make_rec(j, p, ws + B.off_field[i]);
    maxW = std::max(maxW, recs[i].Ws);
    maxH = std::max(maxH, recs[i].Hs);
    maxN = std::max(maxN, recs[i].Wd * recs[i].Hd);
    maxTop = std::max(maxTop, recs[i].t_top);
    maxG = std::max(maxG, recs[i].Ws * recs[i].Hs);
  }
  const int qshift = ilog2i(jobs[0].dst->subpel);
  const int k = p->k;
  const int bh = band_rows_of(p);
  fill_i32(status, 1, 0, stream);
  fill_i32(tickets, (size_t)B.launches, 0, stream);
  write_table(recs, n, table, stream);
  k_clear_xch<<<dim3(64, n), 256, 0, stream>>>(table, kMinBandRows);
  if (p->use_kdtree == 1 || tree_only) {
    prof_mark(FF_PROF_TREE, stream, true);
    ff_status st = enqueue_tree_build(table, n, maxN, maxTop, p->leaf, stream);
    prof_mark(FF_PROF_TREE, stream, false);
    if (st != FF_OK) return st;
  }
  if (tree_only) return launch_status();
  auto pts = [&](int lev) { return ((maxW + (1 << lev) - 1) >> lev) * ((maxH + (1 << lev) - 1) >> lev); };
  // random search: one workgroup per 256 / kLanesPt consecutive points of a grid row
  auto rs_blocks = [&](int lev) {
    const int pt = 256 / kLanesPt;
    return (unsigned)((((maxW + (1 << lev) - 1) >> lev) + pt - 1) / pt * ((maxH + (1 << lev) - 1) >> lev));
  };
  // pipelined launches need tags below 2^12 (progress words) and no
  // inspection stops between their stages
  const bool pipe = p->pipeline == 1 && p->max_steps < 0 && B.launches < 4096;
  int steps = 0, cur_lev = k;
  auto stop = [&]() { return p->max_steps >= 0 && steps >= p->max_steps; };
  auto finish = [&]() -> ff_status {
    if (cur_lev > 0) k_write_grid<<<dim3((maxW + 255) / 256, maxH, n), 256, 0, stream>>>(table, cur_lev);
    return launch_status();
  };
  prof_mark(FF_PROF_SEED, stream, true);
  k_seed<<<dim3((pts(k) + 3) / 4, n), 256, 0, stream>>>(table, k, qshift, p->use_kdtree ? 1 : 0);
  prof_mark(FF_PROF_SEED, stream, false);
  ++steps;
  if (stop()) return finish();
  // watchdog for the propagation's inter-band waits: 2 s of the 100 MHz clock
  const uint64_t timeout = p->watchdog_us > 0 ? (uint64_t)p->watchdog_us * 100u : 200000000ull;
  int launch = 0;
  auto sx_of = [](int i) { return ((i & 3) == 0 || (i & 3) == 3) ? 1 : -1; };
  auto sy_of = [](int i) { return ((i & 3) == 0 || (i & 3) == 2) ? 1 : -1; };
  auto bands_at = [&](int g0, int g1, int lv) {
    int bands = 0;
    for (int g = g0; g < g1; ++g) bands += (((recs[g].Hs + (1 << lv) - 1) >> lv) + bh - 1) / bh;
    return bands;
  };
  // one launch per patch radius group
  auto propagate = [&](PropLaunch L) {
    prof_mark(FF_PROF_PROPAGATE, stream, true);
    for (int g0 = 0; g0 < n;) {
      int g1 = g0;
      while (g1 < n && recs[g1].r == recs[g0].r) ++g1;
      const int bands = bands_at(g0, g1, L.lev);
      const int bands_a = L.pair == kPairCross ? bands_at(g0, g1, L.lev + 1) : bands;
      L.tag = (uint32_t)(launch + 1);
      L.ticket = tickets + launch;
      launch_propagate(bh, recs[g0].r, bands, bands_a, stream, table, g0, g1 - g0, L);
      ++launch;
      g0 = g1;
    }
    prof_mark(FF_PROF_PROPAGATE, stream, false);
  };
  auto rsearch = [&](int lv, int step) {
    prof_mark(FF_PROF_RANDOM_SEARCH, stream, true);
    k_random_search<kLanesPt><<<dim3(rs_blocks(lv), n), 256, 0, stream>>>(table, lv, qshift, step, p->R);
    prof_mark(FF_PROF_RANDOM_SEARCH, stream, false);
  };
  bool entered = false;   // this level's entry and first sweep ran in a cross-level pair
  for (int lev = k; lev >= 0; --lev) {
    cur_lev = lev;
    int i = 0;
    if (entered) {
      i = 1;
      entered = false;
    } else if (lev < k) {
      // one group of lanes per point of the coarser grid
      const unsigned gpts = (unsigned)(((size_t)pts(lev + 1) * kLanesPt + 255) / 256);
      prof_mark(FF_PROF_LEVEL_ENTRY, stream, true);
      k_level_entry<kLanesPt><<<dim3(gpts, n), 256, 0, stream>>>(table, lev, qshift);
      prof_mark(FF_PROF_LEVEL_ENTRY, stream, false);
      ++steps;
      if (stop()) return finish();
    }
    while (i < p->n_prop) {
      PropLaunch L{lev, qshift, sx_of(i), sy_of(i), 0, nullptr, status, timeout, 0, -1, p->R};
      if (pipe && i + 1 < p->n_prop && sx_of(i + 1) == sx_of(i)) {
        // sweeps i and i + 1 (opposite vertical directions) as one pipelined
        // launch with the random search between them; the search after
        // sweep i + 1 follows on its own
        L.pair = kPairSame;
        L.rs = i < p->n_rs ? i : -1;
        propagate(L);
        if (i + 1 < p->n_rs) rsearch(lev, i + 1);
        i += 2;
        continue;
      }
      if (pipe && i == p->n_prop - 1 && i >= p->n_rs && lev > 0 && sx_of(0) == sx_of(i) && sy_of(0) == -sy_of(i)) {
        // the level's last sweep (no search after it), the next level's
        // entry and its first sweep as one pipelined launch
        L.lev = lev - 1;
        L.pair = kPairCross;
        propagate(L);
        if (p->n_rs > 0) rsearch(lev - 1, 0);
        entered = true;
        ++i;
        continue;
      }
      propagate(L);
      ++steps;
      if (stop()) return finish();
      if (i < p->n_rs) {
        rsearch(lev, i);
        ++steps;
        if (stop()) return finish();
      }
      ++i;
    }
  }
  (void)maxG;
  cur_lev = 0;
  return finish();
}

// ---------------------------------------------------------------- no-allocation scratch
// ff_match_field_noalloc keeps what ff_match_field keeps in its workspace
// (status word, tickets, field table, kd-tree, level grids, handoff and
// progress words) in this one static array per device.  On the host its name
// is only a stand-in symbol, not a device address: host code uses the address
// hipGetSymbolAddress returns for the current device, looked up once per
// device (at ff_init, else at the entry point's first call there).
static __device__ __align__(256) char scratch[FF_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
char* g_scratch_ptr[64];
}  // namespace

ff_status noalloc_scratch(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FF_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FF_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  if (out) *out = g_scratch_ptr[dev];
  return FF_OK;
}

__global__ void k_copy_status(const int32_t* __restrict__ from, int32_t* __restrict__ to) { *to = *from; }

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
  p->band_rows = 16;
  p->pipeline = 1;
}

size_t ff_match_batch_workspace_bytes(const ff_field_job* jobs, int32_t n_jobs, const ff_match_params* p) {
  if (!jobs || !p || n_jobs < 1 || n_jobs > 4096) return 0;
  for (int i = 0; i < n_jobs; ++i) {
    ff_match_params q = *p;
    q.field_id = jobs[i].field_id;
    if (!jobs[i].src || !jobs[i].dst || check_params(jobs[i].src, jobs[i].dst, jobs[i].radius, &q) != FF_OK) return 0;
    if (jobs[i].dst->subpel != jobs[0].dst->subpel) return 0;
  }
  return batch_layout(jobs, n_jobs, p).bytes;
}

ff_status ff_match_batch(const ff_field_job* jobs, int32_t n_jobs, const ff_match_params* p, void* workspace,
                         size_t workspace_bytes, hipStream_t stream) {
  if (!jobs || !p || !workspace || n_jobs < 1 || n_jobs > 4096) return FF_ERR_ARG;
  // a tree left in the workspace by ff_match_field_tree belongs to one field
  if (p->use_kdtree == 2 && n_jobs != 1) return FF_ERR_ARG;
  for (int i = 0; i < n_jobs; ++i) {
    if (!jobs[i].src || !jobs[i].dst) return FF_ERR_ARG;
    ff_status st = check_job(jobs[i], p);
    if (st != FF_OK) return st;
    if (jobs[i].dst->subpel != jobs[0].dst->subpel) return FF_ERR_ARG;
  }
  const BatchLayout B = batch_layout(jobs, n_jobs, p);
  if (workspace_bytes < B.bytes) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  return run_batch(jobs, n_jobs, p, static_cast<char*>(workspace), B, stream);
}

static ff_field_job single_job(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                               int32_t radius, const ff_match_params* p, const int32_t* proposal, int32_t* flow,
                               int32_t* cost) {
  ff_field_job j{};
  j.src = src;
  j.src_blob = src_blob;
  j.dst = dst;
  j.dst_blob = dst_blob;
  j.radius = radius;
  j.field_id = p ? p->field_id : 0;
  j.pair_id = p ? p->pair_id : 0;
  j.seed = p ? p->seed : 0;
  j.proposal = proposal;
  j.flow = flow;
  j.cost = cost;
  return j;
}

size_t ff_match_workspace_bytes(const ff_desc* src, const ff_desc* dst, int32_t radius, const ff_match_params* p) {
  if (check_params(src, dst, radius, p) != FF_OK) return 0;
  const ff_field_job j = single_job(src, nullptr, dst, nullptr, radius, p, nullptr, nullptr, nullptr);
  return batch_layout(&j, 1, p).bytes;
}

ff_status ff_match_field(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                         int32_t radius, const ff_match_params* p, const int32_t* proposal, int32_t* flow,
                         int32_t* cost, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!p) return FF_ERR_ARG;
  const ff_field_job j = single_job(src, src_blob, dst, dst_blob, radius, p, proposal, flow, cost);
  return ff_match_batch(&j, 1, p, workspace, workspace_bytes, stream);
}

ff_status ff_match_field_tree(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                              int32_t radius, const ff_match_params* p, void* workspace, size_t workspace_bytes,
                              hipStream_t stream) {
  if (!p || !workspace || !p->use_kdtree) return FF_ERR_ARG;
  ff_status st = check_params(src, dst, radius, p);
  if (st != FF_OK) return st;
  const ff_field_job j = single_job(src, src_blob, dst, dst_blob, radius, p, nullptr, nullptr, nullptr);
  if (!src_blob || !dst_blob) return FF_ERR_ARG;
  const BatchLayout B = batch_layout(&j, 1, p);
  if (workspace_bytes < B.bytes) return FF_ERR_WORKSPACE;
  st = ensure_init();
  if (st != FF_OK) return st;
  return run_batch(&j, 1, p, static_cast<char*>(workspace), B, stream, true);
}

ff_status ff_match_field_noalloc(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                                 int32_t radius, const ff_match_params* p, const int32_t* proposal, int32_t* flow,
                                 int32_t* cost, int32_t* status, hipStream_t stream) {
  // the library's scratch never holds a tree built ahead by ff_match_field_tree
  if (!p || p->use_kdtree == 2) return FF_ERR_ARG;
  ff_status st = check_params(src, dst, radius, p);
  if (st != FF_OK) return st;
  const ff_field_job j = single_job(src, src_blob, dst, dst_blob, radius, p, proposal, flow, cost);
  const BatchLayout B = batch_layout(&j, 1, p);
  if (B.bytes > (size_t)FF_NOALLOC_SCRATCH_BYTES) return FF_ERR_SIZE;
  st = check_job(j, p);
  if (st != FF_OK) return st;
  st = ensure_init();
  if (st != FF_OK) return st;
  char* ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st != FF_OK) return st;
  st = run_batch(&j, 1, p, ws, B, stream);
  if (st != FF_OK) return st;
  if (status) {
    k_copy_status<<<1, 1, 0, stream>>>(reinterpret_cast<const int32_t*>(ws), status);
    return launch_status();
  }
  return FF_OK;
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
  if (!wht_block(d, blob, radius)) return FF_ERR_ARG;
  ff_match_params p;
  ff_default_params(&p);
  p.k = 0;
  p.leaf = leaf;
  const ff_field_job j = single_job(d, blob, d, blob, radius, &p, nullptr, node_dim, node_split);
  const BatchLayout B = batch_layout(&j, 1, &p);
  if (workspace_bytes < B.bytes) return FF_ERR_WORKSPACE;
  ff_status st = ensure_init();
  if (st != FF_OK) return st;
  char* ws = static_cast<char*>(workspace);
  JobArray<FieldRec> recs;
  recs.resize(1);
  recs[0] = make_rec(j, &p, ws + B.off_field[0]);
  FieldRec* table = reinterpret_cast<FieldRec*>(ws + B.off_table);
  write_table(recs, 1, table, stream);
  st = enqueue_tree_build(table, 1, d->width * d->height, recs[0].t_top, leaf, stream);
  if (st != FF_OK) return st;
  const char* fws = ws + B.off_field[0];
  const int N = d->width * d->height;
  if (hipMemcpyAsync(node_dim, fws + recs[0].o_dim, (size_t)recs[0].t_nodes * 4, hipMemcpyDeviceToDevice, stream) !=
          hipSuccess ||
      hipMemcpyAsync(node_split, fws + recs[0].o_split, (size_t)recs[0].t_nodes * 4, hipMemcpyDeviceToDevice,
                     stream) != hipSuccess ||
      hipMemcpyAsync(perm, fws + recs[0].o_perm, (size_t)N * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return FF_ERR_HIP;
  return FF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- load-latency probe
// One wavefront follows a cycle of indices through global memory (every
// lane the same one): every hop is one load whose address is the previous
// load's value, so a hop costs one dependent round trip to wherever the
// cycle's lines live.  The sweep's step
// is such a chain (a step's result decides the next step's target
// addresses), so this round trip times the number of wavefront steps is the
// floor a sweep cannot go below.
namespace ff {
__global__ void k_chase(const int32_t* __restrict__ next, int32_t mask, int32_t warm, int32_t hops,
                        int64_t* __restrict__ out) {
  const __attribute__((address_space(1))) int32_t* p = gp(next);
  // a lane-varying start (0 in every lane of the one wavefront launched)
  // keeps the walk in vector registers, so every hop is a vector-memory load
  // through the vector L1 and the L2, the path of the sweep's target loads,
  // not a scalar-cache load
  int32_t i = (int32_t)(threadIdx.x >> 6);
  for (int h = 0; h < warm; ++h) i = p[i] & mask;
  // the clock is read once the warm walk's last load has returned, and again
  // once the timed walk's has (the asm consumes the index in a register)
  asm volatile("" ::"v"(i));
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  for (int h = 0; h < hops; ++h) i = p[i] & mask;
  asm volatile("" ::"v"(i));
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) {
    out[0] = (int64_t)(t1 - t0);
    out[1] = i;
  }
}
}  // namespace ff

extern "C" ff_status ff_probe_load_latency(const int32_t* next, int32_t n, int32_t warm, int32_t hops, int64_t* out,
                                           hipStream_t stream) {
  if (!next || !out || n < 2 || n > (1 << 28) || (n & (n - 1)) != 0) return FF_ERR_ARG;
  // at most 2^22 hops per walk: a few seconds even if every hop went to HBM
  if (hops < 1 || hops > (1 << 22) || warm < 0 || warm > (1 << 22)) return FF_ERR_ARG;
  k_chase<<<1, 64, 0, stream>>>(next, n - 1, warm, hops, out);
  return launch_status();
}
