// The Flow Field search of sections 3.1 and 3.2 with the SIFT-flow data term
// of section 3.3, for a batch of fields in one call.
//
// Data term E^n_r(p, f): over the (2r+1)^2 samples at stride n, the L2
// distance of the first S colours of the level's smoothed colour images,
// the target side bilinear in the four neighbours of floor(m / Q) + n delta
// at the subpixel phase m mod Q (m = pQ + f; the +1 neighbours clamp), the
// source side scaled by Q^2: floor(sqrt(sum_s d_s^2 * 256 / Q^4)) per sample
// (1/16 code units at every Q), summed; lookups clamp to the image; f is
// invalid ("infinite") unless m lies in the image.  All integer, so every
// decision of the search is exact.
//
// Stages: kd-tree seeds over the CIELab WHT vectors (section 3.1; the tree
// build of the census search), re-ranked by this data term on the 2^k grid
// (Eq. 4); per level the alternating propagation sweeps (Eq. 2) and random
// searches (R_n = R n), coarse flows seeding the next level.
//
// Propagation: one workgroup per band of 4 grid rows, one wavefront per row
// (small bands: more of the chip at work, and each step waits on the
// slowest of fewer memory round trips).
// At step t, row i of the band handles column u = t - i (sweep-transformed
// coordinates): its vertical candidate is row i - 1's result of step t - 1
// (LDS), its horizontal candidate its own result of step t - 1; row 0 takes
// the band above's last-row result from a 64-bit word (cost | flow) that the
// band above stores with an agent-scope atomic.  A candidate is costed with
// a sliding window: its predecessor's cost minus the row (column) leaving
// the patch plus the one entering it, 2 (2r+1) samples, all loaded at once.
// Bands are numbered by a ticket, so a band only ever waits on a band that
// started before it.
#include <algorithm>
#include <vector>

#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

constexpr int kSBand = 4;     // grid rows per propagation band (one wavefront each)
constexpr int kSLanes = 16;   // lanes per point (entry, random search): one DPP row
constexpr int kSiftRecsPerWrite = 16;
constexpr int kSiftStatusBytes = 256;

struct SiftRec {
  const int16_t* src;    // colour levels: (levels) x Hs x Ws x P int16
  const int16_t* dst;
  const int32_t* Vsrc;   // source WHT vectors of radius r (seed queries)
  int32_t* flow;         // outputs (the level-1 grid)
  int32_t* cost;
  char* ws;              // field region: kd-tree, grids of levels 2..2^k, handoff words
  int32_t Ws, Hs, Wd, Hd;
  int32_t P, S, r, vstride;
  uint32_t k0, k1, c3, t_nodes;
  uint32_t o_dim, o_split, o_perm, o_xch;
  uint32_t o_grid[5];
  uint32_t pad[3];
};

struct SCtx {
  const int16_t* src;
  const int16_t* dst;
  int Ws, Hs, Wd, Hd, P, S, r, n, Q, qshift;
};

__device__ __forceinline__ SCtx sctx_of(const SiftRec& f, int lev, int qshift) {
  SCtx c;
  c.src = f.src + (size_t)lev * f.Ws * f.Hs * f.P;
  c.dst = f.dst + (size_t)lev * f.Wd * f.Hd * f.P;
  c.Ws = f.Ws;
  c.Hs = f.Hs;
  c.Wd = f.Wd;
  c.Hd = f.Hd;
  c.P = f.P;
  c.S = f.S;
  c.r = f.r;
  c.n = 1 << lev;
  c.Q = 1 << qshift;
  c.qshift = qshift;
  return c;
}

__device__ __forceinline__ int32_t* sgrid_flow(const SiftRec& f, int lev) {
  return lev == 0 ? f.flow : reinterpret_cast<int32_t*>(f.ws + f.o_grid[lev]);
}
__device__ __forceinline__ int32_t* sgrid_cost(const SiftRec& f, int lev, int G) {
  return lev == 0 ? f.cost : reinterpret_cast<int32_t*>(f.ws + f.o_grid[lev]) + G;
}

__device__ __forceinline__ bool svalid(const SCtx& c, int px, int py, int32_t f) {
  const int mx = px * c.Q + fx_of(f), my = py * c.Q + fy_of(f);
  return mx >= 0 && my >= 0 && mx <= (c.Wd - 1) * c.Q && my <= (c.Hd - 1) * c.Q;
}

// floor(sqrt(v)) for v < 2^46: a float estimate (from the two 32-bit
// halves), corrected exactly; the root is below 2^23, so its squares are
// full-rate 24-bit products
__device__ __forceinline__ uint64_t sq24(uint32_t x) {
  const uint32_t y = x & 0xFFFFFFu;   // no-op here: x < 2^24
  return (uint64_t)y * y;
}
__device__ __forceinline__ uint32_t isqrt_u64(uint64_t v) {
  const float fv = fmaf((float)(uint32_t)(v >> 32), 4294967296.0f, (float)(uint32_t)v);
  uint32_t k = min((uint32_t)sqrtf(fv), 0x7FFFFFu);
  while (sq24(k) > v) --k;
  while (sq24(k + 1) <= v) ++k;
  return k;
}

typedef short short4_t __attribute__((ext_vector_type(4)));

// Bilinear target weights of a candidate and its integer target centre.
struct Tgt {
  int Mx, My, w00, w10, w01, w11;
};

__device__ __forceinline__ Tgt tgt_of(const SCtx& c, int px, int py, int32_t f) {
  const int mx = px * c.Q + fx_of(f), my = py * c.Q + fy_of(f);
  Tgt t;
  t.Mx = mx >> c.qshift;
  t.My = my >> c.qshift;
  const int a = mx & (c.Q - 1), b = my & (c.Q - 1);
  // weights <= Q^2 <= 64: the masks (no-ops) let the products with the
  // colours compile to full-rate 24-bit multiplies
  t.w00 = ((c.Q - a) * (c.Q - b)) & 0x7F;
  t.w10 = (a * (c.Q - b)) & 0x7F;
  t.w01 = ((c.Q - a) * b) & 0x7F;
  t.w11 = (a * b) & 0x7F;
  return t;
}

// The colours of one pixel as SG groups of 4 int16 (8-byte loads).  Groups
// at or past the field's ceil(S/4) are not loaded (zero, and masked out by
// the channel test).
template <int SG>
struct Px {
  short4_t v[SG];
};

template <int SG>
__device__ __forceinline__ Px<SG> load_px(const int16_t* p, int sgf) {
  Px<SG> r;
  const short4_t* q = reinterpret_cast<const short4_t*>(p);
#pragma unroll
  for (int g = 0; g < SG; ++g) {
    if (g < sgf)   // uniform: a field's channel count
      r.v[g] = q[g];
    else
      r.v[g] = short4_t{0, 0, 0, 0};
  }
  return r;
}

// the target's four neighbours of (X, Y) (already clamped)
template <int SG>
struct Quad {
  Px<SG> p00, p10, p01, p11;
};

// int16 offset of pixel (x, y) in a plane of width w and pitch P: below
// 2^27 (pixels < 2^22, P <= 32), so 32-bit full-rate 24-bit products
__device__ __forceinline__ uint32_t pix_off(int x, int y, int w, int P) {
  return __umul24(__umul24((uint32_t)y, (uint32_t)w) + (uint32_t)x, (uint32_t)P);
}

template <int SG>
__device__ __forceinline__ Quad<SG> load_quad(const SCtx& c, int X, int Y, int sgf) {
  const int X1 = min(X + 1, c.Wd - 1), Y1 = min(Y + 1, c.Hd - 1);
  Quad<SG> q;
  q.p00 = load_px<SG>(c.dst + pix_off(X, Y, c.Wd, c.P), sgf);
  q.p10 = load_px<SG>(c.dst + pix_off(X1, Y, c.Wd, c.P), sgf);
  q.p01 = load_px<SG>(c.dst + pix_off(X, Y1, c.Wd, c.P), sgf);
  q.p11 = load_px<SG>(c.dst + pix_off(X1, Y1, c.Wd, c.P), sgf);
  return q;
}

// floor(sqrt(sum_s d_s^2 * 256 / Q^4)) of one sample.  Every factor fits 24
// signed bits (weights and Q^2 <= 64, colours int16, |d_s| < 2^22), so the
// products are full-rate 24-bit multiplies (the 64-bit square from its low
// and high halves).
template <int SG>
__device__ __forceinline__ int32_t dist_of(const SCtx& c, const Px<SG>& a, const Quad<SG>& q, const Tgt& t) {
  const int QQ = (c.Q * c.Q) & 0x7F;
  uint64_t ss = 0;
#pragma unroll
  for (int g = 0; g < SG; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = __mul24(QQ, (int)a.v[g][i]) -
                    (__mul24(t.w00, (int)q.p00.v[g][i]) + __mul24(t.w10, (int)q.p10.v[g][i]) +
                     __mul24(t.w01, (int)q.p01.v[g][i]) + __mul24(t.w11, (int)q.p11.v[g][i]));
      const int em = g * 4 + i < c.S ? e : 0;
      const int e24 = (int)((uint32_t)em << 8) >> 8;   // no-op: |em| < 2^23
      ss += (uint64_t)((int64_t)e24 * e24);
    }
  const uint64_t v = c.qshift <= 2 ? ss << (8 - 4 * c.qshift) : ss >> 4;
  return (int32_t)isqrt_u64(v);
}

// this lane's share (samples lane, lane + L, ...) of E for candidate f
template <int SG>
__device__ __forceinline__ int32_t sift_partial(const SCtx& c, int px, int py, int32_t f, int lane, int L) {
  const Tgt t = tgt_of(c, px, py, f);
  const int Sd = 2 * c.r + 1, sgf = (c.S + 3) >> 2;
  int32_t sum = 0;
  for (int k = lane; k < Sd * Sd; k += L) {
    const int iy = k / Sd, ix = k - iy * Sd;
    const int dx = (ix - c.r) * c.n, dy = (iy - c.r) * c.n;
    const int sx = clampi(px + dx, 0, c.Ws - 1), sy = clampi(py + dy, 0, c.Hs - 1);
    const Px<SG> a = load_px<SG>(c.src + pix_off(sx, sy, c.Ws, c.P), sgf);
    const Quad<SG> q = load_quad<SG>(c, clampi(t.Mx + dx, 0, c.Wd - 1), clampi(t.My + dy, 0, c.Hd - 1), sgf);
    sum += dist_of<SG>(c, a, q, t);
  }
  return sum;
}


// ---------------------------------------------------------------- table, clears
struct SiftChunk {
  SiftRec r[kSiftRecsPerWrite];
};
struct TreeChunk {
  FieldRec r[kSiftRecsPerWrite];
};

__global__ void k_sift_write_table(SiftChunk chunk, int n, SiftRec* __restrict__ out) {
  if ((int)threadIdx.x < n) out[threadIdx.x] = chunk.r[threadIdx.x];
}
__global__ void k_tree_write_table(TreeChunk chunk, int n, FieldRec* __restrict__ out) {
  if ((int)threadIdx.x < n) out[threadIdx.x] = chunk.r[threadIdx.x];
}

// mark every field's first handoff buffer empty (grid: chunks x fields)
__global__ void k_sift_clear_xch(const SiftRec* __restrict__ table) {
  const SiftRec& f = table[blockIdx.y];
  uint64_t* x = reinterpret_cast<uint64_t*>(f.ws + f.o_xch);
  const size_t nw = (size_t)((f.Hs + kSBand - 1) / kSBand) * f.Ws;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x)
    x[i] = ~0ull;
}

// ---------------------------------------------------------------- seeds (Eq. 1 / Eq. 4)
// One wavefront per coarse grid point: descend the kd-tree with the source
// WHT vector, re-rank the leaf (ascending pixel index) by the data term;
// the first minimum wins.  grid: (points / 4, fields)
template <int SG>
__global__ __launch_bounds__(256) void k_sift_seed(const SiftRec* __restrict__ table, int lev, int qshift) {
  const SiftRec& f = table[blockIdx.y];
  const SCtx c = sctx_of(f, lev, qshift);
  const int Gw = (f.Ws + c.n - 1) >> lev, Gh = (f.Hs + c.n - 1) >> lev;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= Gw * Gh) return;
  const int gx = wave % Gw, gy = wave / Gw;
  const int px = gx * c.n, py = gy * c.n;
  const int32_t* node_dim = reinterpret_cast<const int32_t*>(f.ws + f.o_dim);
  const int32_t* node_split = reinterpret_cast<const int32_t*>(f.ws + f.o_split);
  const int32_t* perm = reinterpret_cast<const int32_t*>(f.ws + f.o_perm);
  const int Nd = f.Wd * f.Hd;
  const int32_t* q = f.Vsrc + ((size_t)py * f.Ws + px) * f.vstride;
  int node = 0, start = 0, cnt = Nd;
  for (;;) {
    const int dim = node_dim[node];
    if (dim < 0 || 2 * node + 2 >= (int)f.t_nodes) break;
    const int h = cnt >> 1;
    if (q[dim] >= node_split[node]) {
      node = 2 * node + 2;
      start += h;
      cnt -= h;
    } else {
      node = 2 * node + 1;
      cnt = h;
    }
  }
  int32_t bestF = kEmpty, bestC = kInf;
  for (int i = 0; i < cnt && start + i < Nd; ++i) {
    const int id = perm[start + i];
    const int32_t fl = packf((id % f.Wd - px) * c.Q, (id / f.Wd - py) * c.Q);
    const int32_t e = wave_sum(sift_partial<SG>(c, px, py, fl, lane, 64));
    if (e < bestC) {
      bestC = e;
      bestF = fl;
    }
  }
  if (lane == 0) {
    sgrid_flow(f, lev)[(size_t)gy * Gw + gx] = bestF;
    sgrid_cost(f, lev, Gw * Gh)[(size_t)gy * Gw + gx] = bestC;
  }
}

// ---------------------------------------------------------------- level entry
// Section 3.2: the coarser grid's points keep their flow, re-costed with
// this level's patch; new points start empty.  16 lanes per coarse point,
// which also write the three new points it covers.
template <int SG>
__global__ __launch_bounds__(256) void k_sift_entry(const SiftRec* __restrict__ table, int lev, int qshift) {
  const SiftRec& f = table[blockIdx.y];
  const SCtx c = sctx_of(f, lev, qshift);
  const int Gw = (f.Ws + c.n - 1) >> lev, Gh = (f.Hs + c.n - 1) >> lev;
  const int Gwc = (f.Ws + 2 * c.n - 1) >> (lev + 1), Ghc = (f.Hs + 2 * c.n - 1) >> (lev + 1);
  const int cid = (blockIdx.x * blockDim.x + threadIdx.x) / kSLanes;
  const int lane = threadIdx.x % kSLanes;
  if (cid >= Gwc * Ghc) return;
  const int gx = 2 * (cid % Gwc), gy = 2 * (cid / Gwc);
  const int32_t fl = sgrid_flow(f, lev + 1)[cid];
  int32_t e = kInf;
  if (fl != kEmpty) e = row16_sum(sift_partial<SG>(c, gx * c.n, gy * c.n, fl, lane, kSLanes));
  if (lane < 4) {
    const int x = gx + (lane & 1), y = gy + (lane >> 1);
    if (x < Gw && y < Gh) {
      sgrid_flow(f, lev)[(size_t)y * Gw + x] = lane == 0 ? fl : kEmpty;
      sgrid_cost(f, lev, Gw * Gh)[(size_t)y * Gw + x] = lane == 0 ? e : kInf;
    }
  }
}

// ---------------------------------------------------------------- random search
// One offset per point, per axis an integer in [-nRQ, nRQ] 1/Q px from
// Philox keyed by the seed with counter (pixel, level, step, field | pair
// << 2); replace only on a strictly lower cost.  16 lanes per point.
template <int SG>
__global__ __launch_bounds__(256) void k_sift_rs(const SiftRec* __restrict__ table, int lev, int qshift, int step,
                                                 int R) {
  const SiftRec& f = table[blockIdx.y];
  const SCtx c = sctx_of(f, lev, qshift);
  const int Gw = (f.Ws + c.n - 1) >> lev, Gh = (f.Hs + c.n - 1) >> lev;
  const int pid = (blockIdx.x * blockDim.x + threadIdx.x) / kSLanes;
  const int lane = threadIdx.x % kSLanes;
  if (pid >= Gw * Gh) return;
  int32_t* F = sgrid_flow(f, lev);
  int32_t* C = sgrid_cost(f, lev, Gw * Gh);
  const int32_t fl = F[pid];
  if (fl == kEmpty) return;
  const int px = (pid % Gw) * c.n, py = (pid / Gw) * c.n;
  uint32_t u0, u1;
  philox2((uint32_t)(py * f.Ws + px), (uint32_t)lev, (uint32_t)step, f.c3, f.k0, f.k1, u0, u1);
  const int rad = c.n * R * c.Q;
  const uint64_t span = (uint64_t)(2 * rad + 1);
  const int32_t cand = packf(fx_of(fl) + (int)((u0 * span) >> 32) - rad, fy_of(fl) + (int)((u1 * span) >> 32) - rad);
  if (!svalid(c, px, py, cand)) return;
  const int32_t e = row16_sum(sift_partial<SG>(c, px, py, cand, lane, kSLanes));
  if (lane == 0 && e < C[pid]) {
    F[pid] = cand;
    C[pid] = e;
  }
}

// ---------------------------------------------------------------- propagation (Eq. 2)
// Sweep (sx, sy): 1: (+,+), 2: (-,-), 3: (-,+), 4: (+,-); predecessors at
// -sx (horizontal) and -sy (vertical).  Candidate order of Eq. 2: current,
// vertical, horizontal, replaced only on a strictly lower cost; a candidate
// equal to the current flow is not evaluated (it cannot win).
__device__ __forceinline__ uint64_t rt_now() { return __builtin_amdgcn_s_memrealtime(); }

// One signed sliding-window term of a propagated candidate: lane k of
// 4 (2r+1) covers group k / (2r+1) -- 0 / 1: the row leaving / entering the
// patch of the vertical candidate, 2 / 3: the column leaving / entering for
// the horizontal one -- at free offset k mod (2r+1) - r.  In the sweep
// direction (sx, sy) the entering row is at sy r and the leaving one at
// -sy (r + 1) (columns likewise with sx): E(p, F(q)) = C(q) - leaving +
// entering, exact because every lookup clamps per coordinate.
template <int SG>
__device__ __forceinline__ void slide_terms(const SCtx& c, int px, int py, int sx, int sy, bool useV, const Tgt& tv,
                                            bool useH, const Tgt& th, int lane, int32_t& sV, int32_t& sH) {
  const int Sd = 2 * c.r + 1, sgf = (c.S + 3) >> 2;
  sV = 0;
  sH = 0;
  for (int k = lane; k < 4 * Sd; k += 64) {
    const int grp = k / Sd, o = k - grp * Sd - c.r;
    const bool vert = grp < 2, enter = (grp & 1) != 0;
    const int across = vert ? sy : sx;
    const int a = enter ? across * c.r : -across * (c.r + 1);
    const int dx = (vert ? o : a) * c.n, dy = (vert ? a : o) * c.n;
    const Tgt& t = vert ? tv : th;
    const int sxp = clampi(px + dx, 0, c.Ws - 1), syp = clampi(py + dy, 0, c.Hs - 1);
    const Px<SG> pa = load_px<SG>(c.src + pix_off(sxp, syp, c.Ws, c.P), sgf);
    const Quad<SG> q = load_quad<SG>(c, clampi(t.Mx + dx, 0, c.Wd - 1), clampi(t.My + dy, 0, c.Hd - 1), sgf);
    const int32_t d = dist_of<SG>(c, pa, q, t);
    const int32_t sd = enter ? d : -d;
    if (vert)
      sV += useV ? sd : 0;
    else
      sH += useH ? sd : 0;
  }
}

// Handoff words between bands: (cost << 32) | flow, all ones while not yet
// written (no cost is 0xFFFFFFFF).  Launch L of a call reads and writes
// buffer L & 1 and clears buffer (L + 1) & 1 for the next launch.
constexpr uint64_t kXchEmpty = ~0ull;

template <int SG>
__global__ __launch_bounds__(kSBand * 64) void k_sift_prop(const SiftRec* __restrict__ table, int nf, int lev,
                                                           int qshift, int sx, int sy, int parity,
                                                           int32_t* __restrict__ ticket,
                                                           int32_t* __restrict__ status, uint64_t timeout) {
  __shared__ int32_t s_field, s_band, s_nb;
  __shared__ int32_t resF[2][kSBand], resC[2][kSBand];
  if (threadIdx.x == 0) {
    int tk = atomicAdd(ticket, 1), fi = 0, nb = 0;
    for (; fi < nf; ++fi) {
      const int gh = (table[fi].Hs + (1 << lev) - 1) >> lev;
      nb = (gh + kSBand - 1) / kSBand;
      if (tk < nb) break;
      tk -= nb;
    }
    s_field = fi;
    s_band = tk;
    s_nb = nb;
  }
  __syncthreads();
  if (s_field >= nf) return;
  const SiftRec& f = table[s_field];
  const SCtx c = sctx_of(f, lev, qshift);
  const int n = c.n;
  const int Gw = (f.Ws + n - 1) >> lev, Gh = (f.Hs + n - 1) >> lev;
  const int band = s_band, v0 = band * kSBand;
  const size_t xwords = (size_t)((f.Hs + kSBand - 1) / kSBand) * f.Ws;   // one buffer
  uint64_t* const xbase = reinterpret_cast<uint64_t*>(f.ws + f.o_xch);
  {
    // this band's share of the next launch's buffer
    uint64_t* nxt = xbase + (size_t)(parity ^ 1) * xwords;
    const size_t per = (xwords + s_nb - 1) / s_nb;
    const size_t e0 = (size_t)band * per, e1 = min(xwords, e0 + per);
    for (size_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) nxt[i] = kXchEmpty;
  }
  if (v0 >= Gh) return;
  const int rows = min(kSBand, Gh - v0);
  const int row = threadIdx.x >> 6, lane = threadIdx.x & 63;   // one wavefront per band row
  const bool rowok = row < rows;
  const int gy = sy > 0 ? v0 + row : Gh - 1 - (v0 + row);
  const int py = gy * n;
  int32_t* const F = sgrid_flow(f, lev);
  int32_t* const C = sgrid_cost(f, lev, Gw * Gh);
  uint64_t* const xch = xbase + (size_t)parity * xwords;
  const uint64_t* const xin = xch + (size_t)(band > 0 ? band - 1 : 0) * Gw;
  uint64_t* const xout = xch + (size_t)band * Gw;
  const bool publish = rowok && row == rows - 1 && v0 + rows < Gh;
  const int nsteps = Gw + rows - 1;
  // this row's result of the previous step: its horizontal candidate
  int32_t hF = kEmpty, hC = kInf;
  bool abandoned = false;
  // prefetched for the row's next column: its own flow and cost and, for row
  // 0, the band above's word (each loaded one step ahead, before the barrier)
  auto own_idx = [&](int uu) { return (size_t)gy * Gw + (sx > 0 ? uu : Gw - 1 - uu); };
  int32_t nF = kEmpty, nC = kInf;
  uint64_t nW = kXchEmpty;
  if (row == 0) {
    nF = F[own_idx(0)];
    nC = C[own_idx(0)];
    if (band > 0) nW = __hip_atomic_load(&xin[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int t = 0; t < nsteps; ++t) {
    const int u = t - row;
    const bool active = rowok && u >= 0 && u < Gw;
    if (rowok && u == 0 && row > 0) {
      nF = F[own_idx(0)];
      nC = C[own_idx(0)];
    }
    const int32_t curF0 = nF, curC0 = nC;
    int32_t vF = kEmpty, vC = kInf;
    if (row == 0) {
      if (band > 0 && active) {
        uint64_t w = nW;
        if (w == kXchEmpty && !abandoned) {
          const uint64_t t0 = rt_now();
          do {
            __builtin_amdgcn_s_sleep(1);
            w = __hip_atomic_load(&xin[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (rt_now() - t0 > timeout) {
              __hip_atomic_store(status, (int32_t)FF_ERR_DEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              abandoned = true;
              break;
            }
          } while (w == kXchEmpty);
        }
        if (w != kXchEmpty) {
          vF = (int32_t)(uint32_t)w;
          vC = (int32_t)(uint32_t)(w >> 32);
        }
      }
    } else {
      vF = resF[(t - 1) & 1][row - 1];
      vC = resC[(t - 1) & 1][row - 1];
    }
    int32_t outF = kEmpty, outC = kInf;
    if (active) {
      const size_t pi = own_idx(u);
      const int px = (sx > 0 ? u : Gw - 1 - u) * n;
      const bool useV = vF != curF0 && svalid(c, px, py, vF);
      const bool useH = u > 0 && hF != curF0 && svalid(c, px, py, hF);
      int32_t curF = curF0, curC = curC0;
      if (useV || useH) {
        const Tgt tv = tgt_of(c, px, py, useV ? vF : 0), th = tgt_of(c, px, py, useH ? hF : 0);
        int32_t dV, dH;
        slide_terms<SG>(c, px, py, sx, sy, useV, tv, useH, th, lane, dV, dH);
        const int32_t eV = vC + wave_sum(dV), eH = hC + wave_sum(dH);
        if (useV && eV < curC) {
          curF = vF;
          curC = eV;
        }
        if (useH && eH < curC) {
          curF = hF;
          curC = eH;
        }
      }
      if (lane == 0 && curF != curF0) {
        F[pi] = curF;
        C[pi] = curC;
      }
      outF = curF;
      outC = curC;
      if (publish && lane == 0)
        __hip_atomic_store(&xout[u], ((uint64_t)(uint32_t)outC << 32) | (uint32_t)outF, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      hF = outF;
      hC = outC;
      if (u + 1 < Gw) {
        nF = F[own_idx(u + 1)];
        nC = C[own_idx(u + 1)];
        if (row == 0 && band > 0) nW = __hip_atomic_load(&xin[u + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (lane == 0) {
      resF[t & 1][row] = outF;
      resC[t & 1][row] = outC;
    }
    // only the LDS results cross rows; each row's global stores touch its
    // own points and the next column's prefetches stay in flight
    lds_barrier();
  }
}

// write the grid of level lev into the full-resolution outputs (inspection
// stops); grid: (W / 256, H, fields)
__global__ void k_sift_write_grid(const SiftRec* __restrict__ table, int lev) {
  const SiftRec& f = table[blockIdx.z];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= f.Ws || y >= f.Hs) return;
  const int n = 1 << lev;
  const int Gw = (f.Ws + n - 1) >> lev, Gh = (f.Hs + n - 1) >> lev;
  const size_t o = (size_t)y * f.Ws + x;
  if ((x % n) == 0 && (y % n) == 0) {
    f.flow[o] = sgrid_flow(f, lev)[(size_t)(y / n) * Gw + x / n];
    f.cost[o] = sgrid_cost(f, lev, Gw * Gh)[(size_t)(y / n) * Gw + x / n];
  } else {
    f.flow[o] = kEmpty;
    f.cost[o] = kInf;
  }
}

// ---------------------------------------------------------------- host
struct SiftFieldPlan {
  TreeLayout tree;
  size_t off_grid[5];
  size_t off_xch;
  size_t bytes;
};

static SiftFieldPlan sift_field_plan(const ff_sift_job& j, const ff_match_params* p) {
  SiftFieldPlan P{};
  const int Ws = j.src->width, Hs = j.src->height;
  P.tree = tree_layout(j.dst->width * j.dst->height, p->leaf, 0);
  size_t off = P.tree.bytes;
  for (int lev = 1; lev <= p->k; ++lev) {
    const int n = 1 << lev;
    const size_t G = (size_t)((Ws + n - 1) / n) * ((Hs + n - 1) / n);
    off = align_up(off, 256);
    P.off_grid[lev] = off;
    off += G * 8;
  }
  off = align_up(off, 256);
  P.off_xch = off;
  off += 2 * (size_t)((Hs + kSBand - 1) / kSBand) * Ws * 8;
  P.bytes = align_up(off, 256);
  return P;
}

struct SiftBatchLayout {
  size_t off_tickets, off_table, off_ttable;
  int launches;
  std::vector<size_t> off_field;
  size_t bytes;
};

static SiftBatchLayout sift_batch_layout(const ff_sift_job* jobs, int n, const ff_match_params* p) {
  SiftBatchLayout B;
  size_t off = kSiftStatusBytes;
  B.off_tickets = off;
  B.launches = (p->k + 1) * p->n_prop;
  off = align_up(off + (size_t)B.launches * 4, 256);
  B.off_table = off;
  off = align_up(off + (size_t)n * sizeof(SiftRec), 256);
  B.off_ttable = off;
  off = align_up(off + (size_t)n * sizeof(FieldRec), 256);
  B.off_field.resize(n);
  for (int i = 0; i < n; ++i) {
    B.off_field[i] = off;
    off = align_up(off + sift_field_plan(jobs[i], p).bytes, 256);
  }
  B.bytes = off;
  return B;
}

static ff_status check_sift_job(const ff_sift_job& j, const ff_match_params* p) {
  if (!j.src || !j.dst || !j.src_blob || !j.dst_blob || !j.src_levels || !j.dst_levels || !j.flow || !j.cost)
    return FF_ERR_ARG;
  const ff_desc* s = j.src;
  const ff_desc* d = j.dst;
  if (s->subpel != d->subpel) return FF_ERR_ARG;
  if (j.radius < 1 || j.radius > kMaxRadius) return FF_ERR_ARG;
  if (j.pitch < 4 || j.pitch > 32 || (j.pitch & 3) || j.channels < 1 || j.channels > j.pitch) return FF_ERR_ARG;
  if (p->k < 0 || p->k > j.levels || j.levels > 4) return FF_ERR_ARG;
  if (j.field_id > 3) return FF_ERR_ARG;
  if (!wht_block(s, j.src_blob, j.radius) || !wht_block(d, j.dst_blob, j.radius)) return FF_ERR_ARG;
  return FF_OK;
}

static ff_status check_sift_params(const ff_match_params* p) {
  if (!p) return FF_ERR_ARG;
  if (p->k < 0 || p->k > 4) return FF_ERR_ARG;
  if (p->R < 0 || p->R > 64 || p->n_prop < 0 || p->n_prop > 64 || p->n_rs < 0 || p->n_rs > p->n_prop) return FF_ERR_ARG;
  if (p->use_kdtree != 1) return FF_ERR_UNSUPPORTED;   // seeds come from the kd-tree only
  if (p->leaf < 2 || p->leaf > kMaxLeaf) return FF_ERR_ARG;
  if (p->watchdog_us < 0) return FF_ERR_ARG;
  return FF_OK;
}

static SiftRec make_sift_rec(const ff_sift_job& j, const SiftFieldPlan& P, char* fws) {
  SiftRec r{};
  r.src = j.src_levels;
  r.dst = j.dst_levels;
  r.Vsrc = wht_block(j.src, j.src_blob, j.radius);
  r.flow = j.flow;
  r.cost = j.cost;
  r.ws = fws;
  r.Ws = j.src->width;
  r.Hs = j.src->height;
  r.Wd = j.dst->width;
  r.Hd = j.dst->height;
  r.P = j.pitch;
  r.S = j.channels;
  r.r = j.radius;
  r.vstride = j.src->wht_stride;
  r.k0 = (uint32_t)(j.seed & 0xFFFFFFFFu);
  r.k1 = (uint32_t)(j.seed >> 32);
  r.c3 = j.field_id | (j.pair_id << 2);
  r.t_nodes = (uint32_t)P.tree.nodes;
  r.o_dim = (uint32_t)P.tree.off_dim;
  r.o_split = (uint32_t)P.tree.off_split;
  r.o_perm = (uint32_t)P.tree.off_perm;
  r.o_xch = (uint32_t)P.off_xch;
  for (int l = 0; l < 5; ++l) r.o_grid[l] = (uint32_t)P.off_grid[l];
  return r;
}

// the record the kd-tree build reads: the target's WHT vectors and the tree
// offsets in the field region
static FieldRec make_tree_rec(const ff_sift_job& j, const SiftFieldPlan& P, char* fws) {
  FieldRec r{};
  r.Vdst = wht_block(j.dst, j.dst_blob, j.radius);
  r.Ws = j.src->width;
  r.Hs = j.src->height;
  r.Wd = j.dst->width;
  r.Hd = j.dst->height;
  r.r = j.radius;
  r.D = j.dst->wht_dims;
  r.vstride = j.dst->wht_stride;
  r.ws = fws;
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
  return r;
}

template <int SG>
static ff_status run_sift_batch(const ff_sift_job* jobs, int n, const ff_match_params* p, char* ws,
                                const SiftBatchLayout& B, hipStream_t stream) {
  int32_t* status = reinterpret_cast<int32_t*>(ws);
  int32_t* tickets = reinterpret_cast<int32_t*>(ws + B.off_tickets);
  SiftRec* table = reinterpret_cast<SiftRec*>(ws + B.off_table);
  FieldRec* ttable = reinterpret_cast<FieldRec*>(ws + B.off_ttable);
  std::vector<SiftRec> recs(n);
  std::vector<FieldRec> trecs(n);
  int maxW = 0, maxH = 0, maxN = 0, maxTop = 0;
  for (int i = 0; i < n; ++i) {
    const SiftFieldPlan P = sift_field_plan(jobs[i], p);
    recs[i] = make_sift_rec(jobs[i], P, ws + B.off_field[i]);
    trecs[i] = make_tree_rec(jobs[i], P, ws + B.off_field[i]);
    maxW = std::max(maxW, recs[i].Ws);
    maxH = std::max(maxH, recs[i].Hs);
    maxN = std::max(maxN, recs[i].Wd * recs[i].Hd);
    maxTop = std::max(maxTop, trecs[i].t_top);
  }
  const int qshift = ilog2i(jobs[0].src->subpel);
  const int k = p->k;
  fill_i32(status, 1, 0, stream);
  fill_i32(tickets, (size_t)B.launches, 0, stream);
  for (int i = 0; i < n; i += kSiftRecsPerWrite) {
    SiftChunk sc{};
    TreeChunk tc{};
    const int m = std::min(kSiftRecsPerWrite, n - i);
    for (int q = 0; q < m; ++q) {
      sc.r[q] = recs[i + q];
      tc.r[q] = trecs[i + q];
    }
    k_sift_write_table<<<1, kSiftRecsPerWrite, 0, stream>>>(sc, m, table + i);
    k_tree_write_table<<<1, kSiftRecsPerWrite, 0, stream>>>(tc, m, ttable + i);
  }
  k_sift_clear_xch<<<dim3(64, n), 256, 0, stream>>>(table);
  prof_mark(FF_PROF_TREE, stream, true);
  ff_status st = enqueue_tree_build(ttable, n, maxN, maxTop, p->leaf, stream);
  prof_mark(FF_PROF_TREE, stream, false);
  if (st != FF_OK) return st;
  auto pts = [&](int lev) { return ((maxW + (1 << lev) - 1) >> lev) * ((maxH + (1 << lev) - 1) >> lev); };
  auto groups = [&](int npts) { return (unsigned)(((size_t)npts * kSLanes + 255) / 256); };
  int steps = 0, cur_lev = k;
  auto stop = [&]() { return p->max_steps >= 0 && steps >= p->max_steps; };
  auto finish = [&]() -> ff_status {
    if (cur_lev > 0) k_sift_write_grid<<<dim3((maxW + 255) / 256, maxH, n), 256, 0, stream>>>(table, cur_lev);
    return launch_status();
  };
  k_sift_seed<SG><<<dim3((pts(k) + 3) / 4, n), 256, 0, stream>>>(table, k, qshift);
  ++steps;
  if (stop()) return finish();
  const uint64_t timeout = p->watchdog_us > 0 ? (uint64_t)p->watchdog_us * 100u : 200000000ull;
  auto sx_of = [](int i) { return ((i & 3) == 0 || (i & 3) == 3) ? 1 : -1; };
  auto sy_of = [](int i) { return ((i & 3) == 0 || (i & 3) == 2) ? 1 : -1; };
  int launch = 0;
  for (int lev = k; lev >= 0; --lev) {
    cur_lev = lev;
    if (lev < k) {
      k_sift_entry<SG><<<dim3(groups(pts(lev + 1)), n), 256, 0, stream>>>(table, lev, qshift);
      ++steps;
      if (stop()) return finish();
    }
    for (int i = 0; i < p->n_prop; ++i) {
      int bands = 0;
      for (int g = 0; g < n; ++g) bands += (((recs[g].Hs + (1 << lev) - 1) >> lev) + kSBand - 1) / kSBand;
      prof_mark(FF_PROF_SIFT_PROPAGATE, stream, true);
      k_sift_prop<SG><<<bands, kSBand * 64, 0, stream>>>(table, n, lev, qshift, sx_of(i), sy_of(i), launch & 1,
                                                         tickets + launch, status, timeout);
      prof_mark(FF_PROF_SIFT_PROPAGATE, stream, false);
      ++launch;
      ++steps;
      if (stop()) return finish();
      if (i < p->n_rs) {
        k_sift_rs<SG><<<dim3(groups(pts(lev)), n), 256, 0, stream>>>(table, lev, qshift, i, p->R);
        ++steps;
        if (stop()) return finish();
      }
    }
  }
  cur_lev = 0;
  return finish();
}

}  // namespace ff

using namespace ff;

extern "C" {

size_t ff_match_sift_workspace_bytes(const ff_sift_job* jobs, int32_t n_jobs, const ff_match_params* p) {
  if (!jobs || n_jobs < 1 || check_sift_params(p) != FF_OK) return 0;
  for (int i = 0; i < n_jobs; ++i)
    if (check_sift_job(jobs[i], p) != FF_OK) return 0;
  return sift_batch_layout(jobs, n_jobs, p).bytes;
}

ff_status ff_match_sift(const ff_sift_job* jobs, int32_t n_jobs, const ff_match_params* p, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
  if (!jobs || n_jobs < 1 || !workspace) return FF_ERR_ARG;
  ff_status st = check_sift_params(p);
  if (st != FF_OK) return st;
  for (int i = 0; i < n_jobs; ++i) {
    st = check_sift_job(jobs[i], p);
    if (st != FF_OK) return st;
    if (jobs[i].src->subpel != jobs[0].src->subpel) return FF_ERR_ARG;
  }
  const SiftBatchLayout B = sift_batch_layout(jobs, n_jobs, p);
  if (workspace_bytes < B.bytes) return FF_ERR_WORKSPACE;
  st = ensure_init();
  if (st != FF_OK) return st;
  prof_mark(FF_PROF_SIFT_MATCH, stream, true);
  int sg = 1;
  for (int i = 0; i < n_jobs; ++i) sg = std::max(sg, (jobs[i].channels + 3) / 4);
  char* w = static_cast<char*>(workspace);
  switch (sg) {
    case 1: st = run_sift_batch<1>(jobs, n_jobs, p, w, B, stream); break;
    case 2: st = run_sift_batch<2>(jobs, n_jobs, p, w, B, stream); break;
    case 3: st = run_sift_batch<3>(jobs, n_jobs, p, w, B, stream); break;
    case 4: st = run_sift_batch<4>(jobs, n_jobs, p, w, B, stream); break;
    case 5: st = run_sift_batch<5>(jobs, n_jobs, p, w, B, stream); break;
    case 6: st = run_sift_batch<6>(jobs, n_jobs, p, w, B, stream); break;
    case 7: st = run_sift_batch<7>(jobs, n_jobs, p, w, B, stream); break;
    default: st = run_sift_batch<8>(jobs, n_jobs, p, w, B, stream); break;
  }
  prof_mark(FF_PROF_SIFT_MATCH, stream, false);
  return st;
}

}  // extern "C"
