// ORACLE -- test infrastructure, not product code.
//
// A plain, slow, single-threaded CPU implementation of the Flow Fields hot
// path (Bailer, Taetz, Stricker: "Flow Fields: Dense Correspondence Fields
// for Highly Accurate Large Displacement Optical Flow Estimation", ICCV 2015).
// It exists to check the GPU library against.  Only the test-suite, the smoke
// check and the CPU-baseline leg of the benchmark load it; the GPU path never
// includes, links or calls anything in this directory, and this file shares
// no code, header, table or constant generator with it.
//
// Everything here is integer arithmetic except the one-time generation of
// three small tables (sRGB gamma, Lab f(t), Lanczos weights) in double and
// the dense SIFT vectors of the second data term (double; the PCA that turns
// them into integer colour codes is in oracle/ffo.py, NumPy float64).
// Patch costs are direct sums over the whole patch -- no sliding windows, no
// blocking, no reordering.  Propagation runs in plain raster order in the
// sweep direction.  Where the paper is silent, this file takes one reading
// and states it beside the code (the same readings are listed in the design
// notes of the repository).
//
// Parity status: every function below is pinned by tests under tests/ that
// do not call back into this file for the expected value (closed forms,
// invariants, brute force, independent NumPy formulations).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

constexpr int32_t kInf = INT32_MAX;                  // cost of "no flow"
constexpr int32_t kEmpty = (int32_t)0x80008000u;      // packed (dx,dy) = (-32768,-32768)

inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
inline int64_t floordiv(int64_t a, int64_t b) {      // b > 0
  int64_t q = a / b;
  if ((a % b) != 0 && (a < 0)) --q;
  return q;
}
inline int32_t pack(int dx, int dy) { return (int32_t)(((uint32_t)(uint16_t)(int16_t)dy << 16) | (uint16_t)(int16_t)dx); }
inline int unpack_x(int32_t f) { return (int16_t)(uint16_t)((uint32_t)f & 0xFFFF); }
inline int unpack_y(int32_t f) { return (int16_t)(uint16_t)((uint32_t)f >> 16); }
inline int popc(uint32_t v) { return __builtin_popcount(v); }

// ---------------------------------------------------------------------------
// Section 3.3 (data terms): census transform over the CIELab channels.
// CIELab conversion quantised to 8 bits per channel.
//
// Reading: sRGB (IEC 61966-2-1) transfer curve, sRGB->XYZ matrix with each
// row normalised by its sum (so white maps to (1,1,1) and grays keep
// a = b = 0 exactly), the CIE f(t) with the linear toe below (6/29)^3.
// L8 = round(2.55 L), a8 = round(a) + 128, b8 = round(b) + 128, rounding half
// up, clamped to [0,255].  Tables: gamma Q16, matrix Q14 (rows sum to 2^14
// exactly), f(t) Q15 over t in Q16.
struct LabTables {
  int32_t gamma[256];
  int32_t mat[9];
  std::vector<int32_t> f;  // 65537 entries
};

const LabTables& lab_tables() {
  static LabTables T = [] {
    LabTables t;
    for (int c = 0; c < 256; ++c) {
      double v = c / 255.0;
      double lin = (v <= 0.04045) ? v / 12.92 : std::pow((v + 0.055) / 1.055, 2.4);
      t.gamma[c] = (int32_t)std::floor(lin * 65536.0 + 0.5);
    }
    const double m[3][3] = {{0.4124564, 0.3575761, 0.1804375},
                            {0.2126729, 0.7151522, 0.0721750},
                            {0.0193339, 0.1191920, 0.9503041}};
    for (int i = 0; i < 3; ++i) {
      double s = m[i][0] + m[i][1] + m[i][2];
      int32_t q[3];
      int big = 0;
      for (int j = 0; j < 3; ++j) {
        q[j] = (int32_t)std::floor(16384.0 * m[i][j] / s + 0.5);
        if (m[i][j] > m[i][big]) big = j;
      }
      q[big] += 16384 - (q[0] + q[1] + q[2]);
      for (int j = 0; j < 3; ++j) t.mat[i * 3 + j] = q[j];
    }
    t.f.resize(65537);
    const double toe = 216.0 / 24389.0;  // (6/29)^3
    for (int i = 0; i <= 65536; ++i) {
      double x = i / 65536.0;
      double fx = (x > toe) ? std::cbrt(x) : x * (841.0 / 108.0) + 4.0 / 29.0;
      t.f[i] = (int32_t)std::floor(fx * 32768.0 + 0.5);
    }
    return t;
  }();
  return T;
}

void lab8_pixel(uint8_t R, uint8_t G, uint8_t B, uint8_t out[3]) {
  const LabTables& T = lab_tables();
  int64_t lin[3] = {T.gamma[R], T.gamma[G], T.gamma[B]};
  int32_t fq[3];
  for (int i = 0; i < 3; ++i) {
    int64_t acc = T.mat[i * 3 + 0] * lin[0] + T.mat[i * 3 + 1] * lin[1] + T.mat[i * 3 + 2] * lin[2];
    int64_t xyz = floordiv(acc + 8192, 16384);  // Q16, in [0, 65536]
    fq[i] = T.f[xyz];
  }
  int64_t L = floordiv(2958LL * fq[1] - 408LL * 32768 + 163840, 327680);
  int64_t a = floordiv(500LL * (fq[0] - fq[1]) + 16384, 32768) + 128;
  int64_t b = floordiv(200LL * (fq[1] - fq[2]) + 16384, 32768) + 128;
  out[0] = (uint8_t)clampi((int)L, 0, 255);
  out[1] = (uint8_t)clampi((int)a, 0, 255);
  out[2] = (uint8_t)clampi((int)b, 0, 255);
}

// ---------------------------------------------------------------------------
// Section 3.2 (smoothed images I^n): area-based downsampling by n, then
// Lanczos upsampling back to full resolution.
//
// Reading: Lanczos-3 kernel L(t) = sinc(t) sinc(t/3); pixel-centre alignment
// u = (x + 1/2)/n - 1/2; replicate borders on both grids; the image is
// replicate-padded to a multiple of n before the n x n block sums.  Weights
// are Q14 per phase (x mod n) for taps k = -3..3 around floor(x/n), rounded
// half up, the residual to 2^14 added to the centre tap.  The horizontal pass
// rounds back to block-sum units, the vertical pass divides by 2^14 * n^2 and
// keeps 4 fractional bits (output Q4: a constant image c maps to 16 c).
struct LanczosTable {
  int32_t w[16][7];  // [phase][k+3], n <= 16
};

LanczosTable lanczos_table(int n) {
  LanczosTable t{};
  const double pi = 3.14159265358979323846;
  for (int ph = 0; ph < n; ++ph) {
    double t0 = (ph + 0.5) / n - 0.5;
    int32_t sum = 0;
    for (int k = -3; k <= 3; ++k) {
      double x = t0 - k;
      double L;
      if (x == 0.0) L = 1.0;
      else if (std::fabs(x) < 3.0) L = 3.0 * std::sin(pi * x) * std::sin(pi * x / 3.0) / (pi * pi * x * x);
      else L = 0.0;
      t.w[ph][k + 3] = (int32_t)std::floor(16384.0 * L + 0.5);
      sum += t.w[ph][k + 3];
    }
    t.w[ph][3] += 16384 - sum;
  }
  return t;
}

int ilog2(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

// plane: H x W samples, out: H x W int16 with `frac` fractional bits (the
// census path: uint8 in, Q4 out; the SIFT colours of section 3.3: int16 codes
// in, the same units out)
template <class Px>
void smooth_plane_t(const Px* J, int W, int H, int n, int frac, int16_t* out) {
  if (n == 1) {
    for (int i = 0; i < W * H; ++i) out[i] = (int16_t)(J[i] * (1 << frac));
    return;
  }
  const int Wc = (W + n - 1) / n, Hc = (H + n - 1) / n;
  std::vector<int64_t> A((size_t)Wc * Hc, 0);
  for (int i = 0; i < Hc; ++i)
    for (int j = 0; j < Wc; ++j) {
      int64_t s = 0;
      for (int u = 0; u < n; ++u)
        for (int v = 0; v < n; ++v) s += J[(size_t)std::min(i * n + u, H - 1) * W + std::min(j * n + v, W - 1)];
      A[(size_t)i * Wc + j] = s;
    }
  LanczosTable lt = lanczos_table(n);
  std::vector<int64_t> T((size_t)Hc * W);
  for (int i = 0; i < Hc; ++i)
    for (int x = 0; x < W; ++x) {
      int64_t s = 0;
      for (int k = -3; k <= 3; ++k) s += (int64_t)lt.w[x % n][k + 3] * A[(size_t)i * Wc + clampi(x / n + k, 0, Wc - 1)];
      T[(size_t)i * W + x] = floordiv(s + 8192, 16384);
    }
  const int sh = 14 + 2 * ilog2(n) - frac;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t s = 0;
      for (int k = -3; k <= 3; ++k) s += (int64_t)lt.w[y % n][k + 3] * T[(size_t)clampi(y / n + k, 0, Hc - 1) * W + x];
      out[(size_t)y * W + x] = (int16_t)floordiv(s + (1LL << (sh - 1)), 1LL << sh);
    }
}

void smooth_plane(const uint8_t* J, int W, int H, int n, int16_t* out) { smooth_plane_t(J, W, H, n, 4, out); }

// ---------------------------------------------------------------------------
// Section 3.3 census data term on the subsampled patches of section 3.2, with
// the subpixel positions of the random search (section 3.1) resolved by
// bilinear interpolation.
//
// Reading: one census plane per level n and subpixel phase (a,b), a,b in
// [0,Q).  The smoothed plane is shifted by (a/Q, b/Q) with exact integer
// bilinear weights (no rounding); the census bit t of channel c compares the
// neighbour at stride n in direction delta_t (8 neighbours in raster order,
// bit 0 = (-1,-1)) with the centre: bit = [neighbour < centre].  All lookups
// clamp to the image.  Channel c occupies byte c of the 32-bit word.
const int kDX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
const int kDY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};

void census_plane(const int16_t* S /* C planes */, int W, int H, int C, int n, int Q, int a, int b,
                  uint32_t* out) {
  const size_t N = (size_t)W * H;
  std::vector<int32_t> Bv(N);
  std::fill(out, out + N, 0u);
  for (int c = 0; c < C; ++c) {
    const int16_t* P = S + c * N;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        int x1 = std::min(x + 1, W - 1), y1 = std::min(y + 1, H - 1);
        Bv[(size_t)y * W + x] = (Q - a) * (Q - b) * P[(size_t)y * W + x] + a * (Q - b) * P[(size_t)y * W + x1] +
                                (Q - a) * b * P[(size_t)y1 * W + x] + a * b * P[(size_t)y1 * W + x1];
      }
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        int32_t ctr = Bv[(size_t)y * W + x];
        uint32_t bits = 0;
        for (int t = 0; t < 8; ++t) {
          int xx = clampi(x + n * kDX[t], 0, W - 1), yy = clampi(y + n * kDY[t], 0, H - 1);
          if (Bv[(size_t)yy * W + xx] < ctr) bits |= 1u << t;
        }
        out[(size_t)y * W + x] |= bits << (8 * c);
      }
  }
}

// ---------------------------------------------------------------------------
// Section 3.1: Walsh-Hadamard projections of the unsmoothed patch P_rho, the
// first 9 bases per CIELab channel (footnote: the odd extent 2 rho + 1 is
// split into rho and rho + 1).
//
// Reading: 1-D Walsh functions in sequency order on [-rho, rho]: w0 = +1;
// w1 = + on [-rho,-1], - on [0,rho]; w2 splits each half again, smaller part
// first, signs + - - +.  2-D basis j = (u,v) with u acting on dy and v on dx,
// order (0,0),(0,1),(1,0),(1,1),(0,2),(2,0),(1,2),(2,1),(2,2); feature index
// c*9 + j; border pixels clamped.
int walsh(int s, int t, int rho) {
  if (s == 0) return 1;
  if (s == 1) return t < 0 ? 1 : -1;
  if (t < 0) return (t < -rho + rho / 2) ? 1 : -1;
  return (t < (rho + 1) / 2) ? -1 : 1;
}
const int kBU[9] = {0, 0, 1, 1, 0, 2, 1, 2, 2};
const int kBV[9] = {0, 1, 0, 1, 2, 0, 2, 1, 2};

void wht(const uint8_t* J /* C planes */, int W, int H, int C, int rho, int32_t* out /* N x 9C */) {
  const size_t N = (size_t)W * H;
  const int D = 9 * C;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      for (int c = 0; c < C; ++c)
        for (int j = 0; j < 9; ++j) {
          int64_t s = 0;
          for (int dy = -rho; dy <= rho; ++dy)
            for (int dx = -rho; dx <= rho; ++dx)
              s += walsh(kBU[j], dy, rho) * walsh(kBV[j], dx, rho) *
                   (int)J[c * N + (size_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
          out[((size_t)y * W + x) * D + c * 9 + j] = (int32_t)s;
        }
}

// ---------------------------------------------------------------------------
// Section 3.1: kd-tree over the WHT vectors of every target pixel, leaf size
// l, split on the dimension of maximal spread at the median.
//
// Reading: split while a node holds more than l points; spread = max - min,
// ties to the lowest dimension; order the node's points by (key, pixel
// index); the left child takes the first floor(cnt/2), the split value is the
// key of the first point of the right child; a query goes right iff its key
// is >= the split value.  Nodes live in heap order (children 2i+1, 2i+2);
// node_dim = -1 marks a leaf; a leaf's points are stored in ascending pixel
// index in the permutation array, leaves in left-to-right order.
struct Tree {
  int N = 0, D = 0, leaf = 0;
  std::vector<int32_t> dim, split, perm;
};

int tree_depth(int N, int leaf) {
  int d = 0;
  while (((int64_t)N + (1LL << d) - 1) / (1LL << d) > leaf) ++d;
  return d;
}

void build_node(Tree& T, const int32_t* V, int node, int start, int cnt) {
  int32_t* ids = T.perm.data() + start;
  if (cnt <= T.leaf) {
    std::sort(ids, ids + cnt);
    return;
  }
  int best = 0;
  int64_t bestSpread = -1;
  for (int j = 0; j < T.D; ++j) {
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    for (int i = 0; i < cnt; ++i) {
      int32_t k = V[(size_t)ids[i] * T.D + j];
      mn = std::min(mn, k);
      mx = std::max(mx, k);
    }
    if ((int64_t)mx - mn > bestSpread) { bestSpread = (int64_t)mx - mn; best = j; }
  }
  std::sort(ids, ids + cnt, [&](int32_t p, int32_t q) {
    int32_t kp = V[(size_t)p * T.D + best], kq = V[(size_t)q * T.D + best];
    return kp != kq ? kp < kq : p < q;
  });
  int h = cnt / 2;
  T.dim[node] = best;
  T.split[node] = V[(size_t)ids[h] * T.D + best];
  build_node(T, V, 2 * node + 1, start, h);
  build_node(T, V, 2 * node + 2, start + h, cnt - h);
}

Tree build_tree(const int32_t* V, int N, int D, int leaf) {
  Tree T;
  T.N = N; T.D = D; T.leaf = leaf;
  int depth = tree_depth(N, leaf);
  size_t nodes = ((size_t)2 << depth) - 1;
  T.dim.assign(nodes, -1);
  T.split.assign(nodes, 0);
  T.perm.resize(N);
  std::iota(T.perm.begin(), T.perm.end(), 0);
  build_node(T, V, 0, 0, N);
  return T;
}

// returns the leaf range [start, start + cnt) of the permutation array
void query_tree(const Tree& T, const int32_t* q, int& start, int& cnt) {
  int node = 0;
  start = 0;
  cnt = T.N;
  while (T.dim[node] >= 0) {
    int h = cnt / 2;
    if (q[T.dim[node]] >= T.split[node]) { node = 2 * node + 2; start += h; cnt -= h; }
    else { node = 2 * node + 1; cnt = h; }
  }
}

// ---------------------------------------------------------------------------
// Per-image descriptors: Lab8, smoothed planes, census planes per (level,
// phase), WHT vectors per radius.
struct Desc {
  int W = 0, H = 0, C = 0, k = 0, Q = 0;
  std::vector<uint8_t> lab;                        // C planes
  std::vector<std::vector<int16_t>> smooth;        // [level] C planes
  std::vector<std::vector<uint32_t>> planes;       // [level * Q*Q + b*Q + a]
  std::vector<int> radii;
  std::vector<std::vector<int32_t>> whtv;          // per radius, N x 9C
  const uint32_t* plane(int lev, int a, int b) const { return planes[(size_t)lev * Q * Q + b * Q + a].data(); }
  const int32_t* wht_for(int rho) const {
    for (size_t i = 0; i < radii.size(); ++i) if (radii[i] == rho) return whtv[i].data();
    return nullptr;
  }
};

// ---------------------------------------------------------------------------
// Eq. 1 / Eq. 4 data term E_d on the subsampled patch P^n_r (Eq. 3): the sum
// over the (2r+1)^2 samples at stride n of the census Hamming distance over
// all channels.
//
// Reading: a flow f is in 1/Q px; the target centre m = p Q + f must lie in
// [0,(W-1)Q] x [0,(H-1)Q], else the cost is "infinity" (section 3.2 sets
// uninitialised pixels to infinity).  The integer part of m is a floor
// division, the phase m mod Q selects the census plane; every sample lookup
// clamps to the image.
int32_t cost_at(const Desc& s, const Desc& d, int lev, int r, int px, int py, int fx, int fy) {
  const int Q = d.Q;
  const int n = 1 << lev;
  int64_t mx = (int64_t)px * Q + fx, my = (int64_t)py * Q + fy;
  if (mx < 0 || my < 0 || mx > (int64_t)(d.W - 1) * Q || my > (int64_t)(d.H - 1) * Q) return kInf;
  int Mx = (int)floordiv(mx, Q), My = (int)floordiv(my, Q);
  int a = (int)(mx - (int64_t)Mx * Q), b = (int)(my - (int64_t)My * Q);
  const uint32_t* P1 = s.plane(lev, 0, 0);
  const uint32_t* P2 = d.plane(lev, a, b);
  int32_t sum = 0;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      uint32_t v1 = P1[(size_t)clampi(py + n * dy, 0, s.H - 1) * s.W + clampi(px + n * dx, 0, s.W - 1)];
      uint32_t v2 = P2[(size_t)clampi(My + n * dy, 0, d.H - 1) * d.W + clampi(Mx + n * dx, 0, d.W - 1)];
      sum += popc(v1 ^ v2);
    }
  return sum;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplications
// with the published multipliers and Weyl key increments.
void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ---------------------------------------------------------------------------
// Sections 3.1 and 3.2: the hierarchical Flow Field search.
struct MatchParams {
  int k, R, leaf, n_prop, n_rs, use_kdtree, skip_dup, max_steps;
  uint32_t seed_lo, seed_hi, field_id, pair_id;
};

// The search is written once for any data term: Cost is the cost type
// (int32 census sums; double for the SIFT-flow term), inf its "infinity",
// and cost(lev, px, py, fx, fy) evaluates E^n at grid point (px, py) for
// flow (fx, fy).
template <class Cost>
struct Grid {
  int n, Gw, Gh;
  std::vector<int32_t> F;
  std::vector<Cost> C;
};

// Sweep directions (Fig. 3c is not in the text): sweep 1 goes right and
// down (Eq. 2); sweep 2 left and up; sweep 3 left and down; sweep 4 right and
// up.  sx/sy are the column/row directions; predecessors lie at -sx / -sy.
const int kSweepX[4] = {+1, -1, -1, +1};
const int kSweepY[4] = {+1, -1, +1, -1};

struct Counters {
  int64_t* c;  // [0] cost evaluations total, [1 + level] per level
  void add(int lev) { if (c) { c[0]++; c[1 + lev]++; } }
};

template <class Cost, class CostFn>
void propagate(const CostFn& cost, int lev, Grid<Cost>& g, int dir, const MatchParams& P, Counters& cnt) {
  const int sx = kSweepX[dir & 3], sy = kSweepY[dir & 3];
  const int n = g.n;
  for (int iy = 0; iy < g.Gh; ++iy) {
    int gy = sy > 0 ? iy : g.Gh - 1 - iy;
    for (int ix = 0; ix < g.Gw; ++ix) {
      int gx = sx > 0 ? ix : g.Gw - 1 - ix;
      size_t pi = (size_t)gy * g.Gw + gx;
      // Eq. 2 candidate order: current flow, vertical predecessor, horizontal
      // predecessor; a candidate replaces the current flow only if strictly
      // better, so ties keep the earlier one.
      const int qx[2] = {gx, gx - sx}, qy[2] = {gy - sy, gy};
      for (int c = 0; c < 2; ++c) {
        if (qx[c] < 0 || qx[c] >= g.Gw || qy[c] < 0 || qy[c] >= g.Gh) continue;
        int32_t fq = g.F[(size_t)qy[c] * g.Gw + qx[c]];
        if (fq == kEmpty) continue;
        if (P.skip_dup && fq == g.F[pi]) continue;
        cnt.add(lev);
        Cost e = cost(lev, gx * n, gy * n, unpack_x(fq), unpack_y(fq));
        if (e < g.C[pi]) { g.F[pi] = fq; g.C[pi] = e; }
      }
    }
  }
}

// Random search (section 3.1, with R_n = R n of section 3.2): one uniform
// offset per point, per axis an integer in [-nRQ, nRQ] (1/Q px), drawn with
// Philox4x32-10 keyed by the seed; counter = (pixel index y W + x, log2 n,
// step, field | pair << 2).
template <class Cost, class CostFn>
void random_search(const CostFn& cost, int W, int Q, int lev, Grid<Cost>& g, int step, const MatchParams& P,
                   Counters& cnt) {
  const int n = g.n;
  const int64_t rad = (int64_t)n * P.R * Q;
  const uint64_t span = (uint64_t)(2 * rad + 1);
  const uint32_t key[2] = {P.seed_lo, P.seed_hi};
  for (int gy = 0; gy < g.Gh; ++gy)
    for (int gx = 0; gx < g.Gw; ++gx) {
      size_t pi = (size_t)gy * g.Gw + gx;
      int32_t f = g.F[pi];
      if (f == kEmpty) continue;
      int px = gx * n, py = gy * n;
      uint32_t ctr[4] = {(uint32_t)(py * W + px), (uint32_t)lev, (uint32_t)step, P.field_id | (P.pair_id << 2)};
      uint32_t u[4];
      philox4x32_10(ctr, key, u);
      int ox = (int)((int64_t)(((uint64_t)u[0] * span) >> 32) - rad);
      int oy = (int)((int64_t)(((uint64_t)u[1] * span) >> 32) - rad);
      int fx = unpack_x(f) + ox, fy = unpack_y(f) + oy;
      cnt.add(lev);
      Cost e = cost(lev, px, py, fx, fy);
      if (e < g.C[pi]) { g.F[pi] = pack(fx, fy); g.C[pi] = e; }
    }
}

template <class Cost>
void write_grid(const Grid<Cost>& g, int W, int H, Cost inf, int32_t* flow, Cost* cost) {
  for (int i = 0; i < W * H; ++i) { flow[i] = kEmpty; cost[i] = inf; }
  for (int gy = 0; gy < g.Gh; ++gy)
    for (int gx = 0; gx < g.Gw; ++gx) {
      flow[(size_t)gy * g.n * W + gx * g.n] = g.F[(size_t)gy * g.Gw + gx];
      cost[(size_t)gy * g.n * W + gx * g.n] = g.C[(size_t)gy * g.Gw + gx];
    }
}

// The whole search for one field (src -> dst, patch radius r) with data
// term `cost` (section 3.3 allows either term; the search does not change).
//
// Steps, counted for max_steps: seeding (1); at the coarsest level P1 RS1 P2
// RS2 P3 RS3 P4 (section 3.1: 4 propagations and 3 random searches,
// alternating); at every finer level one level-entry step (carried points
// re-costed with the new patch, new points empty) and the same seven.
template <class Cost, class CostFn>
int match_field_t(const Desc& s, const Desc& d, int r, const MatchParams& P, const int32_t* proposal,
                  const CostFn& cost, Cost inf, int32_t* flow, Cost* out_cost, int64_t* counters) {
  Counters cnt{counters};
  const int K = 1 << P.k;
  int steps = 0;
  auto stop = [&]() { return P.max_steps >= 0 && steps >= P.max_steps; };
  Grid<Cost> g;
  g.n = K;
  g.Gw = (s.W + K - 1) / K;
  g.Gh = (s.H + K - 1) / K;
  g.F.assign((size_t)g.Gw * g.Gh, kEmpty);
  g.C.assign((size_t)g.Gw * g.Gh, inf);
  // Eq. 1 / Eq. 4: seeds on the coarsest grid from the kd-tree leaf of the
  // source patch's WHT vector, re-ranked by the data term on P^K_r.
  {
    Tree T;
    const int32_t* Vs = s.wht_for(r);
    if (P.use_kdtree) T = build_tree(d.wht_for(r), d.W * d.H, 9 * d.C, P.leaf);
    for (int gy = 0; gy < g.Gh; ++gy)
      for (int gx = 0; gx < g.Gw; ++gx) {
        int px = gx * K, py = gy * K;
        int32_t bestF = kEmpty;
        Cost bestC = inf;
        if (P.use_kdtree) {
          int st, c;
          query_tree(T, Vs + ((size_t)py * s.W + px) * 9 * s.C, st, c);
          for (int i = 0; i < c; ++i) {
            int q = T.perm[st + i];
            int fx = (q % d.W - px) * d.Q, fy = (q / d.W - py) * d.Q;
            cnt.add(P.k);
            Cost e = cost(P.k, px, py, fx, fy);
            if (e < bestC) { bestC = e; bestF = pack(fx, fy); }
          }
        }
        if (proposal) {
          int32_t fp = proposal[(size_t)gy * g.Gw + gx];
          if (fp != kEmpty) {
            cnt.add(P.k);
            Cost e = cost(P.k, px, py, unpack_x(fp), unpack_y(fp));
            if (e < bestC) { bestC = e; bestF = fp; }
          }
        }
        g.F[(size_t)gy * g.Gw + gx] = bestF;
        g.C[(size_t)gy * g.Gw + gx] = bestC;
      }
  }
  ++steps;
  if (stop()) { write_grid(g, s.W, s.H, inf, flow, out_cost); return steps; }
  for (int lev = P.k; lev >= 0; --lev) {
    const int n = 1 << lev;
    if (lev < P.k) {
      // Section 3.2: the coarser level's flows seed this level; points that
      // are new on this grid get their first value in the first propagation.
      Grid<Cost> ng;
      ng.n = n;
      ng.Gw = (s.W + n - 1) / n;
      ng.Gh = (s.H + n - 1) / n;
      ng.F.assign((size_t)ng.Gw * ng.Gh, kEmpty);
      ng.C.assign((size_t)ng.Gw * ng.Gh, inf);
      for (int gy = 0; gy < ng.Gh; gy += 2)
        for (int gx = 0; gx < ng.Gw; gx += 2) {
          int32_t f = g.F[(size_t)(gy / 2) * g.Gw + gx / 2];
          if (f == kEmpty) continue;
          ng.F[(size_t)gy * ng.Gw + gx] = f;
          ng.C[(size_t)gy * ng.Gw + gx] = cost(lev, gx * n, gy * n, unpack_x(f), unpack_y(f));
        }
      g = std::move(ng);
      ++steps;
      if (stop()) { write_grid(g, s.W, s.H, inf, flow, out_cost); return steps; }
    }
    for (int i = 0; i < P.n_prop; ++i) {
      propagate(cost, lev, g, i, P, cnt);
      ++steps;
      if (stop()) { write_grid(g, s.W, s.H, inf, flow, out_cost); return steps; }
      if (i < P.n_rs) {
        random_search(cost, s.W, d.Q, lev, g, i, P, cnt);
        ++steps;
        if (stop()) { write_grid(g, s.W, s.H, inf, flow, out_cost); return steps; }
      }
    }
  }
  write_grid(g, s.W, s.H, inf, flow, out_cost);
  return steps;
}

// The census data term of section 3.3 (cost_at above).
int match_field(const Desc& s, const Desc& d, int r, const MatchParams& P, const int32_t* proposal,
                int32_t* flow, int32_t* cost, int64_t* counters) {
  auto census = [&](int lev, int px, int py, int fx, int fy) { return cost_at(s, d, lev, r, px, py, fx, fy); };
  return match_field_t<int32_t>(s, d, r, P, proposal, census, kInf, flow, cost, counters);
}

// ---------------------------------------------------------------------------
// Section 3.4, the region-based filter that follows the consistency check:
// the partly filtered field is segmented into regions (neighbouring pixels
// join a region when their flows differ by less than 3 px; only neighbouring
// differences count, so a region's flow may drift arbitrarily), and each
// region of fewer than s pixels is removed whole if at least one outlier that
// the consistency check deleted could join it by the same rule.
//
// Reading: 4-neighbourhood, both for the segmentation and for "could join";
// "differ by less than 3 px" is the Euclidean length of the flow difference,
// strictly below 3 px: dx^2 + dy^2 < (3Q)^2 in 1/Q px.  A pixel belongs to
// the partly filtered field iff the check kept it and its flow is set; a
// deleted outlier is a pixel the check did not keep whose flow is set, and
// it would join with that flow.  One pass: the regions are those of the
// partly filtered field, and a removed region does not supply outliers to
// another.  Each region is named by its smallest pixel index y W + x.
bool similar3(int32_t f, int32_t g, int Q) {
  const int64_t dx = unpack_x(f) - unpack_x(g), dy = unpack_y(f) - unpack_y(g);
  return dx * dx + dy * dy < 9LL * Q * Q;
}

void region_filter(const int32_t* F, const uint8_t* keep, int W, int H, int Q, int s, int32_t* label,
                   uint8_t* keep_out, int32_t* out) {
  const size_t N = (size_t)W * H;
  auto in_field = [&](size_t i) { return keep[i] != 0 && F[i] != kEmpty; };
  auto deleted = [&](size_t i) { return keep[i] == 0 && F[i] != kEmpty; };
  const int ddx[4] = {-1, 1, 0, 0}, ddy[4] = {0, 0, -1, 1};
  std::vector<int32_t> lab(N, -1);
  std::vector<int64_t> count(N, 0);
  std::vector<char> joinable(N, 0);
  std::vector<size_t> stack;
  // flood fill from each unlabelled field pixel in raster order, so the seed
  // of a region is its smallest pixel index
  for (size_t i = 0; i < N; ++i) {
    if (!in_field(i) || lab[i] >= 0) continue;
    lab[i] = (int32_t)i;
    stack.assign(1, i);
    while (!stack.empty()) {
      const size_t p = stack.back();
      stack.pop_back();
      ++count[i];
      const int x = (int)(p % W), y = (int)(p / W);
      for (int t = 0; t < 4; ++t) {
        const int xx = x + ddx[t], yy = y + ddy[t];
        if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
        const size_t q = (size_t)yy * W + xx;
        if (in_field(q) && lab[q] < 0 && similar3(F[p], F[q], Q)) {
          lab[q] = (int32_t)i;
          stack.push_back(q);
        }
      }
    }
  }
  // could a deleted outlier join the region (a 4-neighbour of one of its
  // pixels, by the same rule)?
  for (size_t p = 0; p < N; ++p) {
    if (lab[p] < 0) continue;
    const int x = (int)(p % W), y = (int)(p / W);
    for (int t = 0; t < 4; ++t) {
      const int xx = x + ddx[t], yy = y + ddy[t];
      if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
      const size_t q = (size_t)yy * W + xx;
      if (deleted(q) && similar3(F[p], F[q], Q)) joinable[lab[p]] = 1;
    }
  }
  for (size_t p = 0; p < N; ++p) {
    const bool removed = lab[p] >= 0 && count[lab[p]] < s && joinable[lab[p]];
    const bool kept = lab[p] >= 0 && !removed;
    if (label) label[p] = lab[p];
    keep_out[p] = kept ? 1 : 0;
    out[p] = kept ? F[p] : kEmpty;
  }
}

// ---------------------------------------------------------------------------
// Section 3.5: sparsification for the interpolation step.  Over the
// outlier-filtered field, one sample is kept per 3x3 region that still holds
// at least e samples: the one whose summed forward-backward consistency
// errors (the |F(p) + F^b_j(p + F(p))| of Eq. 5, over the backward fields) are
// smallest.
//
// Reading: the 3x3 regions tile the image from (0,0) without overlap; those
// at the right and bottom borders are clipped and need e samples all the
// same.  A sample is a pixel whose filtered flow is set.  The backward flows
// are read at the nearest pixel exactly as in the consistency check.  Each
// error |e_j| is measured in fixed point, floor(2^14 |e_j|) with |e_j| in 1/Q
// px, i.e. the integer square root of (ex^2 + ey^2) 2^28, so that the choice
// is exact integer arithmetic (it differs from real-valued sums only when two
// sums lie within 2^-14 of a 1/Q px).  A lookup outside the second image or
// at an empty backward flow makes that sample's error the largest possible.
// The first minimum in raster order wins.
uint64_t isqrt64(uint64_t v) {  // floor(sqrt(v)), v < 2^62, by bisection
  uint64_t lo = 0, hi = (uint64_t)1 << 31;  // hi * hi > v
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (mid * mid <= v) lo = mid; else hi = mid;
  }
  return lo;
}

void sparsify(const int32_t* F, int W1, int H1, const int32_t* const* B, int n_bwd, int W2, int H2, int Q, int e,
              int32_t* pick, int32_t* sparse) {
  const uint64_t kNone = ~(uint64_t)0;
  const int Bw = (W1 + 2) / 3, Bh = (H1 + 2) / 3;
  if (sparse)
    for (size_t i = 0; i < (size_t)W1 * H1; ++i) sparse[i] = kEmpty;
  for (int by = 0; by < Bh; ++by)
    for (int bx = 0; bx < Bw; ++bx) {
      int count = 0, best = -1;
      uint64_t bestErr = 0;
      for (int y = 3 * by; y < std::min(3 * by + 3, H1); ++y)
        for (int x = 3 * bx; x < std::min(3 * bx + 3, W1); ++x) {
          const size_t i = (size_t)y * W1 + x;
          const int32_t f = F[i];
          if (f == kEmpty) continue;
          ++count;
          const int fx = unpack_x(f), fy = unpack_y(f);
          const int64_t mx = floordiv((int64_t)x * Q + fx + Q / 2, Q), my = floordiv((int64_t)y * Q + fy + Q / 2, Q);
          uint64_t err = 0;
          for (int j = 0; j < n_bwd && err != kNone; ++j) {
            if (mx < 0 || my < 0 || mx >= W2 || my >= H2 || B[j][(size_t)my * W2 + mx] == kEmpty) {
              err = kNone;
              break;
            }
            const int32_t b = B[j][(size_t)my * W2 + mx];
            const int64_t ex = fx + unpack_x(b), ey = fy + unpack_y(b);
            err += isqrt64((uint64_t)(ex * ex + ey * ey) << 28);
          }
          if (best < 0 || err < bestErr) { best = (int)i; bestErr = err; }
        }
      const int32_t chosen = count >= e ? best : -1;
      pick[(size_t)by * Bw + bx] = chosen;
      if (sparse && chosen >= 0) sparse[chosen] = F[chosen];
    }
}

// ---------------------------------------------------------------------------
// Section 3.3, the second data term: patch-based SIFT flow.  Every pixel gets
// a 128-dimensional SIFT vector (Lowe, IJCV 2004, computed densely and
// upright as in Liu et al.'s SIFT flow), PCA reduces the vectors to S
// "colours" (done in Python, oracle/ffo.py), the colour images are smoothed
// per level as in section 3.2, and the data term sums L2 colour distances
// over the subsampled patch.  WHTs (the kd-tree seeds) stay on CIELab.
//
// Readings (dense SIFT):
//  - input: the lightness plane of the 8-bit CIELab image (gray passes
//    through);
//  - gradient by central differences, coordinates clamped to the image:
//    gx = (L(x+1,y) - L(x-1,y)) / 2, gy = (L(x,y+1) - L(x,y-1)) / 2, y down;
//  - orientation atan2(gy, gx) in [0, 2 pi); 8 bins centred at o pi/4, the
//    magnitude split linearly between the two nearest bins;
//  - 4 x 4 cells of c = 3 px (SIFT flow's default cell size), cell (i, j)
//    (i the column) centred at p + ((i - 1.5) c, (j - 1.5) c);
//  - every sample q = p + (dx, dy) with |dx|, |dy| < 2.5 c (the support of the
//    bilinear cell weights) inside the image adds its binned magnitude with
//    weight exp(-(dx^2 + dy^2) / (2 sigma^2)), sigma = 2 c (half the window),
//    times max(0, 1 - |dx / c - (i - 1.5)|) max(0, 1 - |dy / c - (j - 1.5)|);
//    samples outside the image add nothing;
//  - element (4 j + i) 8 + o; the vector is scaled to unit length, clamped at
//    0.2 and scaled to unit length again (a zero vector stays zero).
constexpr int kSiftCell = 3;
constexpr int kSiftReach = 7;   // largest |dx| with a non-zero cell weight: < 2.5 c

void dense_sift(const uint8_t* L, int W, int H, double* out /* N x 128 */) {
  const double pi = 3.14159265358979323846;
  const size_t N = (size_t)W * H;
  std::vector<double> mag(N), tbin(N);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      auto at = [&](int xx, int yy) { return (double)L[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)]; };
      double gx = (at(x + 1, y) - at(x - 1, y)) / 2.0, gy = (at(x, y + 1) - at(x, y - 1)) / 2.0;
      double th = std::atan2(gy, gx);
      if (th < 0) th += 2 * pi;
      mag[(size_t)y * W + x] = std::sqrt(gx * gx + gy * gy);
      tbin[(size_t)y * W + x] = th / (pi / 4);
    }
  const double c = kSiftCell, sig = 2.0 * c;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      double v[128] = {0};
      for (int dy = -kSiftReach; dy <= kSiftReach; ++dy)
        for (int dx = -kSiftReach; dx <= kSiftReach; ++dx) {
          int qx = px + dx, qy = py + dy;
          if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
          double m = mag[(size_t)qy * W + qx];
          if (m == 0.0) continue;
          double t = tbin[(size_t)qy * W + qx];
          int o0 = (int)std::floor(t);
          double w1 = t - o0;
          o0 %= 8;
          int o1 = (o0 + 1) % 8;
          double g = std::exp(-(dx * dx + dy * dy) / (2 * sig * sig));
          for (int j = 0; j < 4; ++j) {
            double wy = 1.0 - std::fabs(dy / c - (j - 1.5));
            if (wy <= 0) continue;
            for (int i = 0; i < 4; ++i) {
              double wx = 1.0 - std::fabs(dx / c - (i - 1.5));
              if (wx <= 0) continue;
              double w = g * wx * wy * m;
              v[(4 * j + i) * 8 + o0] += w * (1.0 - w1);
              v[(4 * j + i) * 8 + o1] += w * w1;
            }
          }
        }
      double nn = 0;
      for (int e = 0; e < 128; ++e) nn += v[e] * v[e];
      if (nn > 0) {
        double s = 1.0 / std::sqrt(nn);
        nn = 0;
        for (int e = 0; e < 128; ++e) { v[e] = std::min(v[e] * s, 0.2); nn += v[e] * v[e]; }
        s = 1.0 / std::sqrt(nn);
        for (int e = 0; e < 128; ++e) v[e] *= s;
      }
      std::copy(v, v + 128, out + ((size_t)py * W + px) * 128);
    }
}

// Smoothed colour images of one image: (k+1) levels x S planes of int16
// codes (the PCA colours quantised in oracle/ffo.py), level j smoothed with
// n = 2^j by smooth_plane_t (section 3.2's smoothing on integer codes, output
// in code units).
struct SiftLevels {
  int W = 0, H = 0, S = 0, k = 0;
  std::vector<std::vector<int16_t>> lev;   // [level] S planes of H x W
  const int16_t* plane(int l, int s) const { return lev[l].data() + (size_t)s * W * H; }
};

// Readings (data term): E^n_r(p, f) is the sum over the (2r+1)^2 samples at
// stride n of the L2 distance of the S colours (the first S of the stored
// channels).  The target colour at the subpixel centre m = pQ + f is bilinear
// in the four neighbours of floor(m / Q) + n delta (weights (Q-a)(Q-b),
// a(Q-b), (Q-a)b, ab for the phase (a, b) = m mod Q; the +1 neighbours clamp
// to the image), the source colour is scaled by Q^2 to the same units, and a
// sample's distance is floor(sqrt(sum_s d_s^2 * 256 / Q^4)) (1/16 code units
// at every Q; exact integer square root, floor division for Q = 8).  Validity
// of f and lookup clamping as cost_at.
int32_t sift_cost_at(const SiftLevels& s, const SiftLevels& d, int Q, int lev, int r, int S, int px, int py, int fx,
                     int fy) {
  const int n = 1 << lev;
  int64_t mx = (int64_t)px * Q + fx, my = (int64_t)py * Q + fy;
  if (mx < 0 || my < 0 || mx > (int64_t)(d.W - 1) * Q || my > (int64_t)(d.H - 1) * Q) return kInf;
  int Mx = (int)floordiv(mx, Q), My = (int)floordiv(my, Q);
  int a = (int)(mx - (int64_t)Mx * Q), b = (int)(my - (int64_t)My * Q);
  const int64_t Q4 = (int64_t)Q * Q * Q * Q;
  int64_t total = 0;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      size_t ps = (size_t)clampi(py + n * dy, 0, s.H - 1) * s.W + clampi(px + n * dx, 0, s.W - 1);
      int X = clampi(Mx + n * dx, 0, d.W - 1), Y = clampi(My + n * dy, 0, d.H - 1);
      int X1 = std::min(X + 1, d.W - 1), Y1 = std::min(Y + 1, d.H - 1);
      int64_t ss = 0;
      for (int ch = 0; ch < S; ++ch) {
        const int16_t* P1 = s.plane(lev, ch);
        const int16_t* P2 = d.plane(lev, ch);
        int64_t t = (int64_t)(Q - a) * (Q - b) * P2[(size_t)Y * d.W + X] + (int64_t)a * (Q - b) * P2[(size_t)Y * d.W + X1] +
                    (int64_t)(Q - a) * b * P2[(size_t)Y1 * d.W + X] + (int64_t)a * b * P2[(size_t)Y1 * d.W + X1];
        int64_t e = (int64_t)Q * Q * P1[ps] - t;
        ss += e * e;
      }
      total += (int64_t)isqrt64((uint64_t)(Q <= 4 ? ss * (256 / Q4) : ss / (Q4 / 256)));
    }
  return (int32_t)total;
}

// The search of match_field_t with the SIFT-flow data term: seeds from the
// kd-tree over the CIELab WHTs of s / d (census descriptors), costs from the
// colour levels ss / sd.
int match_field_sift(const Desc& s, const Desc& d, const SiftLevels& ss, const SiftLevels& sd, int r, int S,
                     const MatchParams& P, int32_t* flow, int32_t* cost, int64_t* counters) {
  const int Q = d.Q;
  auto sift = [&](int lev, int px, int py, int fx, int fy) { return sift_cost_at(ss, sd, Q, lev, r, S, px, py, fx, fy); };
  return match_field_t<int32_t>(s, d, r, P, nullptr, sift, kInf, flow, cost, counters);
}

}  // namespace

// ===========================================================================
// C interface (ctypes).  Every function returns 0 on success, < 0 on bad
// arguments.  All buffers are host memory owned by the caller.
extern "C" {

int ffo_lab8(const uint8_t* img, int W, int H, int C, int row_stride, uint8_t* out) {
  if (!img || !out || W <= 0 || H <= 0 || (C != 1 && C != 3) || row_stride < W * C) return -1;
  const size_t N = (size_t)W * H;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const uint8_t* px = img + (size_t)y * row_stride + (size_t)x * C;
      if (C == 1) { out[(size_t)y * W + x] = px[0]; continue; }
      uint8_t lab[3];
      lab8_pixel(px[0], px[1], px[2], lab);
      for (int c = 0; c < 3; ++c) out[c * N + (size_t)y * W + x] = lab[c];
    }
  return 0;
}

int ffo_lanczos_weights(int n, int32_t* out /* n x 7 */) {
  if (n != 2 && n != 4 && n != 8 && n != 16) return -1;
  LanczosTable t = lanczos_table(n);
  for (int ph = 0; ph < n; ++ph) for (int k = 0; k < 7; ++k) out[ph * 7 + k] = t.w[ph][k];
  return 0;
}

int ffo_lab_tables(int32_t* gamma /* 256 */, int32_t* mat /* 9 */, int32_t* ftab /* 65537 */) {
  const LabTables& T = lab_tables();
  std::memcpy(gamma, T.gamma, sizeof(T.gamma));
  std::memcpy(mat, T.mat, sizeof(T.mat));
  std::memcpy(ftab, T.f.data(), 65537 * sizeof(int32_t));
  return 0;
}

int ffo_smooth(const uint8_t* plane, int W, int H, int n, int16_t* out) {
  if (!plane || !out || W <= 0 || H <= 0 || n < 1 || n > 16 || (n & (n - 1))) return -1;
  smooth_plane(plane, W, H, n, out);
  return 0;
}

int ffo_census(const int16_t* S, int W, int H, int C, int n, int Q, int a, int b, uint32_t* out) {
  if (!S || !out || W <= 0 || H <= 0 || a < 0 || a >= Q || b < 0 || b >= Q) return -1;
  census_plane(S, W, H, C, n, Q, a, b, out);
  return 0;
}

int ffo_wht(const uint8_t* lab, int W, int H, int C, int rho, int32_t* out) {
  if (!lab || !out || W <= 0 || H <= 0 || rho < 1) return -1;
  wht(lab, W, H, C, rho, out);
  return 0;
}

int ffo_walsh(int s, int t, int rho) { return walsh(s, t, rho); }

int ffo_tree_depth(int N, int leaf) { return tree_depth(N, leaf); }

// node_dim / node_split: (2 << depth) - 1 entries; perm: N entries
int ffo_kdtree_build(const int32_t* V, int N, int D, int leaf, int32_t* node_dim, int32_t* node_split,
                     int32_t* perm) {
  if (!V || N <= 0 || D <= 0 || leaf < 1) return -1;
  Tree T = build_tree(V, N, D, leaf);
  std::copy(T.dim.begin(), T.dim.end(), node_dim);
  std::copy(T.split.begin(), T.split.end(), node_split);
  std::copy(T.perm.begin(), T.perm.end(), perm);
  return tree_depth(N, leaf);
}

void ffo_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }

void* ffo_desc_create(const uint8_t* img, int W, int H, int C, int row_stride, int k, int Q, const int32_t* radii,
                      int n_radii) {
  if (!img || W <= 0 || H <= 0 || (C != 1 && C != 3) || k < 0 || k > 4 || Q < 1 || Q > 8 || (Q & (Q - 1)) ||
      n_radii < 0 || n_radii > 4)
    return nullptr;
  Desc* d = new Desc;
  d->W = W; d->H = H; d->C = C; d->k = k; d->Q = Q;
  const size_t N = (size_t)W * H;
  d->lab.resize(C * N);
  ffo_lab8(img, W, H, C, row_stride, d->lab.data());
  d->smooth.resize(k + 1);
  for (int lev = 0; lev <= k; ++lev) {
    d->smooth[lev].resize(C * N);
    for (int c = 0; c < C; ++c) smooth_plane(d->lab.data() + c * N, W, H, 1 << lev, d->smooth[lev].data() + c * N);
  }
  d->planes.resize((size_t)(k + 1) * Q * Q);
  for (int lev = 0; lev <= k; ++lev)
    for (int b = 0; b < Q; ++b)
      for (int a = 0; a < Q; ++a) {
        std::vector<uint32_t>& pl = d->planes[(size_t)lev * Q * Q + b * Q + a];
        pl.resize(N);
        census_plane(d->smooth[lev].data(), W, H, C, 1 << lev, Q, a, b, pl.data());
      }
  for (int i = 0; i < n_radii; ++i) {
    d->radii.push_back(radii[i]);
    d->whtv.emplace_back(N * 9 * C);
    wht(d->lab.data(), W, H, C, radii[i], d->whtv.back().data());
  }
  return d;
}

void ffo_desc_free(void* h) { delete static_cast<Desc*>(h); }

int ffo_desc_lab(void* h, uint8_t* out) {
  Desc* d = static_cast<Desc*>(h);
  std::copy(d->lab.begin(), d->lab.end(), out);
  return 0;
}
int ffo_desc_smooth(void* h, int lev, int16_t* out) {
  Desc* d = static_cast<Desc*>(h);
  if (lev < 0 || lev > d->k) return -1;
  std::copy(d->smooth[lev].begin(), d->smooth[lev].end(), out);
  return 0;
}
int ffo_desc_plane(void* h, int lev, int a, int b, uint32_t* out) {
  Desc* d = static_cast<Desc*>(h);
  if (lev < 0 || lev > d->k || a < 0 || a >= d->Q || b < 0 || b >= d->Q) return -1;
  const uint32_t* p = d->plane(lev, a, b);
  std::copy(p, p + (size_t)d->W * d->H, out);
  return 0;
}
int ffo_desc_wht(void* h, int rho, int32_t* out) {
  Desc* d = static_cast<Desc*>(h);
  const int32_t* v = d->wht_for(rho);
  if (!v) return -1;
  std::copy(v, v + (size_t)d->W * d->H * 9 * d->C, out);
  return 0;
}

int32_t ffo_cost(void* hs, void* hd, int lev, int r, int px, int py, int fx, int fy) {
  return cost_at(*static_cast<Desc*>(hs), *static_cast<Desc*>(hd), lev, r, px, py, fx, fy);
}

// params: k, R, leaf, n_prop, n_rs, use_kdtree, skip_dup, max_steps, seed_lo,
// seed_hi, field_id, pair_id (12 int64 values)
int ffo_match_field(void* hs, void* hd, int r, const int64_t* params, const int32_t* proposal, int32_t* flow,
                    int32_t* cost, int64_t* counters) {
  const Desc& s = *static_cast<Desc*>(hs);
  const Desc& d = *static_cast<Desc*>(hd);
  MatchParams P;
  P.k = (int)params[0]; P.R = (int)params[1]; P.leaf = (int)params[2]; P.n_prop = (int)params[3];
  P.n_rs = (int)params[4]; P.use_kdtree = (int)params[5]; P.skip_dup = (int)params[6];
  P.max_steps = (int)params[7]; P.seed_lo = (uint32_t)params[8]; P.seed_hi = (uint32_t)params[9];
  P.field_id = (uint32_t)params[10]; P.pair_id = (uint32_t)params[11];
  if (P.k < 0 || P.k > s.k || P.k > d.k || s.Q != d.Q || s.C != d.C || r < 1) return -1;
  if (P.use_kdtree && (!s.wht_for(r) || !d.wht_for(r))) return -2;
  if (!P.use_kdtree && !proposal) return -3;
  return match_field(s, d, r, P, proposal, flow, cost, counters);
}

// Eq. 5 two-way consistency check (section 3.4).  Reading: the backward flow
// is looked up at the nearest pixel m = round-half-up((p Q + F(p)) / Q); a
// point is kept iff m is inside the second image and, for every backward
// field j, B_j(m) is not empty and |F(p) + B_j(m)|^2 < (eps Q)^2.
int ffo_consistency(const int32_t* F, int W1, int H1, const int32_t* const* B, int n_bwd, int W2, int H2, int Q,
                    int eps_q, uint8_t* keep, int32_t* filtered) {
  if (!F || !keep || !filtered || n_bwd < 1 || n_bwd > 4 || Q < 1) return -1;
  const int64_t lim = (int64_t)eps_q * eps_q;
  for (int y = 0; y < H1; ++y)
    for (int x = 0; x < W1; ++x) {
      size_t i = (size_t)y * W1 + x;
      int32_t f = F[i];
      bool ok = f != kEmpty;
      if (ok) {
        int fx = unpack_x(f), fy = unpack_y(f);
        int64_t mx = floordiv((int64_t)x * Q + fx + Q / 2, Q), my = floordiv((int64_t)y * Q + fy + Q / 2, Q);
        ok = mx >= 0 && my >= 0 && mx < W2 && my < H2;
        for (int j = 0; ok && j < n_bwd; ++j) {
          int32_t b = B[j][(size_t)my * W2 + mx];
          if (b == kEmpty) { ok = false; break; }
          int64_t ex = fx + unpack_x(b), ey = fy + unpack_y(b);
          if (ex * ex + ey * ey >= lim) ok = false;
        }
      }
      keep[i] = ok ? 1 : 0;
      filtered[i] = ok ? f : kEmpty;
    }
  return 0;
}

// Region-based filter of section 3.4 (see region_filter above).  F: the
// field before the consistency check; keep: the check's mask; label
// (nullable): region name per pixel, -1 outside the partly filtered field.
int ffo_region_filter(const int32_t* F, const uint8_t* keep, int W, int H, int Q, int s, int32_t* label,
                      uint8_t* keep_out, int32_t* out) {
  if (!F || !keep || !keep_out || !out || W <= 0 || H <= 0 || Q < 1 || s < 0) return -1;
  region_filter(F, keep, W, H, Q, s, label, keep_out, out);
  return 0;
}

// Sparsification of section 3.5 (see sparsify above).  F: the outlier-
// filtered field; B: n_bwd backward fields; pick: ceil(H1/3) x ceil(W1/3)
// chosen pixel indices (-1: fewer than e samples); sparse (nullable): the
// chosen flows, FF_EMPTY elsewhere.
int ffo_sparsify(const int32_t* F, int W1, int H1, const int32_t* const* B, int n_bwd, int W2, int H2, int Q, int e,
                 int32_t* pick, int32_t* sparse) {
  if (!F || !B || !pick || W1 <= 0 || H1 <= 0 || W2 <= 0 || H2 <= 0 || n_bwd < 1 || n_bwd > 4 || Q < 1) return -1;
  sparsify(F, W1, H1, B, n_bwd, W2, H2, Q, e, pick, sparse);
  return 0;
}

uint64_t ffo_isqrt64(uint64_t v) { return isqrt64(v); }

// Exact nearest-neighbour field (the NNF row of Table 1), for tiny images
// only: for every grid point of level lev, the minimum over every flow whose
// centre lies inside the target image, in 1/Q px steps.  First minimum in
// (fy, fx) raster order.
int ffo_brute_nnf(void* hs, void* hd, int lev, int r, int32_t* flow, int32_t* cost) {
  const Desc& s = *static_cast<Desc*>(hs);
  const Desc& d = *static_cast<Desc*>(hd);
  const int n = 1 << lev, Q = d.Q;
  const int Gw = (s.W + n - 1) / n, Gh = (s.H + n - 1) / n;
  for (int gy = 0; gy < Gh; ++gy)
    for (int gx = 0; gx < Gw; ++gx) {
      int px = gx * n, py = gy * n;
      int32_t best = kInf, bf = kEmpty;
      for (int my = 0; my <= (d.H - 1) * Q; ++my)
        for (int mx = 0; mx <= (d.W - 1) * Q; ++mx) {
          int fx = mx - px * Q, fy = my - py * Q;
          int32_t e = cost_at(s, d, lev, r, px, py, fx, fy);
          if (e < best) { best = e; bf = pack(fx, fy); }
        }
      flow[(size_t)gy * Gw + gx] = bf;
      cost[(size_t)gy * Gw + gx] = best;
    }
  return 0;
}

// ---------------------------------------------------------------------------
// SIFT-flow data term (section 3.3, see dense_sift and sift_cost_at above).

// L: H x W lightness plane; out: H x W x 128 doubles.
int ffo_dense_sift(const uint8_t* L, int W, int H, double* out) {
  if (!L || !out || W <= 0 || H <= 0) return -1;
  dense_sift(L, W, H, out);
  return 0;
}

// One int16 plane smoothed with n (power of two, <= 16), output in the
// input's units.
int ffo_smooth_codes(const int16_t* plane, int W, int H, int n, int16_t* out) {
  if (!plane || !out || W <= 0 || H <= 0 || n < 1 || n > 16 || (n & (n - 1))) return -1;
  smooth_plane_t(plane, W, H, n, 0, out);
  return 0;
}

// codes: H x W x S int16 (channels last).  Levels 0..k.
void* ffo_sift_levels_create(const int16_t* codes, int W, int H, int S, int k) {
  if (!codes || W <= 0 || H <= 0 || S < 1 || S > 128 || k < 0 || k > 4) return nullptr;
  SiftLevels* L = new SiftLevels;
  L->W = W; L->H = H; L->S = S; L->k = k;
  const size_t N = (size_t)W * H;
  std::vector<int16_t> pl(N);
  L->lev.resize(k + 1);
  for (int l = 0; l <= k; ++l) {
    L->lev[l].resize(N * S);
    for (int ch = 0; ch < S; ++ch) {
      for (size_t i = 0; i < N; ++i) pl[i] = codes[i * S + ch];
      smooth_plane_t(pl.data(), W, H, 1 << l, 0, L->lev[l].data() + ch * N);
    }
  }
  return L;
}

void ffo_sift_levels_free(void* h) { delete static_cast<SiftLevels*>(h); }

// out: S x H x W int16
int ffo_sift_levels_get(void* h, int lev, int16_t* out) {
  SiftLevels* L = static_cast<SiftLevels*>(h);
  if (lev < 0 || lev > L->k) return -1;
  std::copy(L->lev[lev].begin(), L->lev[lev].end(), out);
  return 0;
}

int32_t ffo_sift_cost(void* ss, void* sd, int Q, int lev, int r, int S, int px, int py, int fx, int fy) {
  return sift_cost_at(*static_cast<SiftLevels*>(ss), *static_cast<SiftLevels*>(sd), Q, lev, r, S, px, py, fx, fy);
}

// hs / hd: census descriptors (dimensions, Q, WHT vectors for the kd-tree);
// ss / sd: colour levels; params as ffo_match_field (the proposal is not
// used with this data term).
int ffo_match_field_sift(void* hs, void* hd, void* ss, void* sd, int r, int S, const int64_t* params, int32_t* flow,
                         int32_t* cost, int64_t* counters) {
  const Desc& s = *static_cast<Desc*>(hs);
  const Desc& d = *static_cast<Desc*>(hd);
  const SiftLevels& cs = *static_cast<SiftLevels*>(ss);
  const SiftLevels& cd = *static_cast<SiftLevels*>(sd);
  MatchParams P;
  P.k = (int)params[0]; P.R = (int)params[1]; P.leaf = (int)params[2]; P.n_prop = (int)params[3];
  P.n_rs = (int)params[4]; P.use_kdtree = (int)params[5]; P.skip_dup = (int)params[6];
  P.max_steps = (int)params[7]; P.seed_lo = (uint32_t)params[8]; P.seed_hi = (uint32_t)params[9];
  P.field_id = (uint32_t)params[10]; P.pair_id = (uint32_t)params[11];
  if (P.k < 0 || P.k > s.k || P.k > d.k || P.k > cs.k || P.k > cd.k || s.Q != d.Q || r < 1) return -1;
  if (cs.W != s.W || cs.H != s.H || cd.W != d.W || cd.H != d.H || S < 1 || S > cs.S || S > cd.S) return -1;
  if (!P.use_kdtree || !s.wht_for(r) || !d.wht_for(r)) return -2;
  return match_field_sift(s, d, cs, cd, r, S, P, flow, cost, counters);
}

}  // extern "C"

