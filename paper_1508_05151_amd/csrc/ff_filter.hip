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
