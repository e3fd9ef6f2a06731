/*
 * ff.h -- C ABI of the MI355X (gfx950) Flow Fields correspondence-field search.
 *
 * Method: C. Bailer, B. Taetz, D. Stricker, "Flow Fields: Dense Correspondence
 * Fields for Highly Accurate Large Displacement Optical Flow Estimation",
 * ICCV 2015.  Section 3 defines the problem: for every pixel p1 of I1 find the
 * flow F(p1) = M(p1) - p1 that minimises a patch data term against I2.
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE pointers unless a comment says "host".
 *  - Every call that takes a stream only enqueues work on it: it never
 *    allocates, never synchronises and never copies to the host, so it may be
 *    captured in a HIP graph -- except the first call on a device, which
 *    computes the library's constant tables there (two small kernels on the
 *    null stream and a synchronisation; call ff_init() first when the first
 *    use is inside a capture).
 *  - Arguments are validated on the host before anything is enqueued; on an
 *    error nothing is enqueued and a negative ff_status is returned.
 *  - Flows are packed int16x2 words: low half dx, high half dy, both in 1/Q
 *    pixel ("subpel" Q in {1,2,4,8}); FF_EMPTY marks a pixel with no flow.
 *    Costs are int32 Hamming sums; FF_COST_INF marks "no cost".
 *  - The library keeps no per-call device state.  Buffers belong to the
 *    caller; sizes come from the *_bytes / *_init queries below.  The one
 *    exception is ff_match_field_noalloc, whose scratch is a static device
 *    array of the library.
 */
#ifndef FF_H_
#define FF_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FF_EMPTY ((int32_t)0x80008000u)
#define FF_COST_INF ((int32_t)0x7fffffff)
#define FF_MAX_RADII 4

typedef enum {
  FF_OK = 0,
  FF_ERR_ARG = -1,        /* null pointer, bad size, bad parameter */
  FF_ERR_SIZE = -2,       /* image too large for the packed formats */
  FF_ERR_WORKSPACE = -3,  /* workspace or descriptor buffer too small */
  FF_ERR_UNSUPPORTED = -4,
  FF_ERR_HIP = -5,        /* a HIP launch or query failed */
  FF_ERR_DEVICE = -6      /* a device-side watchdog fired (see ff_read_status) */
} ff_status;

/* One image: width x height pixels, channels 3 (RGB, uint8) or 1 (gray),
 * row_stride in bytes (>= width * channels). */
typedef struct {
  int32_t width, height, channels, row_stride;
} ff_image;

/*
 * Descriptor layout of one image (host struct, filled by ff_desc_init).
 * The device blob it describes holds, at the byte offsets given:
 *  - lab:    channels planes of H*W uint8: 8-bit CIELab (section 3.3 computes
 *            the census data term in CIELab); gray images pass through;
 *  - smooth: (k+1) levels x channels planes of H*W int16, Q4 fixed point:
 *            level j is I^n with n = 2^j (section 3.2: area downsampling by
 *            n, then Lanczos upsampling to full resolution; level 0 = 16 x lab);
 *  - census: (k+1) levels x subpel^2 phases of H*W uint32: the 3x3 census
 *            (section 3.3) of I^n with neighbour stride n (the subsampled
 *            patch of Eq. 3), on I^n shifted by the subpixel phase (a/Q, b/Q)
 *            with bilinear weights (section 3.1); byte c = channel c;
 *            plane index = level * Q*Q + b*Q + a;
 *  - census_t: the same planes transposed (W rows of H words), so that the
 *            column walks of the propagation read contiguous words;
 *  - wht:    n_radii blocks of H*W vectors of wht_stride int32: the first 9
 *            Walsh-Hadamard projections per channel of the patch of radius
 *            rho (section 3.1; odd extents split into rho and rho+1).
 */
typedef struct {
  int32_t width, height, channels, k, subpel, n_radii;
  int32_t radii[FF_MAX_RADII];
  int32_t wht_dims;    /* 9 * channels */
  int32_t wht_stride;  /* int32 words per WHT vector (32 for RGB, 16 gray) */
  size_t off_lab, off_smooth, off_census, off_census_t, off_wht;
  size_t plane_bytes;  /* H*W*4, the census plane pitch (both layouts) */
  size_t bytes;        /* total device bytes of the blob */
} ff_desc;

/* Search parameters (section 4 gives the paper's values in brackets). */
typedef struct {
  int32_t k;          /* hierarchy levels: coarsest grid step 2^k [3]; <= desc k */
  int32_t R;          /* random-search radius in px at full resolution [1]; R_n = R n */
  int32_t leaf;       /* kd-tree leaf size l [8], 1..64 */
  int32_t n_prop;     /* propagation sweeps per level [4] */
  int32_t n_rs;       /* random searches per level, after sweeps 1..n_rs [3] */
  int32_t use_kdtree; /* 1: kd-tree seeds (Eq. 1 / Eq. 4), the tree built in the
                         call; 2: kd-tree seeds from the tree that
                         ff_match_field_tree left in the same workspace for
                         the same field and arguments (ff_match_field, or
                         ff_match_batch with one job; refused by
                         ff_match_field_noalloc and ff_match_sift);
                         0: proposal only */
  int32_t max_steps;  /* < 0: whole search; else stop after this many steps
                         (1 seed step, 7 at the coarsest level, 8 per finer
                         level) and write the current grid -- for inspection */
  uint32_t field_id;  /* 0..3, part of the random-search counter */
  uint32_t pair_id;   /* part of the random-search counter */
  int32_t band_rows;  /* propagation band height: 8, 16 (default) or 32 rows per
                         workgroup; results are identical for every value */
  int32_t pipeline;   /* 1 (default): two consecutive sweeps with the same
                         horizontal direction (and the random search between
                         them) run as one launch, the second sweep starting on
                         columns that the first and the search have finished;
                         0: one launch per sweep and per search.  Results are
                         identical; max_steps >= 0 implies 0 */
  int32_t watchdog_us; /* 0 (default): every wait of one workgroup on another
                          gives up after 2 s and the call reports
                          FF_ERR_DEVICE; > 0: that limit in microseconds
                          (a tiny value forces the error path in tests) */
  uint64_t seed;      /* Philox key */
} ff_match_params;

/* Fill the paper's defaults (k=3, R=1, l=8, 4 sweeps, 3 searches). Host. */
void ff_default_params(ff_match_params* p);

/* Compute the constant tables (8-bit CIELab conversion of section 3.3,
 * Lanczos-3 weights of section 3.2) on the current device and look up the
 * no-allocation scratch array there (idempotent, synchronous; allocates
 * nothing).  Returns FF_ERR_HIP if the device cannot be used. */
ff_status ff_init(void);

/* Host-only: compute the descriptor layout for an image.  radii (host) lists
 * the patch radii whose WHT vectors are kept (e.g. {8, 6}), 1..15 each.
 * k in 0..4, subpel in {1,2,4,8}, width*height <= 2^22, width, height <= 8191. */
ff_status ff_desc_init(ff_desc* d, const ff_image* img, int32_t k, int32_t subpel, const int32_t* radii,
                       int32_t n_radii);

/* Compute an image's descriptors (Lab8, I^n, census planes, WHT vectors) into
 * blob (d->bytes device bytes).  pixels: device image as described by img
 * (the same image that d was initialised with).  Section 3.1-3.3. */
ff_status ff_compute_descriptors(const ff_desc* d, const ff_image* img, const uint8_t* pixels, void* blob,
                                 size_t blob_bytes, hipStream_t stream);

/* Workspace bytes for one ff_match_field call (kd-tree, level grids,
 * propagation progress counters, status word). */
size_t ff_match_workspace_bytes(const ff_desc* src, const ff_desc* dst, int32_t radius, const ff_match_params* p);

/*
 * One Flow Field src -> dst with patch radius `radius` (sections 3.1, 3.2):
 * kd-tree over dst's WHT(radius) vectors, seeds on the 2^k grid re-ranked by
 * the data term on P^{2^k}_r (Eq. 4), then per level n = 2^k..1 the
 * alternating propagation sweeps (Eq. 2, four directions) and random
 * searches (offsets up to R n, subpixel), coarse flows seeding the next
 * level.  Both descriptors need the same channels, k >= p->k and subpel, and
 * must hold WHT vectors for `radius` (unless p->use_kdtree == 0).
 *  proposal: nullable; ceil(H/2^k) x ceil(W/2^k) packed flows (1/Q px), one
 *            extra seed candidate per coarse grid point, evaluated after the
 *            kd-tree leaf; FF_EMPTY entries are skipped.
 *  flow, cost: src H*W outputs (row-major).  With max_steps >= 0 only grid
 *            points of the level reached hold values; all others are
 *            FF_EMPTY / FF_COST_INF.
 */
ff_status ff_match_field(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                         int32_t radius, const ff_match_params* p, const int32_t* proposal, int32_t* flow,
                         int32_t* cost, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * The kd-tree of ff_match_field alone (section 3.1, over dst's WHT(radius)
 * vectors), built into `workspace`, so that it can start as soon as the WHT
 * vectors exist (ff_compute_lab_wht) while the census planes are still being
 * computed.  A following ff_match_field with the same arguments, the same
 * workspace and p->use_kdtree = 2 seeds from it instead of building it; its
 * results equal a call with use_kdtree = 1.  p->use_kdtree must be nonzero.
 * The blobs need only their WHT regions at this point.
 */
ff_status ff_match_field_tree(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                              int32_t radius, const ff_match_params* p, void* workspace, size_t workspace_bytes,
                              hipStream_t stream);

/*
 * Batched matching: many fields (of pairs of any sizes) in one call, every
 * stage launched once for all of them.  One job = one ff_match_field call's
 * arguments; p supplies the shared parameters (k, R, leaf, n_prop, n_rs,
 * use_kdtree, max_steps, band_rows) and each job its own radius, field_id,
 * pair_id, seed and proposal.  All descriptors must share subpel.  Each job's
 * flow/cost equal, byte for byte, what ff_match_field gives for it alone.
 * jobs: host array (read during the call only); workspace: device,
 * ff_match_batch_workspace_bytes() bytes.
 */
typedef struct {
  const ff_desc* src;      /* host */
  const void* src_blob;    /* device */
  const ff_desc* dst;      /* host */
  const void* dst_blob;    /* device */
  int32_t radius;
  uint32_t field_id, pair_id;
  uint32_t reserved;
  uint64_t seed;
  const int32_t* proposal; /* device, nullable */
  int32_t* flow;           /* device, src H*W */
  int32_t* cost;           /* device, src H*W */
} ff_field_job;

size_t ff_match_batch_workspace_bytes(const ff_field_job* jobs, int32_t n_jobs, const ff_match_params* p);
ff_status ff_match_batch(const ff_field_job* jobs, int32_t n_jobs, const ff_match_params* p, void* workspace,
                         size_t workspace_bytes, hipStream_t stream);

/*
 * Eq. 5 (section 3.4): two-way forward/backward consistency check.  Keep p iff
 * the nearest pixel m = round-half-up(p + F(p)) lies in the second image and
 * for every backward field j, B_j(m) is not empty and
 * |F(p) + B_j(m)|^2 < eps_q^2 (eps_q = epsilon * Q, in 1/Q px).
 *  flow_bwd: host array of n_bwd (1..4) device pointers to w2*h2 fields.
 *  keep: w1*h1 bytes (1 kept, 0 removed); flow_filtered: w1*h1 flows, FF_EMPTY
 *  where removed.
 */
ff_status ff_consistency_filter(const int32_t* flow_fwd, int32_t w1, int32_t h1, const int32_t* const* flow_bwd,
                                int32_t n_bwd, int32_t w2, int32_t h2, int32_t subpel, int32_t eps_q, uint8_t* keep,
                                int32_t* flow_filtered, hipStream_t stream);

/*
 * Section 3.4, the region-based filter that follows Eq. 5's check.  The
 * partly filtered field (the pixels the check kept) is segmented into
 * regions: 4-neighbours belong to one region when their flows differ by less
 * than 3 px (dx^2 + dy^2 < (3 subpel)^2 in 1/subpel px; only neighbouring
 * differences count).  A region of fewer than min_region pixels (s: 50 for
 * the paper's Sintel and Middlebury settings, 150 for KITTI) is removed whole
 * if some deleted outlier -- a pixel the check did not keep whose flow is
 * set -- 4-adjacent to one of its pixels could join it by the same rule.
 * One pass: removed regions do not supply outliers to other regions.
 *  flow: w*h packed flows before the check (ff_match_field's F);
 *  keep: w*h bytes, the check's mask (ff_consistency_filter's keep; a pixel
 *        with keep != 0 and FF_EMPTY flow counts as neither kept nor deleted);
 *  label: nullable, w*h int32: each kept pixel's region, named by its
 *        smallest pixel index y*w + x; -1 for pixels the check did not keep;
 *  keep_out, flow_out: w*h final mask (1 kept) and field (FF_EMPTY where
 *        removed by either filter);
 *  workspace: ff_region_filter_workspace_bytes(w, h) bytes (two int32 per
 *        pixel), contents on entry irrelevant.
 * Errors: FF_ERR_ARG for null pointers, sizes below 1, subpel not in
 * {1,2,4,8} or min_region < 0; FF_ERR_SIZE beyond 8191 per side or 2^22
 * pixels; FF_ERR_WORKSPACE if the workspace is too small.
 */
size_t ff_region_filter_workspace_bytes(int32_t width, int32_t height);
ff_status ff_region_filter(const int32_t* flow, const uint8_t* keep, int32_t width, int32_t height, int32_t subpel,
                           int32_t min_region, int32_t* label, uint8_t* keep_out, int32_t* flow_out, void* workspace,
                           size_t workspace_bytes, hipStream_t stream);

/*
 * Section 3.5: sparsification of the outlier-filtered field for the
 * interpolation that follows the search (not part of this library).  The
 * image is tiled from (0,0) by non-overlapping 3x3 regions (clipped at the
 * right and bottom borders); each region that still holds at least
 * min_samples samples (e: 4 for the paper's Sintel setting, 7 Middlebury,
 * 9 KITTI) keeps exactly one, the sample whose summed forward-backward
 * consistency errors over the backward fields are smallest; a sample is a
 * pixel whose flow is set.  Errors are those of Eq. 5, |F(p) + B_j(m)| with m
 * the nearest pixel of p + F(p) (rounding half up), each measured as
 * floor(2^14 |e_j|) with |e_j| in 1/subpel px (exact integer square root); a
 * lookup outside the second image or at an FF_EMPTY backward flow counts as
 * the largest error; the first minimum in raster order wins.
 *  flow: w1*h1 filtered field (ff_region_filter's flow_out, or
 *        ff_consistency_filter's flow_filtered), FF_EMPTY where removed;
 *  flow_bwd: host array of n_bwd (1..4) device pointers to w2*h2 fields;
 *  pick: ceil(h1/3) x ceil(w1/3) int32: the chosen pixel index y*w1 + x of
 *        each region, -1 if it holds fewer than min_samples samples;
 *  flow_sparse: nullable, w1*h1: the chosen samples' flows, FF_EMPTY
 *        elsewhere.
 * Errors: FF_ERR_ARG for null pointers, sizes below 1, n_bwd outside 1..4 or
 * subpel not in {1,2,4,8}; FF_ERR_SIZE beyond 8191 per side or 2^22 pixels.
 */
ff_status ff_sparsify(const int32_t* flow, int32_t w1, int32_t h1, const int32_t* const* flow_bwd, int32_t n_bwd,
                      int32_t w2, int32_t h2, int32_t subpel, int32_t min_samples, int32_t* pick,
                      int32_t* flow_sparse, hipStream_t stream);

/*
 * Inspection: build the kd-tree of section 3.1 alone (the one ff_match_field
 * builds first): over every pixel of the image's WHT(radius) vectors, split
 * while a node holds more than `leaf` points, on the dimension of largest
 * max-min spread (lowest on ties), at the median of (key, pixel index); left
 * child = first floor(cnt/2).  Outputs in heap order (children 2i+1, 2i+2):
 * node_dim (-1 = leaf) and node_split, ff_tree_nodes() entries each; perm: the
 * H*W pixel indices, leaves left to right, ascending inside each leaf.
 * workspace: ff_match_workspace_bytes() of a field with this dst suffices.
 */
int32_t ff_tree_nodes(int32_t n_points, int32_t leaf);
ff_status ff_build_kdtree(const ff_desc* d, const void* blob, int32_t radius, int32_t leaf, int32_t* node_dim,
                          int32_t* node_split, int32_t* perm, void* workspace, size_t workspace_bytes,
                          hipStream_t stream);

/*
 * Learned coarse-flow proposal (an extension outside the paper: the paper's
 * initial matches come from the kd-tree of section 3.1 only).  A fixed 6-layer
 * 3x3 convolutional network maps the stacked RGB pair to one flow per point
 * of the 1/8 grid, i.e. the seed grid of a k = 3 match (section 3.2), whose
 * rounded value the seed step evaluates as one more candidate through
 * ff_field_job.proposal / ff_match_field's proposal: the data term of Eq. 1
 * still decides.
 *
 * Layers (Cin, Cout, stride, dilation, ReLU): (6,32,2,1,y) (32,32,2,1,y)
 * (32,32,2,1,y) (32,32,1,4,y) (32,32,1,8,y) (32,2,1,1,n); zero padding equal
 * to the dilation, so an output is ceil(size / stride).  Input x = RGB / 255
 * - 1/2 of both frames (6 channels); flow in px = 32 x output.  Weights and
 * activations are rounded to bf16 (nearest even); sums accumulate in fp32.
 *
 * params: device float32[ff_net_param_count()], per layer W[co][ci][ky][kx]
 *   then b[co] (39330 values).
 * img1, img2: device u8, batch x height x width x 3 each (RGB, rows packed).
 * workspace: device, ff_net_workspace_bytes(batch, width, height) bytes.
 * Errors: FF_ERR_ARG for null pointers, subpel not in {1,2,4,8}, batch not
 * in 1..256 or a side under 8 or above 8191; FF_ERR_SIZE if batch x width x
 * height exceeds 2^30; FF_ERR_WORKSPACE if the workspace is too small.
 */
int32_t ff_net_param_count(void);
size_t ff_net_workspace_bytes(int32_t batch, int32_t width, int32_t height);

/* Inference.  proposal: device int32, batch x ceil(height/8) x ceil(width/8)
 * packed flows in 1/subpel px (round to nearest even of 32 x out x subpel,
 * clamped to +-32767); flow_out (device, nullable): the same points as fp32
 * (x, y) pairs in output units (px / 32). */
ff_status ff_proposal_forward(const float* params, const uint8_t* img1, const uint8_t* img2, int32_t batch,
                              int32_t width, int32_t height, int32_t subpel, int32_t* proposal, float* flow_out,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

/* One training step.  labels: device int32, batch x ceil(height/8) x
 * ceil(width/8) packed flows in 1/subpel px, FF_EMPTY where unlabelled.
 * Loss = mean over labelled points of |out_x - t_x| + |out_y - t_y| with t
 * the label in px / 32.  Gradients of the stored activations are rounded to
 * bf16; weight gradients are summed in a fixed order (run to run identical).
 * With adam_m and adam_v (device float32, param count each, zero at step 1)
 * params get one Adam update (beta 0.9 / 0.999, eps 1e-8, bias-corrected by
 * step >= 1, rate lr); with both null params are left unchanged.
 * grad_out (device float32[param count], nullable): the gradient;
 * loss_out (device float32[1], nullable): the loss before the update. */
ff_status ff_proposal_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                                 const uint8_t* img1, const uint8_t* img2, const int32_t* labels, int32_t batch,
                                 int32_t width, int32_t height, int32_t subpel, float* grad_out, float* loss_out,
                                 void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Section 3.3, the second data term: patch-based SIFT flow.  Every pixel of
 * both images gets a 128-dimensional SIFT vector (Lowe 2004, computed densely
 * and upright as in Liu et al.'s SIFT flow), PCA over the pair reduces them
 * to S "colours", the colour images are smoothed per level as the images of
 * section 3.2, and the data term sums L2 colour distances over the subsampled
 * patch.  The kd-tree seeds still come from the CIELab WHT vectors.
 *
 * Dense SIFT (the readings the library takes where the paper defers to SIFT
 * flow): input the 8-bit CIELab lightness (plane 0 of a descriptor blob's
 * lab planes, or a gray image); central-difference gradients with clamped
 * coordinates; orientation bins o pi/4 (o = 0..7, y down), the magnitude
 * split linearly between the two nearest; 4 x 4 cells of 3 px, cell (i, j)
 * centred at p + ((i - 1.5) 3, (j - 1.5) 3); every pixel q = p + d with
 * |dx|, |dy| <= 7 inside the image adds with weight exp(-|d|^2 / 72) times the
 * bilinear cell weights; element (4 j + i) 8 + o; normalised, clamped at 0.2,
 * normalised (a zero vector stays zero).  fp32 arithmetic.
 */

/* int16 values per pixel of a colour-level array with S colours (S rounded
 * up to a multiple of 4; the extra channels are zero); 0 if S is not in 1..32. */
int32_t ff_sift_pitch(int32_t S);

/* Device workspace bytes that ff_dense_sift, ff_sift_colors (for a pair of
 * these sizes) and ff_sift_levels (for either image) each need; 0 for sizes
 * below 1, above 8191 or above 2^22 pixels. */
size_t ff_sift_workspace_bytes(int32_t w1, int32_t h1, int32_t w2, int32_t h2);

/* Inspection: the dense SIFT vectors of one lightness plane L (device, h*w
 * uint8, rows packed) into desc (device, h*w*128 float32). */
ff_status ff_dense_sift(const uint8_t* L, int32_t width, int32_t height, float* desc, void* workspace,
                        size_t workspace_bytes, hipStream_t stream);

/*
 * The colours of a pair.  L1, L2: device lightness planes (h*w uint8 each).
 * The covariance of the two images' SIFT vectors together (every pixel of
 * both; accumulated in fp64) is decomposed by a Jacobi eigen-solver (fp64);
 * eigenvalues are sorted descending (ties by index) and each eigenvector's
 * largest-magnitude component (the first on ties) is made positive.  codes1 /
 * codes2 (device, h*w*S int16, colours last): the projections on the first S
 * eigenvectors of the vectors minus the mean, round-half-even(1024 c),
 * clamped to +-2047.  S in 1..32.
 *  pca (device, nullable): 128 + 128 + 128*128 doubles: the mean, the
 *      eigenvalues (descending), the basis, element [k*128 + s] = component k
 *      of eigenvector s;
 *  desc1, desc2 (device, nullable): the SIFT vectors, h*w*128 float32 each.
 * Errors: FF_ERR_ARG for null pointers, sizes below 1 or S outside 1..32;
 * FF_ERR_SIZE beyond 8191 per side or 2^22 pixels; FF_ERR_WORKSPACE below
 * ff_sift_workspace_bytes.
 */
ff_status ff_sift_colors(const uint8_t* L1, int32_t w1, int32_t h1, const uint8_t* L2, int32_t w2, int32_t h2,
                         int32_t S, int16_t* codes1, int16_t* codes2, double* pca, float* desc1, float* desc2,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Per-level colour images of one image: levels (device, (k+1) x h x w x
 * ff_sift_pitch(S) int16): level j is the codes smoothed with n = 2^j as in
 * section 3.2 (n x n block sums, replicate-padded; the two Q14 Lanczos-3
 * passes of ff_compute_descriptors; output in code units, rounded half up);
 * level 0 is the codes.  codes: device h*w*S int16.  k in 0..4. */
ff_status ff_sift_levels(const int16_t* codes, int32_t width, int32_t height, int32_t S, int32_t k, int16_t* levels,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Only the Lab8 planes and WHT vectors of ff_compute_descriptors (all the
 * SIFT-flow search reads of a descriptor blob); the other regions of blob are
 * left as they are. */
ff_status ff_compute_lab_wht(const ff_desc* d, const ff_image* img, const uint8_t* pixels, void* blob,
                             size_t blob_bytes, hipStream_t stream);

/* The rest of ff_compute_descriptors (sections 3.2, 3.3): the smoothed levels
 * I^n and the census planes of every level and phase, both layouts, from the
 * Lab8 planes that ff_compute_lab_wht wrote into the same blob (queued before
 * it on the same stream, or waited for).  ff_compute_lab_wht followed by
 * ff_compute_census fills the blob exactly as ff_compute_descriptors does. */
ff_status ff_compute_census(const ff_desc* d, void* blob, size_t blob_bytes, hipStream_t stream);

/*
 * Flow Fields with the SIFT-flow data term (sections 3.1-3.3), a batch of
 * fields in one call; the search is ff_match_field's (kd-tree seeds on the
 * 2^k grid, per level four propagation sweeps and three random searches,
 * R_n = R n) with E^n_r(p, f) = sum over the (2r+1)^2 samples at stride n of
 * floor(sqrt(sum_{s < S} d_s^2 * 256 / Q^4)): d_s = Q^2 c1_s(p + n delta) - the
 * target colour bilinear at the subpixel centre (weights (Q-a)(Q-b), a(Q-b),
 * (Q-a)b, ab of the four neighbours of floor(m/Q) + n delta, the +1
 * neighbours clamped; m = pQ + f, (a, b) = m mod Q); lookups clamp to the
 * image; f counts only if m lies in the image.  Costs are exact integers.
 * The paper's KITTI setting: r = 3 with S = 12 for F and B1, r2 = 2 with
 * S2 = 18 for B2.  p->use_kdtree must be 1 (FF_ERR_UNSUPPORTED otherwise);
 * p->band_rows and p->pipeline are ignored; all jobs share subpel.
 */
typedef struct {
  const ff_desc* src;        /* host: dimensions, subpel, WHT layout */
  const void* src_blob;      /* device: holds the WHT vectors of `radius` */
  const ff_desc* dst;        /* host */
  const void* dst_blob;      /* device */
  const int16_t* src_levels; /* device: ff_sift_levels of the source */
  const int16_t* dst_levels; /* device: ff_sift_levels of the target */
  int32_t pitch;             /* int16 per pixel of both level arrays (4..32, multiple of 4) */
  int32_t channels;          /* S: colours used, 1..pitch */
  int32_t levels;            /* k of both level arrays (>= p->k) */
  int32_t radius;
  uint32_t field_id, pair_id;
  uint64_t seed;
  int32_t* flow;             /* device, src h*w */
  int32_t* cost;             /* device, src h*w */
} ff_sift_job;

size_t ff_match_sift_workspace_bytes(const ff_sift_job* jobs, int32_t n_jobs, const ff_match_params* p);
ff_status ff_match_sift(const ff_sift_job* jobs, int32_t n_jobs, const ff_match_params* p, void* workspace,
                        size_t workspace_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as ff_match_field, with the same arguments minus the workspace, and
 * identical outputs.  Its scratch (what ff_match_field keeps in the
 * workspace) is one static device array of FF_NOALLOC_SCRATCH_BYTES per GPU,
 * held until the process ends; the call allocates nothing (no hipMalloc, no
 * host heap).  ff_init() looks the array up on the current device; call it
 * before the first use inside a capture.
 *  - Limit: FF_ERR_SIZE if ff_match_workspace_bytes() of the same arguments
 *    exceeds FF_NOALLOC_SCRATCH_BYTES (64 MiB: fields of up to about 1.7 Mpx
 *    at k = 3 and leaf 8, e.g. 1024x436, 1242x375, 1280x720, 1600x1000; not
 *    1920x1080).  Checked before anything is enqueued.
 *  - Every call on one GPU uses that GPU's single array and the array keeps
 *    the last call's contents (each call clears what it needs).  Calls that
 *    overlap on one GPU (from other streams or host threads) race and give
 *    wrong results: serialise them on one stream.
 *  - status: nullable device int32; after the call's work it receives the
 *    device status word (FF_OK, or FF_ERR_DEVICE if a watchdog fired) -- what
 *    ff_read_status reports for a workspace.
 */
#define FF_NOALLOC_SCRATCH_BYTES (64u << 20)
ff_status ff_match_field_noalloc(const ff_desc* src, const void* src_blob, const ff_desc* dst, const void* dst_blob,
                                 int32_t radius, const ff_match_params* p, const int32_t* proposal, int32_t* flow,
                                 int32_t* cost, int32_t* status, hipStream_t stream);

/* After the stream has finished: read the device status word a match call
 * left in its workspace (FF_OK, or FF_ERR_DEVICE if a watchdog fired). */
ff_status ff_read_status(const void* workspace, int32_t* status_host);

const char* ff_status_string(ff_status s);

/*
 * Profiling hook (measurement only; not used on the search path).  Arm one
 * kernel class: every later launch of it (for the multi-kernel classes, every
 * launch sequence) is bracketed by two HIP events recorded on the stream it
 * runs on, for up to max_launches launches.  ff_profile_begin creates the
 * events (host allocation: call it outside any capture or timed loop);
 * ff_profile_end waits for them, returns the summed elapsed milliseconds and
 * the number of launches, destroys the events and disarms the hook.
 * Errors: FF_ERR_ARG for a class outside 1..15, max_launches outside
 * 1..2^20 or null outputs; FF_ERR_HIP if creating, recording, waiting for or
 * timing an event failed (ff_profile_end still disarms the hook).
 */
typedef enum {
  FF_PROF_DESCRIPTORS = 1,   /* the whole ff_compute_descriptors sequence */
  FF_PROF_TREE = 2,          /* the kd-tree build sequence of a match */
  FF_PROF_SEED = 3,
  FF_PROF_LEVEL_ENTRY = 4,
  FF_PROF_PROPAGATE = 5,     /* one propagation sweep kernel */
  FF_PROF_RANDOM_SEARCH = 6,
  FF_PROF_FILTER = 7,
  FF_PROF_PROPOSAL = 8,      /* the whole ff_proposal_forward sequence */
  FF_PROF_TRAIN = 9,         /* the whole ff_proposal_train_step sequence */
  FF_PROF_REGION = 10,       /* the whole ff_region_filter sequence */
  FF_PROF_SPARSIFY = 11,     /* ff_sparsify */
  FF_PROF_LAB = 12,          /* descriptor stages: Lab8 */
  FF_PROF_SMOOTH = 13,       /*   smoothed images I^n (all levels) */
  FF_PROF_CENSUS = 14,       /*   census planes (all levels and phases, both layouts) */
  FF_PROF_WHT = 15,          /*   WHT vectors (all radii) */
  FF_PROF_SIFT_COLORS = 16,  /* the whole ff_sift_colors (or ff_dense_sift) sequence */
  FF_PROF_SIFT_PCA = 17,     /*   its covariance and eigen-decomposition */
  FF_PROF_SIFT_LEVELS = 18,  /* ff_sift_levels */
  FF_PROF_SIFT_MATCH = 19,   /* the whole ff_match_sift_batch sequence */
  FF_PROF_SIFT_PROPAGATE = 20 /*   one of its propagation sweeps */
} ff_prof_class;
ff_status ff_profile_begin(int32_t kernel_class, int32_t max_launches);
ff_status ff_profile_end(double* total_ms, int32_t* launches);
/* The same, also writing the first max_each launches' durations (ms, host
 * array, in the order the launches were issued) to each_ms. */
ff_status ff_profile_end_each(double* total_ms, int32_t* launches, double* each_ms, int32_t max_each);

/*
 * Dependent-load latency probe (measurement only; not used on the search
 * path).  A propagation sweep is a chain of wavefront steps, each step's
 * result deciding the next step's target addresses (Eq. 2 in raster order,
 * section 3.2), so one dependent memory round trip per step is a floor on
 * its time.  This call measures that round trip: one wavefront follows next[]
 * from index 0 for `warm` hops (bringing the cycle into the caches), then
 * for `hops` more, timed with the 100 MHz real-time counter.  Every hop is
 * one global load whose address is the previous load's value masked to
 * [0, n), so it costs one round trip to where the cycle's lines live: the
 * vector L1 for a cycle of a few KB, the L2 for one of a few MB.
 * next: device, n int32 (n a power of two), filled by the caller with a
 * cycle through index 0.  out: device, 2 int64: the timed walk's ticks
 * (10 ns each) and the final index.  Errors (nothing enqueued): FF_ERR_ARG
 * for null pointers, n outside [2, 2^28] or not a power of two, hops outside
 * [1, 2^22], warm outside [0, 2^22] (a walk stays within a few seconds even
 * if every hop goes to HBM).
 */
ff_status ff_probe_load_latency(const int32_t* next, int32_t n, int32_t warm, int32_t hops, int64_t* out,
                                hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FF_H_ */
