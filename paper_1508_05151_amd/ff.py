"""Python binding of libff (ctypes).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and streams.  If the
library is not built the import fails loudly -- there is no fallback.

Names follow the C ABI in include/ff.h.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libff.so")

FF_EMPTY = -2147450880
FF_COST_INF = 2147483647
MAX_RADII = 4

STATUS = {0: "FF_OK", -1: "FF_ERR_ARG", -2: "FF_ERR_SIZE", -3: "FF_ERR_WORKSPACE", -4: "FF_ERR_UNSUPPORTED",
          -5: "FF_ERR_HIP", -6: "FF_ERR_DEVICE"}


class FFError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class ff_image(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("channels", C.c_int32), ("row_stride", C.c_int32)]


class ff_desc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("channels", C.c_int32), ("k", C.c_int32),
                ("subpel", C.c_int32), ("n_radii", C.c_int32), ("radii", C.c_int32 * MAX_RADII),
                ("wht_dims", C.c_int32), ("wht_stride", C.c_int32), ("off_lab", C.c_size_t),
                ("off_smooth", C.c_size_t), ("off_census", C.c_size_t), ("off_census_t", C.c_size_t),
                ("off_wht", C.c_size_t),
                ("plane_bytes", C.c_size_t), ("bytes", C.c_size_t)]


class ff_match_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("R", C.c_int32), ("leaf", C.c_int32), ("n_prop", C.c_int32),
                ("n_rs", C.c_int32), ("use_kdtree", C.c_int32), ("max_steps", C.c_int32),
                ("field_id", C.c_uint32), ("pair_id", C.c_uint32), ("band_rows", C.c_int32),
                ("pipeline", C.c_int32), ("watchdog_us", C.c_int32), ("seed", C.c_uint64)]


class ff_field_job(C.Structure):
    _fields_ = [("src", C.POINTER(ff_desc)), ("src_blob", C.c_void_p), ("dst", C.POINTER(ff_desc)),
                ("dst_blob", C.c_void_p), ("radius", C.c_int32), ("field_id", C.c_uint32), ("pair_id", C.c_uint32),
                ("reserved", C.c_uint32), ("seed", C.c_uint64), ("proposal", C.c_void_p), ("flow", C.c_void_p),
                ("cost", C.c_void_p)]


_lib = None


class ff_sift_job(C.Structure):
    _fields_ = [("src", C.POINTER(ff_desc)), ("src_blob", C.c_void_p), ("dst", C.POINTER(ff_desc)),
                ("dst_blob", C.c_void_p), ("src_levels", C.c_void_p), ("dst_levels", C.c_void_p),
                ("pitch", C.c_int32), ("channels", C.c_int32), ("levels", C.c_int32), ("radius", C.c_int32),
                ("field_id", C.c_uint32), ("pair_id", C.c_uint32), ("seed", C.c_uint64),
                ("flow", C.c_void_p), ("cost", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (the GPU path has no fallback)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32 = C.c_int32
        L.ff_init.restype = i32
        L.ff_default_params.argtypes = [C.POINTER(ff_match_params)]
        L.ff_default_params.restype = None
        L.ff_desc_init.argtypes = [C.POINTER(ff_desc), C.POINTER(ff_image), i32, i32, P, i32]
        L.ff_desc_init.restype = i32
        L.ff_compute_descriptors.argtypes = [C.POINTER(ff_desc), C.POINTER(ff_image), P, P, C.c_size_t, P]
        L.ff_compute_descriptors.restype = i32
        L.ff_match_workspace_bytes.argtypes = [C.POINTER(ff_desc), C.POINTER(ff_desc), i32,
                                               C.POINTER(ff_match_params)]
        L.ff_match_workspace_bytes.restype = C.c_size_t
        L.ff_match_field.argtypes = [C.POINTER(ff_desc), P, C.POINTER(ff_desc), P, i32, C.POINTER(ff_match_params),
                                     P, P, P, P, C.c_size_t, P]
        L.ff_match_field.restype = i32
        L.ff_match_batch_workspace_bytes.argtypes = [C.POINTER(ff_field_job), i32, C.POINTER(ff_match_params)]
        L.ff_match_batch_workspace_bytes.restype = C.c_size_t
        L.ff_match_batch.argtypes = [C.POINTER(ff_field_job), i32, C.POINTER(ff_match_params), P, C.c_size_t, P]
        L.ff_match_batch.restype = i32
        L.ff_profile_begin.argtypes = [i32, i32]
        L.ff_profile_begin.restype = i32
        L.ff_profile_end.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.ff_profile_end.restype = i32
        L.ff_profile_end_each.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32), P, i32]
        L.ff_profile_end_each.restype = i32
        L.ff_probe_load_latency.argtypes = [P, i32, i32, i32, P, P]
        L.ff_probe_load_latency.restype = i32
        L.ff_consistency_filter.argtypes = [P, i32, i32, P, i32, i32, i32, i32, i32, P, P, P]
        L.ff_consistency_filter.restype = i32
        L.ff_region_filter_workspace_bytes.argtypes = [i32, i32]
        L.ff_region_filter_workspace_bytes.restype = C.c_size_t
        L.ff_region_filter.argtypes = [P, P, i32, i32, i32, i32, P, P, P, P, C.c_size_t, P]
        L.ff_region_filter.restype = i32
        L.ff_sparsify.argtypes = [P, i32, i32, P, i32, i32, i32, i32, i32, P, P, P]
        L.ff_sparsify.restype = i32
        L.ff_tree_nodes.argtypes = [i32, i32]
        L.ff_tree_nodes.restype = i32
        L.ff_build_kdtree.argtypes = [C.POINTER(ff_desc), P, i32, i32, P, P, P, P, C.c_size_t, P]
        L.ff_build_kdtree.restype = i32
        L.ff_match_field_noalloc.argtypes = [C.POINTER(ff_desc), P, C.POINTER(ff_desc), P, i32,
                                             C.POINTER(ff_match_params), P, P, P, P, P]
        L.ff_match_field_noalloc.restype = i32
        L.ff_read_status.argtypes = [P, C.POINTER(C.c_int32)]
        L.ff_read_status.restype = i32
        L.ff_status_string.argtypes = [i32]
        L.ff_status_string.restype = C.c_char_p
        L.ff_net_param_count.argtypes = []
        L.ff_net_param_count.restype = i32
        L.ff_net_workspace_bytes.argtypes = [i32, i32, i32]
        L.ff_net_workspace_bytes.restype = C.c_size_t
        L.ff_proposal_forward.argtypes = [P, P, P, i32, i32, i32, i32, P, P, P, C.c_size_t, P]
        L.ff_proposal_forward.restype = i32
        L.ff_proposal_train_step.argtypes = [P, P, P, i32, C.c_float, P, P, P, i32, i32, i32, i32, P, P, P,
                                             C.c_size_t, P]
        L.ff_proposal_train_step.restype = i32
        L.ff_sift_pitch.argtypes = [i32]
        L.ff_sift_pitch.restype = i32
        L.ff_sift_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.ff_sift_workspace_bytes.restype = C.c_size_t
        L.ff_dense_sift.argtypes = [P, i32, i32, P, P, C.c_size_t, P]
        L.ff_dense_sift.restype = i32
        L.ff_sift_colors.argtypes = [P, i32, i32, P, i32, i32, i32, P, P, P, P, P, P, C.c_size_t, P]
        L.ff_sift_colors.restype = i32
        L.ff_sift_levels.argtypes = [P, i32, i32, i32, i32, P, P, C.c_size_t, P]
        L.ff_sift_levels.restype = i32
        L.ff_compute_lab_wht.argtypes = [C.POINTER(ff_desc), C.POINTER(ff_image), P, P, C.c_size_t, P]
        L.ff_compute_lab_wht.restype = i32
        L.ff_compute_census.argtypes = [C.POINTER(ff_desc), P, C.c_size_t, P]
        L.ff_compute_census.restype = i32
        L.ff_match_field_tree.argtypes = [C.POINTER(ff_desc), P, C.POINTER(ff_desc), P, i32,
                                          C.POINTER(ff_match_params), P, C.c_size_t, P]
        L.ff_match_field_tree.restype = i32
        L.ff_match_sift_workspace_bytes.argtypes = [C.POINTER(ff_sift_job), i32, C.POINTER(ff_match_params)]
        L.ff_match_sift_workspace_bytes.restype = C.c_size_t
        L.ff_match_sift.argtypes = [C.POINTER(ff_sift_job), i32, C.POINTER(ff_match_params), P, C.c_size_t, P]
        L.ff_match_sift.restype = i32
        _lib = L
    return _lib


def _check(code, what):
    if code != 0:
        raise FFError(code, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ C ABI
def ff_init():
    _check(lib().ff_init(), "ff_init")


def ff_default_params(**overrides) -> ff_match_params:
    p = ff_match_params()
    lib().ff_default_params(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def ff_desc_init(width, height, channels=3, k=3, subpel=4, radii=(8, 6)) -> ff_desc:
    d = ff_desc()
    img = ff_image(width, height, channels, width * channels)
    r = (C.c_int32 * MAX_RADII)(*radii)
    _check(lib().ff_desc_init(C.byref(d), C.byref(img), k, subpel, C.cast(r, C.c_void_p), len(radii)),
           "ff_desc_init")
    return d


def ff_compute_descriptors(d: ff_desc, pixels: torch.Tensor, blob: torch.Tensor, stream=None):
    """pixels: H x W x C uint8 device tensor (contiguous); blob: d.bytes
    device bytes (uint8 tensor)."""
    assert pixels.is_cuda and pixels.dtype == torch.uint8 and pixels.is_contiguous()
    H, W = pixels.shape[:2]
    Cc = 1 if pixels.dim() == 2 else pixels.shape[2]
    img = ff_image(W, H, Cc, W * Cc)
    _check(lib().ff_compute_descriptors(C.byref(d), C.byref(img), _ptr(pixels), _ptr(blob), blob.numel(),
                                        _stream(stream)), "ff_compute_descriptors")


def ff_match_workspace_bytes(src: ff_desc, dst: ff_desc, radius: int, p: ff_match_params) -> int:
    n = lib().ff_match_workspace_bytes(C.byref(src), C.byref(dst), radius, C.byref(p))
    if n == 0:
        raise FFError(-1, "ff_match_workspace_bytes")
    return n


def _check_i32(t, numel, what):
    """A buffer handed to the library as a plain pointer: it must be a
    contiguous int32 device tensor of exactly `numel` elements (the kernels
    index it by the image or grid size and cannot check it themselves)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_contiguous():
        raise FFError(-1, f"{what}: expected a contiguous int32 tensor")
    if t.numel() != numel:
        raise FFError(-1, f"{what}: {t.numel()} elements, the call needs {numel}")
    if not t.is_cuda:
        raise FFError(-1, f"{what}: expected a device (CUDA) tensor")


def check_proposal(proposal, src: ff_desc, k: int):
    """A proposal holds one packed flow per point of the coarsest grid of a
    k-level match over src: ceil(H / 2^k) x ceil(W / 2^k)."""
    if proposal is None:
        return
    hc, wc = seed_grid(src.width, src.height, k)
    if isinstance(proposal, torch.Tensor) and proposal.dim() >= 2 and tuple(proposal.shape[-2:]) != (hc, wc):
        raise FFError(-1, f"proposal: shape {tuple(proposal.shape)}, the seed grid is {(hc, wc)}")
    _check_i32(proposal, hc * wc, "proposal")


def ff_match_field(src: ff_desc, src_blob, dst: ff_desc, dst_blob, radius: int, p: ff_match_params, proposal,
                   flow, cost, workspace, stream=None):
    check_proposal(proposal, src, p.k)
    _check_i32(flow, src.width * src.height, "flow")
    _check_i32(cost, src.width * src.height, "cost")
    _check(lib().ff_match_field(C.byref(src), _ptr(src_blob), C.byref(dst), _ptr(dst_blob), radius, C.byref(p),
                                _ptr(proposal), _ptr(flow), _ptr(cost), _ptr(workspace), workspace.numel(),
                                _stream(stream)), "ff_match_field")


def ff_match_field_tree(src: ff_desc, src_blob, dst: ff_desc, dst_blob, radius: int, p: ff_match_params, workspace,
                        stream=None):
    """The kd-tree of a later ff_match_field call (same arguments and
    workspace, p.use_kdtree = 2 there) built ahead of it."""
    _check(lib().ff_match_field_tree(C.byref(src), _ptr(src_blob), C.byref(dst), _ptr(dst_blob), radius, C.byref(p),
                                     _ptr(workspace), workspace.numel(), _stream(stream)), "ff_match_field_tree")


NOALLOC_SCRATCH_BYTES = 64 << 20


def ff_match_field_noalloc(src: ff_desc, src_blob, dst: ff_desc, dst_blob, radius: int, p: ff_match_params,
                           proposal, flow, cost, status=None, stream=None):
    """ff_match_field without a workspace: the library's static per-device
    scratch serves it (calls on one GPU must not overlap)."""
    check_proposal(proposal, src, p.k)
    _check_i32(flow, src.width * src.height, "flow")
    _check_i32(cost, src.width * src.height, "cost")
    if status is not None:
        _check_i32(status, 1, "status")
    _check(lib().ff_match_field_noalloc(C.byref(src), _ptr(src_blob), C.byref(dst), _ptr(dst_blob), radius,
                                        C.byref(p), _ptr(proposal), _ptr(flow), _ptr(cost), _ptr(status),
                                        _stream(stream)), "ff_match_field_noalloc")


def make_job(src: ff_desc, src_blob, dst: ff_desc, dst_blob, radius, flow, cost, field_id=0, pair_id=0, seed=0,
             proposal=None, k=3) -> ff_field_job:
    """One field of a batched call; k is the batch's hierarchy depth (the
    proposal must cover its seed grid)."""
    check_proposal(proposal, src, k)
    _check_i32(flow, src.width * src.height, "flow")
    _check_i32(cost, src.width * src.height, "cost")
    j = ff_field_job()
    j.src = C.pointer(src)
    j.src_blob = src_blob.data_ptr()
    j.dst = C.pointer(dst)
    j.dst_blob = dst_blob.data_ptr()
    j.radius = radius
    j.field_id = field_id
    j.pair_id = pair_id
    j.seed = seed
    j.proposal = None if proposal is None else proposal.data_ptr()
    j.flow = flow.data_ptr()
    j.cost = cost.data_ptr()
    return j


def ff_match_batch_workspace_bytes(jobs, p: ff_match_params) -> int:
    arr = (ff_field_job * len(jobs))(*jobs)
    n = lib().ff_match_batch_workspace_bytes(arr, len(jobs), C.byref(p))
    if n == 0:
        raise FFError(-1, "ff_match_batch_workspace_bytes")
    return n


def ff_match_batch(jobs, p: ff_match_params, workspace, stream=None):
    arr = (ff_field_job * len(jobs))(*jobs)
    _check(lib().ff_match_batch(arr, len(jobs), C.byref(p), _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_match_batch")


def ff_consistency_filter(flow_fwd, flows_bwd, subpel, eps_q, keep, flow_filtered, stream=None):
    h1, w1 = flow_fwd.shape
    h2, w2 = flows_bwd[0].shape
    arr = (C.c_void_p * len(flows_bwd))(*[b.data_ptr() for b in flows_bwd])
    _check(lib().ff_consistency_filter(_ptr(flow_fwd), w1, h1, C.cast(arr, C.c_void_p), len(flows_bwd), w2, h2,
                                       subpel, eps_q, _ptr(keep), _ptr(flow_filtered), _stream(stream)),
           "ff_consistency_filter")


def ff_region_filter_workspace_bytes(width, height) -> int:
    n = lib().ff_region_filter_workspace_bytes(width, height)
    if n == 0:
        raise FFError(-1, "ff_region_filter_workspace_bytes")
    return n


def ff_region_filter(flow, keep, subpel, min_region, keep_out, flow_out, workspace, label=None, stream=None):
    """Section 3.4's region filter after the consistency check: flow is the
    field before the check, keep the check's mask (H x W tensors)."""
    h, w = flow.shape
    _check_i32(flow, w * h, "flow")
    _check_i32(flow_out, w * h, "flow_out")
    if label is not None:
        _check_i32(label, w * h, "label")
    for t, what in ((keep, "keep"), (keep_out, "keep_out")):
        if t.dtype != torch.uint8 or not t.is_contiguous() or t.numel() != w * h or not t.is_cuda:
            raise FFError(-1, f"{what}: expected a contiguous uint8 CUDA tensor of {w * h} elements")
    _check(lib().ff_region_filter(_ptr(flow), _ptr(keep), w, h, subpel, min_region, _ptr(label), _ptr(keep_out),
                                  _ptr(flow_out), _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_region_filter")


def ff_sparsify(flow, flows_bwd, subpel, min_samples, pick, flow_sparse=None, stream=None):
    """Section 3.5's sparsification: flow is the outlier-filtered field,
    pick the ceil(H/3) x ceil(W/3) int32 output."""
    h1, w1 = flow.shape
    h2, w2 = flows_bwd[0].shape
    _check_i32(flow, w1 * h1, "flow")
    for b in flows_bwd:
        _check_i32(b, w2 * h2, "flow_bwd")
    _check_i32(pick, ((h1 + 2) // 3) * ((w1 + 2) // 3), "pick")
    if flow_sparse is not None:
        _check_i32(flow_sparse, w1 * h1, "flow_sparse")
    arr = (C.c_void_p * len(flows_bwd))(*[b.data_ptr() for b in flows_bwd])
    _check(lib().ff_sparsify(_ptr(flow), w1, h1, C.cast(arr, C.c_void_p), len(flows_bwd), w2, h2, subpel,
                             min_samples, _ptr(pick), _ptr(flow_sparse), _stream(stream)), "ff_sparsify")


def ff_tree_nodes(n_points: int, leaf: int) -> int:
    return lib().ff_tree_nodes(n_points, leaf)


def ff_build_kdtree(d: ff_desc, blob, radius, leaf, node_dim, node_split, perm, workspace, stream=None):
    _check(lib().ff_build_kdtree(C.byref(d), _ptr(blob), radius, leaf, _ptr(node_dim), _ptr(node_split), _ptr(perm),
                                 _ptr(workspace), workspace.numel(), _stream(stream)), "ff_build_kdtree")


PROF = {"descriptors": 1, "tree": 2, "seed": 3, "level_entry": 4, "propagate": 5, "random_search": 6, "filter": 7,
        "proposal": 8, "train": 9, "region": 10, "sparsify": 11, "lab": 12, "smooth": 13, "census": 14, "wht": 15,
        "sift_colors": 16, "sift_pca": 17, "sift_levels": 18, "sift_match": 19, "sift_propagate": 20}


def ff_profile_begin(kernel_class: str, max_launches: int):
    _check(lib().ff_profile_begin(PROF[kernel_class], max_launches), "ff_profile_begin")


def ff_profile_end(each: int = 0):
    """Returns (total ms, launches, per-launch ms of the first `each`)."""
    tot = C.c_double(0)
    n = C.c_int32(0)
    buf = (C.c_double * max(each, 1))()
    _check(lib().ff_profile_end_each(C.byref(tot), C.byref(n), C.cast(buf, C.c_void_p) if each else None, each),
           "ff_profile_end")
    return tot.value, n.value, [buf[i] for i in range(min(each, n.value))]


def ff_probe_load_latency(nxt, warm: int, hops: int, out, stream=None):
    """One thread walks the cycle nxt (contiguous int32 device tensor, a
    power-of-two length) for `warm` hops, then times `hops` more; out (int64
    device tensor of 2) receives the timed walk's 10 ns ticks and the final
    index."""
    if not isinstance(nxt, torch.Tensor) or nxt.dtype != torch.int32 or not nxt.is_contiguous() or not nxt.is_cuda:
        raise FFError(-1, "ff_probe_load_latency: expected a contiguous int32 device tensor")
    if not isinstance(out, torch.Tensor) or out.dtype != torch.int64 or out.numel() != 2 or not out.is_cuda:
        raise FFError(-1, "ff_probe_load_latency: out must be 2 int64 on the device")
    _check(lib().ff_probe_load_latency(_ptr(nxt), nxt.numel(), warm, hops, _ptr(out), _stream(stream)),
           "ff_probe_load_latency")


def load_cycle(n_ints: int, line_ints: int = 32, seed: int = 0):
    """A cycle through index 0 that visits the first word of every
    `line_ints`-word line of an n_ints buffer once, in a seeded random order
    (host NumPy array), for ff_probe_load_latency."""
    import numpy as np
    lines = n_ints // line_ints
    order = np.random.default_rng(seed).permutation(lines)
    order = np.concatenate([[0], order[order != 0]])
    nxt = np.zeros(n_ints, dtype=np.int32)
    nxt[order * line_ints] = np.roll(order, -1) * line_ints
    return nxt


def ff_read_status(workspace) -> int:
    s = C.c_int32(0)
    _check(lib().ff_read_status(_ptr(workspace), C.byref(s)), "ff_read_status")
    return s.value


# ------------------------------------------------------------------ SIFT-flow data term (section 3.3)
SIFT_DIM = 128


def ff_sift_pitch(S: int) -> int:
    return lib().ff_sift_pitch(S)


def ff_sift_workspace_bytes(w1, h1, w2, h2) -> int:
    n = lib().ff_sift_workspace_bytes(w1, h1, w2, h2)
    if n == 0:
        raise FFError(-1, "ff_sift_workspace_bytes")
    return n


def _check_dev(t, dtype, numel, what):
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel or not t.is_cuda:
        raise FFError(-1, f"{what}: expected a contiguous {dtype} CUDA tensor of {numel} elements")


def ff_dense_sift(L, desc, workspace, stream=None):
    """L: H x W uint8 lightness plane; desc: H x W x 128 float32."""
    h, w = L.shape
    _check_dev(L, torch.uint8, w * h, "L")
    _check_dev(desc, torch.float32, w * h * SIFT_DIM, "desc")
    _check(lib().ff_dense_sift(_ptr(L), w, h, _ptr(desc), _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_dense_sift")


def ff_sift_colors(L1, L2, S, codes1, codes2, workspace, pca=None, desc1=None, desc2=None, stream=None):
    """L1, L2: lightness planes; codes: H x W x S int16 each; pca (optional):
    128 + 128 + 128 * 128 float64 (mean, eigenvalues, basis)."""
    h1, w1 = L1.shape
    h2, w2 = L2.shape
    _check_dev(L1, torch.uint8, w1 * h1, "L1")
    _check_dev(L2, torch.uint8, w2 * h2, "L2")
    _check_dev(codes1, torch.int16, w1 * h1 * S, "codes1")
    _check_dev(codes2, torch.int16, w2 * h2 * S, "codes2")
    if pca is not None:
        _check_dev(pca, torch.float64, 2 * SIFT_DIM + SIFT_DIM * SIFT_DIM, "pca")
    if desc1 is not None:
        _check_dev(desc1, torch.float32, w1 * h1 * SIFT_DIM, "desc1")
    if desc2 is not None:
        _check_dev(desc2, torch.float32, w2 * h2 * SIFT_DIM, "desc2")
    _check(lib().ff_sift_colors(_ptr(L1), w1, h1, _ptr(L2), w2, h2, S, _ptr(codes1), _ptr(codes2), _ptr(pca),
                                _ptr(desc1), _ptr(desc2), _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_sift_colors")


def ff_sift_levels(codes, k, levels, workspace, stream=None):
    """codes: H x W x S int16; levels: (k+1) x H x W x ff_sift_pitch(S) int16."""
    h, w, S = codes.shape
    _check_dev(codes, torch.int16, w * h * S, "codes")
    _check_dev(levels, torch.int16, (k + 1) * w * h * ff_sift_pitch(S), "levels")
    _check(lib().ff_sift_levels(_ptr(codes), w, h, S, k, _ptr(levels), _ptr(workspace), workspace.numel(),
                                _stream(stream)), "ff_sift_levels")


def ff_compute_lab_wht(d: ff_desc, pixels: torch.Tensor, blob: torch.Tensor, stream=None):
    assert pixels.is_cuda and pixels.dtype == torch.uint8 and pixels.is_contiguous()
    H, W = pixels.shape[:2]
    Cc = 1 if pixels.dim() == 2 else pixels.shape[2]
    img = ff_image(W, H, Cc, W * Cc)
    _check(lib().ff_compute_lab_wht(C.byref(d), C.byref(img), _ptr(pixels), _ptr(blob), blob.numel(),
                                    _stream(stream)), "ff_compute_lab_wht")


def ff_compute_census(d: ff_desc, blob: torch.Tensor, stream=None):
    """Smoothed levels and census planes from the blob's Lab8 planes."""
    _check(lib().ff_compute_census(C.byref(d), _ptr(blob), blob.numel(), _stream(stream)), "ff_compute_census")


def make_sift_job(src: ff_desc, src_blob, dst: ff_desc, dst_blob, src_levels, dst_levels, S, levels_k, radius,
                  flow, cost, field_id=0, pair_id=0, seed=0) -> ff_sift_job:
    _check_i32(flow, src.width * src.height, "flow")
    _check_i32(cost, src.width * src.height, "cost")
    P = src_levels.shape[-1]
    j = ff_sift_job()
    j.src = C.pointer(src)
    j.src_blob = src_blob.data_ptr()
    j.dst = C.pointer(dst)
    j.dst_blob = dst_blob.data_ptr()
    j.src_levels = src_levels.data_ptr()
    j.dst_levels = dst_levels.data_ptr()
    j.pitch = P
    j.channels = S
    j.levels = levels_k
    j.radius = radius
    j.field_id = field_id
    j.pair_id = pair_id
    j.seed = seed
    j.flow = flow.data_ptr()
    j.cost = cost.data_ptr()
    return j


def ff_match_sift_workspace_bytes(jobs, p: ff_match_params) -> int:
    arr = (ff_sift_job * len(jobs))(*jobs)
    n = lib().ff_match_sift_workspace_bytes(arr, len(jobs), C.byref(p))
    if n == 0:
        raise FFError(-1, "ff_match_sift_workspace_bytes")
    return n


def ff_match_sift(jobs, p: ff_match_params, workspace, stream=None):
    arr = (ff_sift_job * len(jobs))(*jobs)
    _check(lib().ff_match_sift(arr, len(jobs), C.byref(p), _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_match_sift")


class SiftPairMatcher:
    """The hot path with the SIFT-flow data term for one pair (the paper's
    KITTI setting by default): Lab8 and WHT vectors of both images, the pair's
    SIFT colours (S2 = max(S, S2) channels) and their levels, one
    ff_match_sift call for F (r, S), B1 (r, S) and B2 (r2, S2), the
    consistency check (epsilon), the region filter (s) and the sparsification
    (e).  Buffers are allocated once for the given sizes and reused."""

    def __init__(self, width, height, channels=3, r=3, r2=2, S=12, S2=18, k=3, subpel=4, eps=1, region_s=150,
                 sparse_e=9, device="cuda", **params):
        self.W, self.H = width, height
        self.r, self.r2, self.S, self.S2, self.k, self.Q, self.eps = r, r2, S, S2, k, subpel, eps
        self.region_s, self.sparse_e = region_s, sparse_e
        self.Sc = max(S, S2)
        self.P = ff_sift_pitch(self.Sc)
        radii = (r, r2) if r2 != r else (r,)
        self.desc = ff_desc_init(width, height, channels, k, subpel, radii)
        dev = device
        self.blob1 = torch.empty(self.desc.bytes, dtype=torch.uint8, device=dev)
        self.blob2 = torch.empty(self.desc.bytes, dtype=torch.uint8, device=dev)
        self.codes1 = torch.empty((height, width, self.Sc), dtype=torch.int16, device=dev)
        self.codes2 = torch.empty_like(self.codes1)
        self.pca = torch.empty(2 * SIFT_DIM + SIFT_DIM * SIFT_DIM, dtype=torch.float64, device=dev)
        self.levels1 = torch.empty((k + 1, height, width, self.P), dtype=torch.int16, device=dev)
        self.levels2 = torch.empty_like(self.levels1)
        self.sift_ws = torch.empty(ff_sift_workspace_bytes(width, height, width, height), dtype=torch.uint8,
                                   device=dev)
        self.params = ff_default_params(k=k, **params)
        self.flow = {n: torch.empty((height, width), dtype=torch.int32, device=dev) for n in ("F", "B1", "B2")}
        self.cost = {n: torch.empty((height, width), dtype=torch.int32, device=dev) for n in ("F", "B1", "B2")}
        self.match_ws = torch.empty(ff_match_sift_workspace_bytes(self.jobs(0, 0), self.params), dtype=torch.uint8,
                                    device=dev)
        self.keep = torch.empty((height, width), dtype=torch.uint8, device=dev)
        self.filtered = torch.empty((height, width), dtype=torch.int32, device=dev)
        self.keep_region = torch.empty_like(self.keep)
        self.filtered_region = torch.empty_like(self.filtered)
        self.region_label = torch.empty_like(self.filtered)
        self.region_ws = torch.empty(ff_region_filter_workspace_bytes(width, height), dtype=torch.uint8, device=dev)
        self.pick = torch.empty(((height + 2) // 3, (width + 2) // 3), dtype=torch.int32, device=dev)
        self.sparse = torch.empty_like(self.filtered)

    def jobs(self, seed, pair_id):
        d, b1, b2, l1, l2 = self.desc, self.blob1, self.blob2, self.levels1, self.levels2
        return [make_sift_job(d, b1, d, b2, l1, l2, self.S, self.k, self.r, self.flow["F"], self.cost["F"], 0,
                              pair_id, seed),
                make_sift_job(d, b2, d, b1, l2, l1, self.S, self.k, self.r, self.flow["B1"], self.cost["B1"], 1,
                              pair_id, seed),
                make_sift_job(d, b2, d, b1, l2, l1, self.S2, self.k, self.r2, self.flow["B2"], self.cost["B2"], 2,
                              pair_id, seed)]

    def colors(self, img1, img2, codes=None, stream=None):
        """Lab8 / WHT of both images, then their colours -- computed here, or
        given as codes = (H x W x S2 int16, H x W x S2 int16) device tensors
        -- and the colour levels."""
        ff_compute_lab_wht(self.desc, img1, self.blob1, stream)
        ff_compute_lab_wht(self.desc, img2, self.blob2, stream)
        N = self.W * self.H
        L1 = self.blob1[self.desc.off_lab:self.desc.off_lab + N].view(self.H, self.W)
        L2 = self.blob2[self.desc.off_lab:self.desc.off_lab + N].view(self.H, self.W)
        if codes is None:
            ff_sift_colors(L1, L2, self.Sc, self.codes1, self.codes2, self.sift_ws, pca=self.pca, stream=stream)
        else:
            self.codes1.copy_(codes[0])
            self.codes2.copy_(codes[1])
        ff_sift_levels(self.codes1, self.k, self.levels1, self.sift_ws, stream)
        ff_sift_levels(self.codes2, self.k, self.levels2, self.sift_ws, stream)

    def run(self, img1, img2, seed=0, pair_id=0, codes=None, stream=None):
        self.colors(img1, img2, codes, stream)
        ff_match_sift(self.jobs(seed, pair_id), self.params, self.match_ws, stream)
        Q = self.Q
        bwd = [self.flow["B1"], self.flow["B2"]]
        ff_consistency_filter(self.flow["F"], bwd, Q, self.eps * Q, self.keep, self.filtered, stream)
        out = dict(codes1=self.codes1, codes2=self.codes2, pca=self.pca, F=self.flow["F"], CF=self.cost["F"],
                   B1=self.flow["B1"], CB1=self.cost["B1"], B2=self.flow["B2"], CB2=self.cost["B2"], keep=self.keep,
                   filtered=self.filtered)
        if self.region_s is not None:
            ff_region_filter(self.flow["F"], self.keep, Q, self.region_s, self.keep_region, self.filtered_region,
                             self.region_ws, label=self.region_label, stream=stream)
            out.update(keep_region=self.keep_region, filtered_region=self.filtered_region,
                       region_label=self.region_label)
            if self.sparse_e is not None:
                ff_sparsify(self.filtered_region, bwd, Q, self.sparse_e, self.pick, self.sparse, stream=stream)
                out.update(pick=self.pick, sparse=self.sparse)
        return out

    def status(self):
        return ff_read_status(self.match_ws)


# ------------------------------------------------------------------ helpers
def blob_views(d: ff_desc, blob: torch.Tensor):
    """Typed views of a descriptor blob's sections (for inspection)."""
    N = d.width * d.height
    H, W, Cc, K, Q = d.height, d.width, d.channels, d.k, d.subpel
    lab = blob[d.off_lab:d.off_lab + Cc * N].view(Cc, H, W)
    smooth = blob[d.off_smooth:d.off_smooth + (K + 1) * Cc * N * 2].view(torch.int16).view(K + 1, Cc, H, W)
    census = blob[d.off_census:d.off_census + (K + 1) * Q * Q * N * 4].view(torch.int32).view(K + 1, Q, Q, H, W)
    census_t = blob[d.off_census_t:d.off_census_t + (K + 1) * Q * Q * N * 4].view(torch.int32).view(K + 1, Q, Q, W, H)
    whts = {}
    for i in range(d.n_radii):
        o = d.off_wht + i * N * d.wht_stride * 4
        whts[d.radii[i]] = blob[o:o + N * d.wht_stride * 4].view(torch.int32).view(H, W, d.wht_stride)
    return dict(lab=lab, smooth=smooth, census=census, census_t=census_t, wht=whts)


class PairMatcher:
    """The whole hot path for one image pair on three streams: descriptors of
    both images, F = I1 -> I2 (r), B1 = I2 -> I1 (r), B2 = I2 -> I1 (r2), then
    the two-way consistency filter (sections 3.1-3.4).  Buffers are allocated
    once for a given image size and reused.  run() works on the caller's
    current stream plus three field streams: call it on the default stream,
    or capture it in a HIP graph; a fifth stream of the caller's would share
    one of HIP's four hardware queues with a field and serialise behind it."""

    def __init__(self, width, height, channels=3, r=8, r2=6, k=3, subpel=4, eps=5, n_bwd=2, device="cuda",
                 region_s=None, sparse_e=None, early_trees=True, **params):
        """region_s: None, or s of section 3.4's region filter, which then
        runs after the consistency check (outputs keep_region,
        filtered_region, region_label); sparse_e: None, or e of section
        3.5's sparsification of the region-filtered field (outputs pick,
        sparse; needs region_s); early_trees: build each field's kd-tree from
        its target's WHT vectors while the census planes are computed
        (ff_compute_lab_wht, ff_match_field_tree, ff_compute_census) instead
        of after whole descriptors; the results are the same."""
        if sparse_e is not None and region_s is None:
            raise ValueError("sparse_e needs region_s (sparsification follows the region filter)")
        self.W, self.H, self.C = width, height, channels
        self.region_s, self.sparse_e = region_s, sparse_e
        self.r, self.r2, self.k, self.Q, self.eps, self.n_bwd = r, r2, k, subpel, eps, n_bwd
        radii = (r,) if (n_bwd == 1 or r2 == r) else (r, r2)
        self.desc = ff_desc_init(width, height, channels, k, subpel, radii)
        self.blob1 = torch.empty(self.desc.bytes, dtype=torch.uint8, device=device)
        self.blob2 = torch.empty(self.desc.bytes, dtype=torch.uint8, device=device)
        self.params = [ff_default_params(k=k, field_id=i, **params) for i in range(3)]
        self.fields = [("F", r, 0), ("B1", r, 1)] + ([("B2", r2, 2)] if n_bwd == 2 else [])
        self.ws = []
        self.flow = {}
        self.cost = {}
        for name, rad, fid in self.fields:
            nb = ff_match_workspace_bytes(self.desc, self.desc, rad, self.params[fid])
            self.ws.append(torch.empty(nb, dtype=torch.uint8, device=device))
            self.flow[name] = torch.empty((height, width), dtype=torch.int32, device=device)
            self.cost[name] = torch.empty((height, width), dtype=torch.int32, device=device)
        self.keep = torch.empty((height, width), dtype=torch.uint8, device=device)
        self.filtered = torch.empty((height, width), dtype=torch.int32, device=device)
        if region_s is not None:
            self.keep_region = torch.empty((height, width), dtype=torch.uint8, device=device)
            self.filtered_region = torch.empty((height, width), dtype=torch.int32, device=device)
            self.region_label = torch.empty((height, width), dtype=torch.int32, device=device)
            self.region_ws = torch.empty(ff_region_filter_workspace_bytes(width, height), dtype=torch.uint8,
                                         device=device)
        if sparse_e is not None:
            self.pick = torch.empty(((height + 2) // 3, (width + 2) // 3), dtype=torch.int32, device=device)
            self.sparse = torch.empty((height, width), dtype=torch.int32, device=device)
        # four streams in all (the caller's and three field streams): HIP gives
        # a process four hardware queues by default, and a fifth stream would
        # share one with a field and serialise behind it
        self.streams = [torch.cuda.Stream(device=device) for _ in range(3)]
        # build each field's kd-tree as soon as its target's WHT vectors exist
        # (ff_match_field_tree), ahead of the census planes
        self.early_trees = early_trees

    def run(self, img1: torch.Tensor, img2: torch.Tensor, seed: int = 0, pair_id: int = 0, proposal=None):
        """proposal: None, a seed-grid tensor for F, or (forward, backward)
        where the backward proposal serves B1 and B2."""
        main = torch.cuda.current_stream()
        fs = self.streams
        tree_first = self.early_trees and any(self.params[fid].use_kdtree for _, _, fid in self.fields)
        if tree_first:
            # the kd-trees start on the WHT vectors (section 3.1) while the
            # census planes are computed: the second image's Lab8 and WHT on
            # F's stream (F's tree is over them), the first image's on the
            # caller's stream, whose census and smoothed levels follow
            fs[0].wait_stream(main)
            ff_compute_lab_wht(self.desc, img2, self.blob2, fs[0])
            img2.record_stream(fs[0])
            e2 = torch.cuda.Event()
            e2.record(fs[0])
            ff_compute_lab_wht(self.desc, img1, self.blob1, main)
            e1 = torch.cuda.Event()
            e1.record(main)
            for (name, rad, fid), ws, s in zip(self.fields, self.ws, fs):
                p = self.params[fid]
                if not p.use_kdtree:
                    continue
                if name != "F":
                    s.wait_event(e1)
                src, sb, dst, db = ((self.desc, self.blob1, self.desc, self.blob2) if name == "F"
                                    else (self.desc, self.blob2, self.desc, self.blob1))
                ff_match_field_tree(src, sb, dst, db, rad, p, ws, s)
            ff_compute_census(self.desc, self.blob1, main)
            main.wait_event(e2)
            ff_compute_census(self.desc, self.blob2, main)
        else:
            # the two images' descriptors run concurrently (each is a chain of
            # small kernels that leaves most of the chip idle); the second
            # image's go to the last field stream, which waits for both anyway
            ds = fs[len(self.fields) - 1]
            ds.wait_stream(main)
            ff_compute_descriptors(self.desc, img2, self.blob2, ds)
            img2.record_stream(ds)
            ff_compute_descriptors(self.desc, img1, self.blob1, main)
            main.wait_stream(ds)
        ev = torch.cuda.Event()
        ev.record(main)
        for (name, rad, fid), ws, s in zip(self.fields, self.ws, fs):
            s.wait_event(ev)
            p = self.params[fid]
            p.seed = seed
            p.pair_id = pair_id
            src, sb, dst, db = ((self.desc, self.blob1, self.desc, self.blob2) if name == "F"
                                else (self.desc, self.blob2, self.desc, self.blob1))
            if isinstance(proposal, (tuple, list)):
                prop = proposal[0] if name == "F" else proposal[1]
            else:
                prop = proposal if name == "F" else None
            built = tree_first and p.use_kdtree
            if built:
                p.use_kdtree = 2   # the tree built above, in this workspace
            try:
                ff_match_field(src, sb, dst, db, rad, p, prop, self.flow[name], self.cost[name], ws, s)
            finally:
                if built:
                    p.use_kdtree = 1
        for s in self.streams[:len(self.fields)]:
            e = torch.cuda.Event()
            e.record(s)
            main.wait_event(e)
        bwd = [self.flow["B1"]] + ([self.flow["B2"]] if self.n_bwd == 2 else [])
        ff_consistency_filter(self.flow["F"], bwd, self.Q, self.eps * self.Q, self.keep, self.filtered, main)
        out = dict(F=self.flow["F"], CF=self.cost["F"], B1=self.flow["B1"], CB1=self.cost["B1"],
                   B2=self.flow.get("B2"), CB2=self.cost.get("B2"), keep=self.keep, filtered=self.filtered)
        if self.region_s is not None:
            ff_region_filter(self.flow["F"], self.keep, self.Q, self.region_s, self.keep_region,
                             self.filtered_region, self.region_ws, label=self.region_label, stream=main)
            out.update(keep_region=self.keep_region, filtered_region=self.filtered_region,
                       region_label=self.region_label)
            if self.sparse_e is not None:
                ff_sparsify(self.filtered_region, bwd, self.Q, self.sparse_e, self.pick, self.sparse, stream=main)
                out.update(pick=self.pick, sparse=self.sparse)
        return out

    def status(self):
        return [ff_read_status(w) for w in self.ws]


class BatchMatcher:
    """The whole hot path for many pairs (any sizes) at once: descriptors of
    every image, then one ff_match_batch call for all 3 fields of all pairs
    (each stage one launch), then the consistency filter of every pair.
    `run` can be captured in a HIP graph (see `capture`)."""

    def __init__(self, shapes, channels=3, r=8, r2=6, k=3, subpel=4, eps=5, device="cuda", band_rows=16,
                 use_kdtree=1, pipeline=0):
        self.shapes = list(shapes)            # (W, H) per pair
        self.C, self.r, self.r2, self.k, self.Q, self.eps = channels, r, r2, k, subpel, eps
        # a batch keeps the GPU full of bands: pipelined sweep pairs, which
        # add workgroups to overlap a field's sweeps, are off unless asked for
        # (autotune() times both)
        self.params = ff_default_params(k=k, band_rows=band_rows, use_kdtree=use_kdtree, pipeline=pipeline)
        self.descs, self.blobs1, self.blobs2, self.out = [], [], [], []
        for (W, H) in self.shapes:
            d = ff_desc_init(W, H, channels, k, subpel, (r, r2) if r2 != r else (r,))
            self.descs.append(d)
            self.blobs1.append(torch.empty(d.bytes, dtype=torch.uint8, device=device))
            self.blobs2.append(torch.empty(d.bytes, dtype=torch.uint8, device=device))
            o = {name: (torch.empty((H, W), dtype=torch.int32, device=device),
                        torch.empty((H, W), dtype=torch.int32, device=device)) for name in ("F", "B1", "B2")}
            o["keep"] = torch.empty((H, W), dtype=torch.uint8, device=device)
            o["filtered"] = torch.empty((H, W), dtype=torch.int32, device=device)
            self.out.append(o)
        self.proposals = [None] * len(self.shapes)
        self.seeds = [0] * len(self.shapes)
        self._jobs_cache = None
        self.ws = None

    def _proposal(self, i, name):
        """Per pair: None, a tensor (F only) or (forward, backward) where the
        backward proposal serves B1 and B2."""
        p = self.proposals[i]
        if isinstance(p, (tuple, list)):
            return p[0] if name == "F" else p[1]
        return p if name == "F" else None

    def jobs(self):
        jobs = []
        for i, d in enumerate(self.descs):
            o = self.out[i]
            for name, rad, fid, (s, sb, t, tb) in (("F", self.r, 0, (d, self.blobs1[i], d, self.blobs2[i])),
                                                    ("B1", self.r, 1, (d, self.blobs2[i], d, self.blobs1[i])),
                                                    ("B2", self.r2, 2, (d, self.blobs2[i], d, self.blobs1[i]))):
                jobs.append(make_job(s, sb, t, tb, rad, o[name][0], o[name][1], field_id=fid, pair_id=i,
                                     seed=self.seeds[i], proposal=self._proposal(i, name), k=self.k))
        return jobs

    def run(self, imgs1, imgs2, seeds=None, proposals=None, stream=None):
        stream = stream or torch.cuda.current_stream()
        if seeds is not None:
            self.seeds = list(seeds)
        if proposals is not None:
            self.proposals = list(proposals)
        for i, d in enumerate(self.descs):
            ff_compute_descriptors(d, imgs1[i], self.blobs1[i], stream)
            ff_compute_descriptors(d, imgs2[i], self.blobs2[i], stream)
        jobs = self.jobs()
        need = ff_match_batch_workspace_bytes(jobs, self.params)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.blobs1[0].device)
        ff_match_batch(jobs, self.params, self.ws, stream)
        for o in self.out:
            ff_consistency_filter(o["F"][0], [o["B1"][0], o["B2"][0]], self.Q, self.eps * self.Q, o["keep"],
                                  o["filtered"], stream)
        return self.out

    def status(self):
        return ff_read_status(self.ws)

    def autotune(self, imgs1, imgs2, band_rows=(8, 16, 32), pipeline=(1, 0), reps=2):
        """Time every (band height, sweep-pair pipelining) combination on this
        batch and keep the fastest (all give identical bytes).  Returns
        (band_rows, pipeline, ms)."""
        best = None
        for bh in band_rows:
            for pipe in pipeline:
                self.params.band_rows = bh
                self.params.pipeline = pipe
                self.run(imgs1, imgs2)
                torch.cuda.synchronize()
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record()
                for _ in range(reps):
                    self.run(imgs1, imgs2)
                t1.record()
                torch.cuda.synchronize()
                ms = t0.elapsed_time(t1) / reps
                if best is None or ms < best[2]:
                    best = (bh, pipe, ms)
        self.params.band_rows, self.params.pipeline = best[0], best[1]
        return best


# ------------------------------------------------------------------ learned proposal
NET_FLOW_SCALE = 32.0   # flow in px = 32 x network output
NET_LAYERS = [(6, 32, 2, 1, True), (32, 32, 2, 1, True), (32, 32, 2, 1, True),
              (32, 32, 1, 4, True), (32, 32, 1, 8, True), (32, 2, 1, 1, False)]


def ff_net_param_count() -> int:
    return lib().ff_net_param_count()


def ff_net_workspace_bytes(batch, width, height) -> int:
    n = lib().ff_net_workspace_bytes(batch, width, height)
    if n == 0:
        raise FFError(-1, "ff_net_workspace_bytes")
    return n


def ff_proposal_forward(params, img1, img2, proposal, workspace, subpel=4, flow_out=None, stream=None):
    B, H, W = img1.shape[:3]
    _check(lib().ff_proposal_forward(_ptr(params), _ptr(img1), _ptr(img2), B, W, H, subpel, _ptr(proposal),
                                     _ptr(flow_out), _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_proposal_forward")


def ff_proposal_train_step(params, adam_m, adam_v, step, lr, img1, img2, labels, workspace, subpel=4,
                           grad_out=None, loss_out=None, stream=None):
    B, H, W = img1.shape[:3]
    _check(lib().ff_proposal_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), step, lr, _ptr(img1), _ptr(img2),
                                        _ptr(labels), B, W, H, subpel, _ptr(grad_out), _ptr(loss_out),
                                        _ptr(workspace), workspace.numel(), _stream(stream)),
           "ff_proposal_train_step")


def net_init_params(seed=0):
    """He-normal weights, zero biases, float32 on the host (parameter layout
    of ff_proposal_forward)."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for ci, co, _, _, relu in NET_LAYERS:
        std = (2.0 / (ci * 9)) ** 0.5 if relu else (1.0 / (ci * 9)) ** 0.5
        parts.append(torch.randn(co * ci * 9, generator=g, dtype=torch.float32) * std)
        parts.append(torch.zeros(co, dtype=torch.float32))
    return torch.cat(parts)


def seed_grid(width, height, k=3):
    s = 1 << k
    return (height + s - 1) // s, (width + s - 1) // s


class ProposalNet:
    """Parameters, Adam state and workspaces of the proposal network on one
    device.  Images: uint8 tensors batch x H x W x 3 (or H x W x 3)."""

    def __init__(self, params=None, seed=0, device="cuda", subpel=4):
        if ff_net_param_count() != sum(co * ci * 9 + co for ci, co, _, _, _ in NET_LAYERS):
            raise FFError(-1, "network layout mismatch")
        p = net_init_params(seed) if params is None else torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        self.device = device
        self.subpel = subpel
        self.params = p.to(device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self._ws = {}

    def workspace(self, batch, width, height):
        key = (batch, width, height)
        if key not in self._ws:
            self._ws[key] = torch.empty(ff_net_workspace_bytes(batch, width, height), dtype=torch.uint8,
                                        device=self.device)
        return self._ws[key]

    @staticmethod
    def _b(img):
        return img if img.dim() == 4 else img.unsqueeze(0)

    def forward(self, img1, img2, proposal=None, flow_out=None, stream=None):
        i1, i2 = self._b(img1), self._b(img2)
        B, H, W = i1.shape[:3]
        hc, wc = seed_grid(W, H)
        if proposal is None:
            proposal = torch.empty((B, hc, wc), dtype=torch.int32, device=self.device)
        ff_proposal_forward(self.params, i1, i2, proposal, self.workspace(B, W, H), self.subpel, flow_out, stream)
        return proposal

    def gradient(self, img1, img2, labels, stream=None):
        """Loss and parameter gradient without an update."""
        i1, i2 = self._b(img1), self._b(img2)
        B, H, W = i1.shape[:3]
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        ff_proposal_train_step(self.params, None, None, 0, 0.0, i1, i2, labels, self.workspace(B, W, H),
                               self.subpel, g, loss, stream)
        return loss, g

    def train_step(self, img1, img2, labels, lr, stream=None):
        i1, i2 = self._b(img1), self._b(img2)
        B, H, W = i1.shape[:3]
        self.step += 1
        ff_proposal_train_step(self.params, self.m, self.v, self.step, lr, i1, i2, labels,
                               self.workspace(B, W, H), self.subpel, None, self.loss, stream)
        return self.loss

    def state_dict(self):
        return dict(params=self.params.cpu(), m=self.m.cpu(), v=self.v.cpu(),
                    step=torch.tensor(self.step, dtype=torch.int64))

    def load_state_dict(self, sd):
        self.params.copy_(sd["params"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step = int(sd["step"])
