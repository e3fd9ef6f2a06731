"""The C-ABI library loads, exports every function include/ff.h declares, and
validates arguments on the host (no compute call: these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ff_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def ff():
    from paper_1508_05151_amd import ff as _ff
    if not os.path.exists(_ff.LIB_PATH):
        pytest.fail("libff.so is not built (run __graft_entry__.build())")
    return _ff


def test_every_declared_symbol_is_exported(ff):
    lib = C.CDLL(ff.LIB_PATH)
    names = _declared()
    assert "ff_match_field" in names and "ff_compute_descriptors" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(ff):
    # ff_desc: 12 int32 then 7 size_t; ff_match_params: 10 x 4-byte fields then uint64
    assert C.sizeof(ff.ff_desc) == 12 * 4 + 7 * 8
    assert C.sizeof(ff.ff_match_params) == 12 * 4 + 8
    assert ff.ff_match_params.seed.offset == 48
    # ff_field_job: 4 pointers, 4 x 4-byte fields, uint64 seed, 3 pointers
    assert C.sizeof(ff.ff_field_job) == 4 * 8 + 4 * 4 + 8 + 3 * 8
    assert ff.ff_field_job.seed.offset == 48 and ff.ff_field_job.cost.offset == 72


def test_desc_init_validation(ff):
    d = ff.ff_desc_init(128, 96, 3, 3, 4, (8, 6))
    assert d.bytes > 0 and d.off_census < d.off_census_t < d.off_wht
    assert d.plane_bytes == 128 * 96 * 4
    for bad in [dict(width=0, height=5), dict(width=5, height=5, channels=2), dict(width=5, height=5, k=5),
                dict(width=5, height=5, subpel=3), dict(width=5, height=5, radii=(0,)),
                dict(width=5, height=5, radii=(4, 4)), dict(width=5, height=5, radii=(16,))]:
        kw = dict(channels=3, k=3, subpel=4, radii=(8,))
        kw.update(bad)
        with pytest.raises(ff.FFError):
            ff.ff_desc_init(kw.pop("width"), kw.pop("height"), **kw)
    with pytest.raises(ff.FFError) as e:
        ff.ff_desc_init(8192, 8, 3, 3, 4, (8,))
    assert e.value.code == -2


def test_match_argument_checks_before_any_launch(ff):
    d = ff.ff_desc_init(64, 48, 3, 3, 4, (8,))
    p = ff.ff_default_params()
    assert (p.k, p.R, p.leaf, p.n_prop, p.n_rs, p.use_kdtree, p.max_steps) == (3, 1, 8, 4, 3, 1, -1)
    assert (p.band_rows, p.pipeline, p.watchdog_us) == (16, 1, 0)
    assert ff.ff_match_workspace_bytes(d, d, 8, p) > 0
    L = ff.lib()
    # radius without WHT vectors, leaf out of range, k above the descriptors'
    # pipeline flag 0/1 only, watchdog not negative
    for r, kw in [(6, {}), (8, dict(leaf=1)), (8, dict(k=4)), (8, dict(n_rs=5)), (8, dict(field_id=4)),
                  (8, dict(pipeline=2)), (8, dict(watchdog_us=-1))]:
        q = ff.ff_default_params(**kw)
        assert L.ff_match_workspace_bytes(C.byref(d), C.byref(d), r, C.byref(q)) == 0
    # null buffers are rejected before anything is enqueued
    rc = L.ff_match_field(C.byref(d), None, C.byref(d), None, 8, C.byref(p), None, None, None, None, 0, None)
    assert rc == -1
    assert L.ff_consistency_filter(None, 4, 4, None, 1, 4, 4, 4, 20, None, None, None) == -1
    assert ff.ff_tree_nodes(446464, 8) == (2 << 16) - 1
    assert L.ff_status_string(-6) == b"device watchdog fired"


def test_network_entry_points_validate(ff):
    L = ff.lib()
    assert ff.ff_net_param_count() == 39330
    assert L.ff_net_workspace_bytes(0, 64, 64) == 0 and L.ff_net_workspace_bytes(1, 7, 64) == 0
    assert L.ff_net_workspace_bytes(257, 64, 64) == 0
    assert L.ff_net_workspace_bytes(2, 64, 48) > 0
    assert L.ff_proposal_forward(None, None, None, 1, 64, 64, 4, None, None, None, 0, None) == -1
    assert L.ff_proposal_train_step(None, None, None, 1, 1e-3, None, None, None, 1, 64, 64, 4, None, None, None, 0,
                                    None) == -1


def test_batch_entry_points_validate(ff):
    L = ff.lib()
    p = ff.ff_default_params()
    assert L.ff_match_batch_workspace_bytes(None, 1, C.byref(p)) == 0
    assert L.ff_match_batch(None, 1, C.byref(p), None, 0, None) == -1
    d = ff.ff_desc_init(64, 48, 3, 3, 4, (8,))
    jobs = (ff.ff_field_job * 1)()
    jobs[0].src = C.pointer(d)
    jobs[0].dst = C.pointer(d)
    jobs[0].radius = 8
    # sizing needs only descriptors and radius; a radius without WHT vectors
    # is refused; launching with null blobs, outputs or workspace is refused
    assert L.ff_match_batch_workspace_bytes(jobs, 1, C.byref(p)) > 0
    jobs[0].radius = 6
    assert L.ff_match_batch_workspace_bytes(jobs, 1, C.byref(p)) == 0
    jobs[0].radius = 8
    assert L.ff_match_batch(jobs, 1, C.byref(p), None, 0, None) == -1
    assert L.ff_match_batch(jobs, 0, C.byref(p), None, 0, None) == -1


def test_tree_ahead_entry_points_validate(ff):
    """use_kdtree is 0, 1 or 2; 2 (the tree left in the workspace by
    ff_match_field_tree) serves one-field calls only; the tree-only call needs
    kd-tree seeding, both blobs and a large enough workspace; the census-only
    call needs a blob of the descriptor's size.  All refused before any
    launch."""
    L = ff.lib()
    d = ff.ff_desc_init(64, 48, 3, 3, 4, (8,))
    for v in (-1, 3):
        q = ff.ff_default_params(use_kdtree=v)
        assert L.ff_match_workspace_bytes(C.byref(d), C.byref(d), 8, C.byref(q)) == 0
    q2 = ff.ff_default_params(use_kdtree=2)
    assert L.ff_match_workspace_bytes(C.byref(d), C.byref(d), 8, C.byref(q2)) > 0
    jobs = (ff.ff_field_job * 2)()
    for j in jobs:
        j.src = C.pointer(d)
        j.dst = C.pointer(d)
        j.radius = 8
    fake = C.c_void_p(0x1000)
    assert L.ff_match_batch(jobs, 2, C.byref(q2), fake, 1 << 30, None) == -1
    p = ff.ff_default_params()
    q0 = ff.ff_default_params(use_kdtree=0)
    assert L.ff_match_field_tree(C.byref(d), fake, C.byref(d), fake, 8, C.byref(q0), fake, 1 << 30, None) == -1
    assert L.ff_match_field_tree(C.byref(d), None, C.byref(d), fake, 8, C.byref(p), fake, 1 << 30, None) == -1
    assert L.ff_match_field_tree(C.byref(d), fake, C.byref(d), fake, 6, C.byref(p), fake, 1 << 30, None) == -1
    assert L.ff_match_field_tree(C.byref(d), fake, C.byref(d), fake, 8, C.byref(p), fake, 16, None) == -3
    assert L.ff_compute_census(C.byref(d), None, d.bytes, None) == -1
    assert L.ff_compute_census(C.byref(d), fake, d.bytes - 1, None) == -3


def test_desc_init_refuses_layouts_beyond_the_sweeps_32bit_offsets(ff):
    """The sweep addresses the row-major and transposed census planes of a
    level from one base with 32-bit byte offsets; its largest word index is
    (census region words) + Q^2 N - 1, which must stay below 2^30.  At Q = 8
    that caps the image: k = 3 allows (k + 2) 64 N <= 2^30, N <= 3,355,443."""
    with pytest.raises(ff.FFError) as e:
        ff.ff_desc_init(4095, 1024, 3, 3, 8, (8, 6))
    assert e.value.code == -2
    with pytest.raises(ff.FFError) as e:
        ff.ff_desc_init(4095, 1024, 3, 4, 8, (8,))
    assert e.value.code == -2
    for (W, H, k, q) in [(4095, 818, 3, 8), (4095, 1024, 2, 8), (4095, 1024, 1, 8), (4096, 1024, 4, 4),
                         (8191, 512, 3, 4)]:
        d = ff.ff_desc_init(W, H, 3, k, q, (8, 6))
        words = (d.off_census_t - d.off_census) // 4 + q * q * W * H
        assert words <= 1 << 30, (W, H, k, q)
    # every accepted (size, k, Q) keeps the bound; every refused one breaks it
    for (W, H) in [(4095, 819), (4095, 820), (3000, 1200), (2048, 2048), (4095, 1024)]:
        for k in range(5):
            try:
                d = ff.ff_desc_init(W, H, 3, k, 8, (8,))
            except ff.FFError as err:
                assert err.code == -2
                assert (k + 2) * 64 * W * H > 1 << 30, (W, H, k)
                continue
            assert (d.off_census_t - d.off_census) // 4 + 64 * W * H <= 1 << 30


def test_binding_checks_proposal_and_outputs_before_any_launch(ff):
    """The seed step reads proposal[gy * Gw + gx] over the k-level seed grid
    and the outputs over the whole source image, through plain pointers: the
    binding refuses a buffer of the wrong type, size or shape (or a host
    tensor) before anything reaches the library."""
    import torch
    d = ff.ff_desc_init(64, 48, 3, 3, 4, (8,))
    p = ff.ff_default_params()
    ok_flow = torch.empty((48, 64), dtype=torch.int32)
    cases = [
        (torch.zeros((6, 8), dtype=torch.int32), "device"),          # right shape, host memory
        (torch.zeros((12, 16), dtype=torch.int32), "seed grid"),     # the k = 2 grid
        (torch.zeros((6, 9), dtype=torch.int32), "seed grid"),
        (torch.zeros((48,), dtype=torch.int32), "device"),           # flat, right size
        (torch.zeros((47,), dtype=torch.int32), "elements"),
        (torch.zeros((6, 8), dtype=torch.int64), "int32"),
        (torch.zeros((8, 6), dtype=torch.int32).t(), "contiguous"),
    ]
    for prop, msg in cases:
        with pytest.raises(ff.FFError, match=msg):
            ff.ff_match_field(d, None, d, None, 8, p, prop, ok_flow, ok_flow, None)
        with pytest.raises(ff.FFError, match=msg):
            ff.make_job(d, None, d, None, 8, ok_flow, ok_flow, proposal=prop, k=3)
    with pytest.raises(ff.FFError, match="elements"):
        ff.ff_match_field(d, None, d, None, 8, p, None, torch.empty((48, 63), dtype=torch.int32), ok_flow, None)
    # a k = 2 batch needs the 12 x 16 grid
    with pytest.raises(ff.FFError, match="device"):
        ff.make_job(d, None, d, None, 8, ok_flow, ok_flow, proposal=torch.zeros((12, 16), dtype=torch.int32), k=2)


def test_noalloc_entry_refuses_before_any_launch(ff):
    """ff_match_field_noalloc checks the parameters, then the field's scratch
    need against FF_NOALLOC_SCRATCH_BYTES (FF_ERR_SIZE), then the pointers
    (FF_ERR_ARG) -- all before anything is enqueued."""
    L = ff.lib()
    p = ff.ff_default_params()
    big = ff.ff_desc_init(1920, 1080, 3, 3, 4, (8,))
    assert ff.ff_match_workspace_bytes(big, big, 8, p) > ff.NOALLOC_SCRATCH_BYTES
    assert L.ff_match_field_noalloc(C.byref(big), None, C.byref(big), None, 8, C.byref(p), None, None, None, None,
                                    None) == -2
    ok = ff.ff_desc_init(1280, 720, 3, 3, 4, (8,))
    assert ff.ff_match_workspace_bytes(ok, ok, 8, p) <= ff.NOALLOC_SCRATCH_BYTES
    assert L.ff_match_field_noalloc(C.byref(ok), None, C.byref(ok), None, 8, C.byref(p), None, None, None, None,
                                    None) == -1
    # a radius without WHT vectors
    assert L.ff_match_field_noalloc(C.byref(ok), None, C.byref(ok), None, 6, C.byref(p), None, None, None, None,
                                    None) == -1
    assert L.ff_match_field_noalloc(None, None, None, None, 8, None, None, None, None, None, None) == -1
    # its scratch never holds a tree built ahead
    q2 = ff.ff_default_params(use_kdtree=2)
    fake = C.c_void_p(0x1000)
    assert L.ff_match_field_noalloc(C.byref(ok), fake, C.byref(ok), fake, 8, C.byref(q2), None, fake, fake, None,
                                    None) == -1


def test_load_latency_probe_validation(ff):
    """The load-latency probe refuses bad sizes and null pointers on the host,
    before anything is enqueued (fake device pointers are never touched)."""
    lib = C.CDLL(ff.LIB_PATH)
    lib.ff_probe_load_latency.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
    lib.ff_probe_load_latency.restype = C.c_int32
    fake = C.c_void_p(0x10000)
    for nxt, n, warm, hops, out in [(None, 1024, 0, 10, fake), (fake, 1024, 0, 10, None), (fake, 1000, 0, 10, fake),
                                    (fake, 1, 0, 10, fake), (fake, 1 << 29, 0, 10, fake), (fake, 1024, -1, 10, fake),
                                    (fake, 1024, 0, 0, fake), (fake, 1024, 0, (1 << 22) + 1, fake),
                                    (fake, 1024, (1 << 22) + 1, 10, fake)]:
        assert lib.ff_probe_load_latency(nxt, n, warm, hops, out, None) == -1, (n, warm, hops)


def test_load_cycle_visits_every_line_once(ff):
    """The probe's cycle starts at index 0, visits the first word of every
    128-byte line exactly once and returns to 0."""
    import numpy as np
    n = 1 << 14
    nxt = ff.load_cycle(n, seed=3)
    i, seen = 0, []
    for _ in range(n // 32):
        seen.append(i)
        i = int(nxt[i])
    assert i == 0 and sorted(seen) == list(range(0, n, 32))
    assert np.all(nxt[np.arange(n) % 32 != 0] == 0)
