#!/usr/bin/env python
"""Benchmark of the Flow Fields hot path on one MI355X.

One step = the whole path on one 1024x436 RGB pair (Sintel-shaped synthetic
pair, seeded): descriptors of both images, the three fields F = I1->I2 (r=8),
B1 = I2->I1 (r=8), B2 = I2->I1 (r2=6) each with its kd-tree, and the two-way
consistency filter (sections 3.1-3.4, parameters of section 4: k=3, R=1,
l=8, eps=5).  Inputs are resident in HBM before the timed region.

Prints one JSON line with the throughput (Mpixel/s = W*H / time per pair),
the dominant kernel's measured rate against its roofline and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and chip figures
HBM_PEAK_GBS = 8000.0
CUS, LANES_PER_CU, CLOCK_GHZ = 256, 64, 2.4
INT_PEAK_TOPS = CUS * LANES_PER_CU * CLOCK_GHZ / 1000.0   # 32-bit integer VALU ops, 39.3 T/s

# HBM bytes per k_propagate launch (average over the 27 launches of one pair:
# single sweeps and pipelined sweep pairs),
# from FETCH_SIZE and WRITE_SIZE counter runs scaled by a plain-copy
# calibration; profiles/hotpath_1024x436_hbm_counters.md holds the runs.
# Valid for the current k_propagate only.
PROPAGATE_HBM_BYTES_PER_LAUNCH = 68.47e6

PROF_CLASS = {"descriptors": 1, "tree": 2, "seed": 3, "level_entry": 4, "propagate": 5, "random_search": 6,
              "filter": 7}


def grid_points(W, H, k):
    return [((W + (1 << l) - 1) >> l) * ((H + (1 << l) - 1) >> l) for l in range(k + 1)]


def propagate_ops_per_pair(W, H, k, radii, n_prop=4):
    """Algorithmic integer ops of all propagation sweeps of one pair: per grid
    point and sweep, two candidates costed by sliding windows, each 2(2r+1)
    census terms of one XOR and one popcount-accumulate (2 ops)."""
    pts = sum(grid_points(W, H, k))
    return sum(n_prop * pts * 2 * 2 * (2 * r + 1) * 2 for r in radii)


def per_point_ops_in_sweep_launches(W, H, k, radii, n_prop=4, n_rs=3):
    """Algorithmic integer ops of the per-point stages that run inside
    pipelined sweep-pair launches, following the library's pairing: two
    sweeps of one level with the same horizontal direction hold the random
    search between them (all grid points), and a level's last sweep paired
    with the next level's first holds that level's entry (the carried points,
    one per point of the coarser grid); each point costs (2r+1)^2 census
    terms of 2 ops."""
    sx = lambda i: 1 if (i & 3) in (0, 3) else -1
    sy = lambda i: 1 if (i & 3) in (0, 2) else -1
    pts = grid_points(W, H, k)
    terms = 0          # grid points costed inside launches, per field
    entered = False
    for lev in range(k, -1, -1):
        i = 1 if entered else 0
        entered = False
        while i < n_prop:
            if i + 1 < n_prop and sx(i + 1) == sx(i):
                terms += pts[lev] if i < n_rs else 0
                i += 2
            elif (i == n_prop - 1 and i >= n_rs and lev > 0 and sx(0) == sx(i) and sy(0) == -sy(i)):
                terms += pts[lev]       # points of level lev = the carried points of level lev - 1
                entered = True
                i += 1
            else:
                i += 1
    return sum(terms * (2 * r + 1) ** 2 * 2 for r in radii)


def cpu_sample(crop_w, crop_h):
    """The oracle (plain single-threaded C++) on the same hot path over a
    crop of the benchmark pair; returns Mpixel/s of that sample."""
    from oracle import ffo
    from synth import pairs
    p = pairs.layered_pair(1000)
    i1 = p.img1[:crop_h, :crop_w].copy()
    i2 = p.img2[:crop_h, :crop_w].copy()
    t0 = time.perf_counter()
    ffo.match_pair(i1, i2, r=8, r2=6, k=3, Q=4, eps=5, seed=1000)
    dt = time.perf_counter() - t0
    return crop_w * crop_h / dt / 1e6, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--crop", default="768x327", help="CPU baseline sample: crop WxH of the pair")
    ap.add_argument("--dominant", default="propagate", choices=sorted(PROF_CLASS))
    ap.add_argument("--mode", default="pair", choices=("pair", "batch", "outliers"),
                    help="pair: one 1024x436 pair (headline); batch: 64 mixed-size pairs in one batched call; "
                         "outliers: removed outliers vs removed inliers of the filters over epsilon")
    ap.add_argument("--pairs", type=int, default=64, help="batch mode: number of pairs")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes drawing the synthetic pairs (0 = in-process; use 0 under a profiler)")
    ap.add_argument("--no-learned", action="store_true",
                    help="pair mode: skip the learned-proposal comparison")
    ap.add_argument("--learned-pairs", type=int, default=16,
                    help="pair mode: held-out 1024x436 pairs of the learned-proposal comparison")
    ap.add_argument("--band-rows", type=int, default=16, choices=(8, 16, 32),
                    help="pair mode: propagation band height (results are identical for every value)")
    ap.add_argument("--pipeline", type=int, default=1, choices=(0, 1),
                    help="pair mode: pipelined sweep pairs (results are identical)")
    ap.add_argument("--outlier-pairs", type=int, default=8,
                    help="outliers mode: layered 1024x436 pairs (seeds 1000..)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (the reference dispatch "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the matcher runs on one GPU: each pair is matched on one MI355X; "
                                   "--gpus must be 1"}), flush=True)
        sys.exit(2)

    from synth import pairs
    # synthetic pairs are drawn before anything touches the GPU (worker
    # processes are started from a process that has not initialised it)
    batch_pairs = eval_pairs = None
    if args.mode == "outliers":
        outlier_pairs = pairs.layered_pairs(OUTLIER_SEED0, args.outlier_pairs, workers=args.gen_workers)
    if args.mode == "batch":
        if args.gen_workers > 0:
            batch_pairs = pairs.mixed_pairs_parallel(args.pairs, workers=args.gen_workers)
        else:
            batch_pairs = pairs.mixed_pairs(args.pairs)
    elif not args.no_learned:
        eval_pairs = pairs.layered_pairs(LEARNED_SEED0, args.learned_pairs, workers=args.gen_workers)

    import numpy as np
    import torch
    from paper_1508_05151_amd import ff

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.mode == "batch":
        return bench_batch(args, ff, batch_pairs, torch, dev)
    if args.mode == "outliers":
        return bench_outliers(args, ff, outlier_pairs, torch, dev)
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pair = pairs.layered_pair(1000)
    H, W, C = pair.img1.shape
    k, r, r2, Q, eps = 3, 8, 6, 4, 5
    img1 = torch.from_numpy(pair.img1).to(dev)
    img2 = torch.from_numpy(pair.img2).to(dev)
    ff.ff_init()
    m = ff.PairMatcher(W, H, C, r=r, r2=r2, k=k, subpel=Q, eps=eps, band_rows=args.band_rows,
                       pipeline=args.pipeline)
    for _ in range(args.warmup):
        m.run(img1, img2, seed=1000)
    torch.cuda.synchronize()
    if args.warmup:
        assert m.status() == [0, 0, 0], m.status()

    # timed region: K whole-path steps; the dominant kernel class is bracketed
    # with HIP events on the streams it runs on (library profiling hook)
    launches_per_step = {"propagate": 3 * (k + 1) * 4, "random_search": 3 * (k + 1) * 3, "descriptors": 2,
                         "tree": 3, "seed": 3, "level_entry": 3 * k, "filter": 1}[args.dominant]
    ff._check(ff.lib().ff_profile_begin(PROF_CLASS[args.dominant], launches_per_step * args.steps + 8),
              "ff_profile_begin")
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record()
        out = m.run(img1, img2, seed=1000)
        ends[i].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    import ctypes
    tot = ctypes.c_double(0)
    nl = ctypes.c_int32(0)
    ff._check(ff.lib().ff_profile_end(ctypes.byref(tot), ctypes.byref(nl)), "ff_profile_end")
    assert m.status() == [0, 0, 0], m.status()
    per_step = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = W * H / (ms_per_step / 1000.0) / 1e6

    # dominant kernel against its roofline (integer VALU: census terms)
    avg_launch_ms = tot.value / max(nl.value, 1)
    roof = None
    if args.dominant == "propagate":
        # launches per step as measured (a pipelined sweep pair is one launch)
        ops_per_launch = (propagate_ops_per_pair(W, H, k, (r, r, r2)) +
                          per_point_ops_in_sweep_launches(W, H, k, (r, r, r2))) / (nl.value / args.steps)
        achieved = ops_per_launch / (avg_launch_ms / 1000.0) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(INT_PEAK_TOPS, 2), "unit": "TOP/s",
                "frac": round(achieved / INT_PEAK_TOPS, 5), "traffic": PROPAGATE_HBM_BYTES_PER_LAUNCH,
                "traffic_GBps": round(PROPAGATE_HBM_BYTES_PER_LAUNCH / (avg_launch_ms / 1000.0) / 1e9, 2),
                "kernel": "k_propagate", "avg_launch_ms": round(avg_launch_ms, 4), "launches": nl.value,
                "ops_per_launch": int(ops_per_launch)}

    keep = out["keep"].float().mean().item()
    rate = pairs.inlier_rate(out["F"].cpu().numpy(), pair, Q)
    line = {
        "metric": "flow-field Mpixel/s at 1024\u00d7436, plain vs learned proposal; % of HBM roofline",
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "median_ms_per_step": round(statistics.median(per_step), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "one 1024x436 RGB Sintel-shaped layered pair (seed 1000): descriptors x2, "
                               "F/B1/B2 fields with kd-trees, two-way consistency filter",
                   "k": k, "r": r, "r2": r2, "R": 1, "leaf": 8, "subpel": Q, "eps": eps,
                   "band_rows": args.band_rows, "pipelined_sweep_pairs": bool(args.pipeline)},
        "roofline": roof,
        "quality": {"F_inlier_rate_epe_lt_3px": round(rate, 4), "kept_fraction": round(keep, 4)},
    }
    if eval_pairs is not None:
        line["learned_proposal"] = bench_learned(ff, pair, img1, img2, eval_pairs, torch, dev, value, rate)
    if not args.no_cpu:
        cw, ch = (int(v) for v in args.crop.split("x"))
        mpx, dt = cpu_sample(cw, ch)
        line["cpu_baseline"] = {"value": round(mpx, 5), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
                                "sample": f"whole hot path on the top-left {cw}x{ch} crop of the same pair "
                                          f"({cw * ch} px, {dt:.1f} s single-threaded)"}
    print(json.dumps(line), flush=True)


LEARNED_SEED0 = 4000
WEIGHTS = os.path.join(ROOT, "paper_1508_05151_amd", "weights", "proposal_1024x436.safetensors")


def bench_learned(ff, pair, img1, img2, eval_pairs, torch, dev, plain_value, plain_rate, steps=5):
    """The learned proposal against the plain method: on the headline pair
    (plain + learned candidate; learned only, no kd-tree; the network's
    forward pass in both directions is inside the timed region) and on a
    batch of held-out 1024x436 pairs matched in one batched call."""
    from paper_1508_05151_amd import proposal
    from synth import pairs
    net = proposal.load(WEIGHTS)
    H, W = pair.img1.shape[:2]
    b1, b2 = img1.unsqueeze(0), img2.unsqueeze(0)
    res = {"weights": os.path.relpath(WEIGHTS, ROOT),
           "pair": {"plain": {"Mpixel_per_s": round(plain_value, 3), "inlier_F": round(plain_rate, 4)}}}
    for mode, use_tree in (("plain+learned", 1), ("learned", 0)):
        m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=4, eps=5, use_kdtree=use_tree)

        def once():
            pf, pb = proposal.proposals_both_ways(net, b1, b2)
            return m.run(img1, img2, seed=1000, proposal=(pf[0], pb[0]))

        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        assert m.status() == [0, 0, 0], m.status()
        res["pair"][mode] = {"Mpixel_per_s": round(W * H / ms / 1e3, 3),
                             "inlier_F": round(pairs.inlier_rate(out["F"].cpu().numpy(), pair, 4), 4)}
    ev = proposal.evaluate(net, eval_pairs, reps=3, log=lambda s: None)
    res["batch"] = {"workload": f"{len(eval_pairs)} held-out 1024x436 layered pairs (seeds {LEARNED_SEED0}.."
                                f"{LEARNED_SEED0 + len(eval_pairs) - 1}) in one batched call",
                    **{m: {"Mpixel_per_s": round(ev[m]["mpx_s"], 3), "inlier_F": round(ev[m]["inlier_F"], 4),
                           "inlier_filtered": round(ev[m]["inlier_filtered"], 4)}
                       for m in ("plain", "plain+learned", "learned")},
                    "network_alone_at_seed_points": round(ev["network_only_seed_points"], 4)}
    return res


def bench_batch(args, ff, prs, torch, dev):
    """64 pairs of mixed sizes: descriptors of all 128 images, one
    ff_match_batch call for all 192 fields, 64 consistency filters -- the
    whole batch captured in one HIP graph; against the same pairs run one
    pair per launch sequence (PairMatcher, three streams per pair)."""
    shapes = [(p.img1.shape[1], p.img1.shape[0]) for p in prs]
    i1 = [torch.from_numpy(p.img1).to(dev) for p in prs]
    i2 = [torch.from_numpy(p.img2).to(dev) for p in prs]
    seeds = [p.seed for p in prs]
    total_px = sum(w * h for w, h in shapes)
    ff.ff_init()
    m = ff.BatchMatcher(shapes)
    m.run(i1, i2, seeds=seeds)
    torch.cuda.synchronize()
    best_bh, best_pipe, tune_ms = m.autotune(i1, i2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        m.run(i1, i2, seeds=seeds)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        m.run(i1, i2, seeds=seeds)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert m.status() == 0
    ms_batch = (t1 - t0) * 1000.0 / args.steps
    # one pair per launch sequence, same pairs (buffers allocated up front)
    singles = [ff.PairMatcher(w, h, 3, r=8, r2=6, k=3, subpel=4, eps=5) for (w, h) in shapes]
    for i, sm in enumerate(singles):
        sm.run(i1[i], i2[i], seed=seeds[i], pair_id=i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        for i, sm in enumerate(singles):
            sm.run(i1[i], i2[i], seed=seeds[i], pair_id=i)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1000.0 / max(1, args.steps // 2)
    same = all(torch.equal(singles[i].flow["F"], m.out[i]["F"][0]) and
               torch.equal(singles[i].keep, m.out[i]["keep"]) for i in range(len(prs)))
    line = {
        "metric": "batched matching of mixed-size pairs: Mpixel/s and pairs/s, one batched call vs one pair "
                  "per launch",
        "value": round(total_px / (ms_batch / 1000.0) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_batch, 3),
        "pairs_per_s": round(len(prs) / (ms_batch / 1000.0), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{len(prs)} layered pairs of mixed sizes (320x240 to 1242x375, 2-8 layers), "
                               f"{total_px} px per batch; whole batch replayed from one HIP graph",
                   "band_rows": best_bh, "pipelined_sweep_pairs": bool(best_pipe)},
        "one_pair_per_launch": {"ms_per_batch": round(ms_single, 3),
                                "Mpixel_per_s": round(total_px / (ms_single / 1000.0) / 1e6, 3),
                                "pairs_per_s": round(len(prs) / (ms_single / 1000.0), 2)},
        "speedup_vs_one_pair_per_launch": round(ms_single / ms_batch, 3),
        "batch_equals_one_pair_path": bool(same),
    }
    print(json.dumps(line), flush=True)


OUTLIER_SEED0 = 1000
OUTLIER_EPS = (0.5, 1, 1.5, 2, 2.5, 3, 4, 5, 6, 8, 10, 15, 20)


def bench_outliers(args, ff, prs, torch, dev, outlier_px=5.0, s=50):
    """Figure 6 of the paper (section 4.1) on synthetic ground truth: for each
    epsilon, the share of outliers (end-point error above 5 px) and of
    inliers that a filter removes, for the one-way check (F against B1), the
    two-way check (B1 and B2) and the two-way check followed by the region
    filter (s = 50).  Over every pixel whose F is set (occluded ones
    included: their ground truth is defined), summed over the pairs."""
    import numpy as np
    Q = 4
    ff.ff_init()
    H, W = prs[0].img1.shape[:2]
    m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=Q, eps=5)
    keep = torch.empty((H, W), dtype=torch.uint8, device=dev)
    filt = torch.empty((H, W), dtype=torch.int32, device=dev)
    keep2 = torch.empty_like(keep)
    filt2 = torch.empty_like(filt)
    ws = torch.empty(ff.ff_region_filter_workspace_bytes(W, H), dtype=torch.uint8, device=dev)
    modes = ("one-way", "two-way", "two-way+region")
    tally = {mode: {e: [0, 0] for e in OUTLIER_EPS} for mode in modes}   # removed outliers, removed inliers
    n_out = n_in = 0
    for p in prs:
        out = m.run(torch.from_numpy(p.img1).to(dev), torch.from_numpy(p.img2).to(dev), seed=p.seed)
        torch.cuda.synchronize()
        assert m.status() == [0, 0, 0]
        F = out["F"].cpu().numpy()
        u = F.astype(np.int64) & 0xFFFFFFFF
        dx = (((u & 0xFFFF) ^ 0x8000) - 0x8000) / Q
        dy = ((((u >> 16) & 0xFFFF) ^ 0x8000) - 0x8000) / Q
        valid = F != ff.FF_EMPTY
        epe = np.hypot(dx - p.flow[..., 0], dy - p.flow[..., 1])
        outl = valid & (epe > outlier_px)
        inl = valid & ~outl
        n_out += int(outl.sum())
        n_in += int(inl.sum())
        for e in OUTLIER_EPS:
            for mode in modes:
                bwd = [out["B1"]] if mode == "one-way" else [out["B1"], out["B2"]]
                ff.ff_consistency_filter(out["F"], bwd, Q, int(round(e * Q)), keep, filt)
                k = keep
                if mode == "two-way+region":
                    ff.ff_region_filter(out["F"], keep, Q, s, keep2, filt2, ws)
                    k = keep2
                rem = k.cpu().numpy() == 0
                tally[mode][e][0] += int((rem & outl).sum())
                tally[mode][e][1] += int((rem & inl).sum())
    curve = {mode: [[e, round(100.0 * tally[mode][e][0] / max(n_out, 1), 3),
                     round(100.0 * tally[mode][e][1] / max(n_in, 1), 3)] for e in OUTLIER_EPS] for mode in modes}
    line = {"experiment": "removed outliers vs removed inliers over epsilon (the paper's Figure 6)",
            "workload": f"{len(prs)} layered 1024x436 pairs (seeds {OUTLIER_SEED0}..{OUTLIER_SEED0 + len(prs) - 1}), "
                        f"outlier = end-point error > {outlier_px} px, region filter s = {s}",
            "pixels_with_flow": n_out + n_in, "outlier_share_pct": round(100.0 * n_out / max(n_out + n_in, 1), 3),
            "curve_eps_removed_outliers_pct_removed_inliers_pct": curve}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
