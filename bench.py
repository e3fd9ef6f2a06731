#!/usr/bin/env python
"""Benchmark of the Flow Fields hot path on one MI355X.

One step = the whole path on one 1024x436 RGB pair (Sintel-shaped synthetic
pair, seeded): descriptors of both images, the three fields F = I1->I2 (r=8),
B1 = I2->I1 (r=8), B2 = I2->I1 (r2=6) each with its kd-tree, and the two-way
consistency filter (sections 3.1-3.4, parameters of section 4: k=3, R=1,
l=8, eps=5).  Inputs are resident in HBM before the timed region.

Prints one JSON line: the throughput (Mpixel/s = W*H / time per pair); the
dominant kernel's measured rate against its roofline; every other kernel
class against its own bound (algorithmic bytes per launch over the measured
launch time); the level-1 propagation sweep's time per wavefront step;
secondary workloads (the paper's fast variant, the skewed-motion recipe, the
path through the region filter and sparsification of sections 3.4-3.5, 64
mixed-size pairs in one batched call, the learned proposal); the path with
the SIFT-flow data term (section 3.3, the KITTI setting) on the KITTI-shaped
pair and the benchmark pair; and the CPU oracle on the same pair, split by
stage (and on a bounded sample of the SIFT-flow workload).
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
# single sweeps and pipelined sweep pairs), from FETCH_SIZE and WRITE_SIZE
# counter runs scaled by a plain-copy calibration; the counter runs are
# summarised in profiles/hotpath_1024x436_hbm_counters.md.  Valid for the
# k_propagate the summary names only.
PROPAGATE_HBM_BYTES_PER_LAUNCH = 74.38e6

K, R, R2, Q, EPS, LEAF = 3, 8, 6, 4, 5, 8
SPARSE_S, SPARSE_E = 50, 4            # section 4: s and e for Sintel
HEADLINE_SEED = 1000
LEARNED_SEED0 = 4000
OUTLIER_SEED0 = 1000
WEIGHTS = os.path.join(ROOT, "paper_1508_05151_amd", "weights", "proposal_1024x436.safetensors")
# the SIFT-flow data term with the paper's KITTI setting (section 4.2)
SIFT_R, SIFT_R2, SIFT_S, SIFT_S2, SIFT_EPS, SIFT_REGION_S, SIFT_E = 3, 2, 12, 18, 1, 150, 9
SIFT_SEED = 2000
SIFT_CPU_SAMPLE = (621, 188)          # the oracle's bounded sample: the same recipe at 1/4 of the pixels


def grid_points(W, H, k):
    return [((W + (1 << l) - 1) >> l) * ((H + (1 << l) - 1) >> l) for l in range(k + 1)]


def tree_depth(N, leaf):
    d = 0
    while (N + (1 << d) - 1) // (1 << d) > leaf:
        d += 1
    return d


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


def algorithmic_bytes(W, H, C=3, k=K, q=Q, n_radii=2, leaf=LEAF):
    """Bytes each kernel class must move per launch at this size: its inputs
    read once and its outputs written once (per image for the descriptor
    stages, per tree for the kd-tree)."""
    N = W * H
    return {
        "lab": N * (C + C),                                   # RGB in, Lab8 out
        "smooth": N * (C + (k + 1) * C * 2),                  # Lab8 in, (k+1) int16 levels out
        "census": N * ((k + 1) * C * 2 + 2 * (k + 1) * q * q * 4),   # levels in, planes in both layouts out
        "wht": N * (C + n_radii * 9 * C * 4),                 # Lab8 in, 9 C int32 per radius out
        "descriptors": N * (C + C + (k + 1) * C * 2 + 2 * (k + 1) * q * q * 4 + n_radii * 9 * C * 4),
        # the survey's bound for a median-split build: every level reads the
        # node's vectors (9 C int32) once
        "tree": tree_depth(N, leaf) * 9 * C * 4 * N,
        "filter": N * (4 + 2 * 4 + 1 + 4),                    # F, B1, B2 (looked up) in; keep, field out
        "region": N * (4 + 1 + 4 + 1 + 4),                    # F, keep in; names, mask, field out
        "sparsify": N * (4 + 2 * 4 + 4) + ((W + 2) // 3) * ((H + 2) // 3) * 4,   # field, 2 lookups, sparse, picks
    }


# ------------------------------------------------------------------ CPU oracle (rank 0 only)
def _oracle_stages(args):
    """One full run of the oracle on the pair, stage by stage, on one core."""
    img1, img2, core = args
    try:
        os.sched_setaffinity(0, {core})
    except (AttributeError, OSError):
        pass
    from oracle import ffo
    t = {}
    t0 = time.perf_counter()
    d1 = ffo.Desc(img1, K, Q, (R, R2))
    d2 = ffo.Desc(img2, K, Q, (R, R2))
    t["descriptors"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    for d, rad in ((d2, R), (d1, R), (d1, R2)):       # the trees of F, B1, B2 (each field builds its own)
        ffo.kdtree_build(d.wht(rad).reshape(-1, 27), LEAF)
    t["trees"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    F, _ = ffo.match_field(d1, d2, R, k=K, seed=HEADLINE_SEED, field_id=0)
    t["F"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    B1, _ = ffo.match_field(d2, d1, R, k=K, seed=HEADLINE_SEED, field_id=1)
    t["B1"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    B2, _ = ffo.match_field(d2, d1, R2, k=K, seed=HEADLINE_SEED, field_id=2)
    t["B2"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    keep, _ = ffo.consistency(F, [B1, B2], Q, EPS * Q)
    t["filter"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _, fr = ffo.region_filter(F, keep, Q, SPARSE_S)
    t["region_filter"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ffo.sparsify(fr, [B1, B2], Q, SPARSE_E)
    t["sparsify"] = time.perf_counter() - t0
    # the benchmark's step: descriptors, three fields (each with its tree), check
    t["path"] = t["descriptors"] + t["F"] + t["B1"] + t["B2"] + t["filter"]
    return t


def cpu_baseline(pair, reps=3):
    """The oracle (plain single-threaded C++) on the benchmark pair, `reps`
    runs side by side in processes pinned to distinct cores; median per
    stage.  Mpixel/s = W*H / median time of the benchmark's step."""
    import multiprocessing as mp
    cores = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else list(range(reps))
    jobs = [(pair.img1, pair.img2, cores[i % len(cores)]) for i in range(reps)]
    with mp.get_context("spawn").Pool(reps) as pool:
        runs = pool.map(_oracle_stages, jobs)
    med = {key: statistics.median(r[key] for r in runs) for key in runs[0]}
    H, W = pair.img1.shape[:2]
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(W * H / med["path"] / 1e6, 5), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole benchmark pair ({W}x{H}): descriptors x2, F, B1, B2 (each with its kd-tree), "
                      f"two-way check; median of {reps} single-threaded runs made side by side on distinct cores",
            "seconds_median": {k: round(v, 3) for k, v in med.items()},
            "host": {"cpu_model": model, "nproc": os.cpu_count(),
                     "cores_available": len(cores)}}


def sift_cpu_baseline():
    """The oracle's SIFT-flow path (colours, three fields, check, region
    filter, sparsification) on one core, on a bounded sample: the
    KITTI-shaped driving recipe (seed 2000) at 621x188 (1/4 of the pixels of
    the GPU workload, the same motions in pixels; the full pair takes the
    oracle about 100 s)."""
    from oracle import ffo
    from synth import pairs
    W, H = SIFT_CPU_SAMPLE
    p = pairs.driving_pair(SIFT_SEED, W=W, H=H)
    g1, g2 = p.img1.reshape(H, W), p.img2.reshape(H, W)
    t0 = time.perf_counter()
    ffo.match_pair_sift(g1, g2, r=SIFT_R, r2=SIFT_R2, S=SIFT_S, S2=SIFT_S2, eps=SIFT_EPS, seed=SIFT_SEED,
                        region_s=SIFT_REGION_S, sparse_e=SIFT_E)
    sec = time.perf_counter() - t0
    return {"value": round(W * H / sec / 1e6, 5), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"the KITTI-shaped gray driving recipe (seed {SIFT_SEED}) at {W}x{H} (1/4 of the GPU "
                      f"workload's pixels, the same motions in pixels): colours, F, B1, B2, check, region "
                      f"filter, sparsification; one single-threaded run", "seconds": round(sec, 3)}


def bench_sift(ff, torch, dev, workloads, steps):
    """The SIFT-flow path (section 3.3) with the paper's KITTI setting: Lab8
    and WHT vectors of both images, the pair's colours (dense SIFT, PCA to 18,
    codes) and their levels, F (r = 3, S = 12), B1 (r = 3, S = 12), B2 (r2 = 2,
    S2 = 18) in one batched call, consistency check (epsilon = 1), region
    filter (s = 150) and sparsification (e = 9)."""
    from synth import pairs
    res = {}
    for name, p in workloads.items():
        H, W = p.img1.shape[:2]
        C = p.img1.shape[2] if p.img1.ndim == 3 else 1
        a = torch.from_numpy(p.img1.reshape(H, W) if C == 1 else p.img1).to(dev)
        b = torch.from_numpy(p.img2.reshape(H, W) if C == 1 else p.img2).to(dev)
        m = ff.SiftPairMatcher(W, H, channels=C, r=SIFT_R, r2=SIFT_R2, S=SIFT_S, S2=SIFT_S2, k=K, subpel=Q,
                               eps=SIFT_EPS, region_s=SIFT_REGION_S, sparse_e=SIFT_E)
        run = lambda: m.run(a, b, seed=p.seed)
        run()
        torch.cuda.synchronize()
        ms, per, out = time_steps(run, torch, steps)
        assert m.status() == 0, m.status()
        classes = ["sift_colors", "sift_pca", "sift_levels", "sift_match", "tree", "filter", "region", "sparsify"]
        t = class_times(ff, run, torch, classes, reps=3)
        ff.ff_profile_begin("sift_propagate", 64)
        run()
        torch.cuda.synchronize()
        ptot, pn, each = ff.ff_profile_end(each=16)
        # level 0's four sweeps are the last launches; a sweep runs about
        # Gw + Gh wavefront steps (4-row bands, each one step behind per row)
        lvl0 = statistics.median(each[-4:])
        wsteps = W + H
        # bytes the sweep's loads request per point: per candidate the two
        # sliding rows or columns of 2r+1 samples, 5 pixels each (source and
        # the bilinear target quad) of 2S bytes, for F, B1 and B2
        req = sum(2 * 2 * (2 * r + 1) * 5 * 2 * S for r, S in ((SIFT_R, SIFT_S), (SIFT_R, SIFT_S), (SIFT_R2, SIFT_S2)))
        res[name] = {
            "Mpixel_per_s": round(W * H / ms / 1e3, 3), "ms_per_pair": round(ms, 4),
            "median_ms_per_pair": round(statistics.median(per), 4),
            "stages_ms_per_pair": {c: round(t[c][0] * t[c][1], 4) for c in classes},
            "propagation": {"kernel": "k_sift_prop", "launches_per_pair": pn, "ms_per_pair": round(ptot, 4),
                            "level0_sweep_ms": round(lvl0, 4), "wavefront_steps_level0": wsteps,
                            "ns_per_wavefront_step": round(lvl0 * 1e6 / wsteps, 1),
                            "requested_bytes_per_point_three_fields": req,
                            "requested_GBps_level0": round(req * W * H / (lvl0 / 1000.0) / 1e9, 1),
                            "bound": "the sweep's dependency chain: one memory round trip per wavefront step"},
            "quality": {"F_inlier_rate_epe_lt_3px": round(pairs.inlier_rate(out["F"].cpu().numpy(), p, Q), 4),
                        "kept_after_filters": round(out["keep_region"].float().mean().item(), 4),
                        "filtered_inlier_rate_epe_lt_3px": round(
                            pairs.inlier_rate(out["filtered_region"].cpu().numpy(), p, Q), 4),
                        "sparse_samples": int((out["pick"] >= 0).sum().item())}}
        del m
        # the census data term on the same pair (r = 8, r2 = 6; epsilon 1 on
        # gray, as the KITTI setting), for the accuracy comparison
        cm = ff.PairMatcher(W, H, C, r=R, r2=R2, k=K, subpel=Q, eps=EPS if C == 3 else SIFT_EPS)
        crun = lambda: cm.run(a, b, seed=p.seed)
        crun()
        cms, _, cout = time_steps(crun, torch, steps)
        assert cm.status() == [0, 0, 0], cm.status()
        res[name]["census_same_pair"] = {
            "Mpixel_per_s": round(W * H / cms / 1e3, 3),
            "F_inlier_rate_epe_lt_3px": round(pairs.inlier_rate(cout["F"].cpu().numpy(), p, Q), 4)}
        del cm
    return res


# ------------------------------------------------------------------ GPU timing helpers
def time_steps(run, torch, steps):
    """Wall time per step of `run` (K steps between synchronisations) and
    the per-step event times."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for i in range(steps):
        starts[i].record()
        out = run()
        ends[i].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1000.0 / steps, [s.elapsed_time(e) for s, e in zip(starts, ends)], out


def class_times(ff, run, torch, classes, reps=5, per_step=64):
    """Average launch time (ms) and launches per step of each kernel class,
    each from its own profiled run of `reps` steps."""
    res = {}
    for c in classes:
        torch.cuda.synchronize()
        ff.ff_profile_begin(c, per_step * reps)
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        tot, n, _ = ff.ff_profile_end()
        res[c] = (tot / max(n, 1), n / reps)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-reps", type=int, default=3, help="CPU baseline: oracle runs (side by side)")
    ap.add_argument("--mode", default="pair", choices=("pair", "batch", "outliers", "ablation", "sift", "frontier"),
                    help="pair: one 1024x436 pair (headline, with every secondary block); batch: 64 mixed-size "
                         "pairs in one batched call alone; outliers: removed outliers vs removed inliers of the "
                         "filters over epsilon; ablation: the measures of Table 1 over k, l, R and the fast "
                         "variant; sift: the SIFT-flow data term path alone (KITTI setting); frontier: "
                         "throughput against inlier rate over the kd-tree leaf size, with and without the "
                         "learned proposal")
    ap.add_argument("--pairs", type=int, default=64, help="batch block: number of mixed-size pairs")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes drawing the synthetic pairs (0 = in-process; use 0 under a profiler)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--no-sift", action="store_true", help="skip the SIFT-flow data term block")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-pair batch block")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the per-kernel table and the secondary workloads")
    ap.add_argument("--learned-pairs", type=int, default=16,
                    help="held-out 1024x436 pairs of the learned-proposal comparison")
    ap.add_argument("--outlier-pairs", type=int, default=8,
                    help="outliers mode: layered 1024x436 pairs (seeds 1000..)")
    ap.add_argument("--band-rows", type=int, default=16, choices=(8, 16, 32),
                    help="propagation band height of the headline pair (results are identical for every value)")
    ap.add_argument("--pipeline", type=int, default=1, choices=(0, 1),
                    help="pipelined sweep pairs on the headline pair (results are identical)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (the reference dispatch "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU: the build matches each pair on one MI355X "
                                   "and runs no multi-GPU path; --gpus must be 1"}), flush=True)
        sys.exit(2)

    from synth import pairs
    # synthetic pairs are drawn before anything touches the GPU (worker
    # processes are started from a process that has not initialised it)
    batch_pairs = eval_pairs = outlier_pairs = None
    if args.mode in ("outliers", "ablation"):
        outlier_pairs = pairs.layered_pairs(OUTLIER_SEED0, args.outlier_pairs, workers=args.gen_workers)
    if args.mode == "ablation":
        outlier_pairs = {
            "layered 1024x436, translations U(+-200) px, noise 2": outlier_pairs,
            "layered 1024x436, translations U(+-200) px, noise 12": pairs.layered_pairs(
                OUTLIER_SEED0, args.outlier_pairs, workers=args.gen_workers, noise=12.0),
            "layered 1024x436, smooth 1/f^2 textures, translations U(+-200) px, noise 4": pairs.layered_pairs(
                OUTLIER_SEED0, args.outlier_pairs, workers=args.gen_workers, noise=4.0, beta=2.0),
            "layered 1024x436, smooth 1/f^2.5 textures, translations U(+-200) px, noise 6": pairs.layered_pairs(
                OUTLIER_SEED0, args.outlier_pairs, workers=args.gen_workers, noise=6.0, beta=2.5),
            "KITTI-shaped 1242x375 gray (radial expansion to 250 px, flat regions, noise 3)": pairs.driving_pairs(
                2000, args.outlier_pairs, workers=args.gen_workers)}
    if args.mode == "batch" or (args.mode == "pair" and not args.no_batch):
        batch_pairs = (pairs.mixed_pairs_parallel(args.pairs, workers=args.gen_workers) if args.gen_workers > 0
                       else pairs.mixed_pairs(args.pairs))
    if args.mode == "frontier" or (args.mode == "pair" and not args.no_learned):
        eval_pairs = pairs.layered_pairs(LEARNED_SEED0, args.learned_pairs, workers=args.gen_workers)
    pair = pairs.layered_pair(HEADLINE_SEED)
    skewed = pairs.layered_pair(HEADLINE_SEED, motion="skewed") if args.mode == "pair" else None
    cpu = None
    if args.mode == "pair" and not args.no_cpu:
        cpu = cpu_baseline(pair, args.cpu_reps)
    sift_workloads = sift_cpu = None
    if args.mode == "sift" or (args.mode == "pair" and not args.no_sift):
        sift_workloads = {"driving_1242x375_gray": pairs.driving_pair(SIFT_SEED),
                          "layered_1024x436_rgb": pair}
        if not args.no_cpu:
            sift_cpu = sift_cpu_baseline()

    import torch
    from paper_1508_05151_amd import ff

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ff.ff_init()
    if args.mode == "batch":
        print(json.dumps(bench_batch(args, ff, batch_pairs, torch, dev)), flush=True)
        return
    if args.mode == "outliers":
        return bench_outliers(args, ff, outlier_pairs, torch, dev)
    if args.mode == "ablation":
        return bench_ablation(args, ff, outlier_pairs, torch, dev)
    if args.mode == "frontier":
        return bench_frontier(args, ff, pair, eval_pairs, torch, dev)
    if args.mode == "sift":
        res = bench_sift(ff, torch, dev, sift_workloads, args.steps)
        d = res["driving_1242x375_gray"]
        line = {"metric": "SIFT-flow data term path, Mpixel/s (KITTI setting, section 4.2)",
                "value": d["Mpixel_per_s"], "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": d["ms_per_pair"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "int16/int32 (colours fp32/fp64)",
                "data": "synthetic", "config": {"workload": "KITTI-shaped 1242x375 gray driving pair (seed 2000)",
                                                "r": SIFT_R, "r2": SIFT_R2, "S": SIFT_S, "S2": SIFT_S2,
                                                "eps": SIFT_EPS, "s": SIFT_REGION_S, "e": SIFT_E, "k": K,
                                                "subpel": Q},
                "workloads": res}
        if sift_cpu is not None:
            line["cpu_baseline"] = sift_cpu
        print(json.dumps(line), flush=True)
        return
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    H, W, C = pair.img1.shape
    img1 = torch.from_numpy(pair.img1).to(dev)
    img2 = torch.from_numpy(pair.img2).to(dev)
    m = ff.PairMatcher(W, H, C, r=R, r2=R2, k=K, subpel=Q, eps=EPS, band_rows=args.band_rows,
                       pipeline=args.pipeline)
    run = lambda: m.run(img1, img2, seed=HEADLINE_SEED)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    if args.warmup:
        assert m.status() == [0, 0, 0], m.status()

    # timed region: K whole-path steps; the dominant kernel class is bracketed
    # with HIP events on the streams it runs on (library profiling hook), and
    # each of its launches is timed
    per_field = 9 if args.pipeline else 12
    ff.ff_profile_begin("propagate", 3 * 16 * args.steps + 8)
    ms_per_step, per_step, out = time_steps(run, torch, args.steps)
    tot, nl, each = ff.ff_profile_end(each=3 * per_field * args.steps)
    assert m.status() == [0, 0, 0], m.status()
    value = W * H / (ms_per_step / 1000.0) / 1e6

    # dominant kernel against its roofline (integer VALU: census terms)
    avg_launch_ms = tot / max(nl, 1)
    ops_per_launch = (propagate_ops_per_pair(W, H, K, (R, R, R2)) +
                      per_point_ops_in_sweep_launches(W, H, K, (R, R, R2))) / (nl / args.steps)
    achieved = ops_per_launch / (avg_launch_ms / 1000.0) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(INT_PEAK_TOPS, 2), "unit": "TOP/s",
            "frac": round(achieved / INT_PEAK_TOPS, 5), "traffic": PROPAGATE_HBM_BYTES_PER_LAUNCH,
            "traffic_GBps": round(PROPAGATE_HBM_BYTES_PER_LAUNCH / (avg_launch_ms / 1000.0) / 1e9, 2),
            "kernel": "k_propagate", "avg_launch_ms": round(avg_launch_ms, 4), "launches": nl,
            "ops_per_launch": int(ops_per_launch)}

    keep = out["keep"].float().mean().item()
    rate = pairs.inlier_rate(out["F"].cpu().numpy(), pair, Q)
    line = {
        "metric": "flow-field Mpixel/s at 1024×436, plain vs learned proposal; % of HBM roofline",
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
        "config": {"workload": "one 1024x436 RGB Sintel-shaped layered pair (seed 1000, 6 layers, translations "
                               "U(+-200) px): descriptors x2, F/B1/B2 fields with kd-trees, two-way consistency "
                               "filter",
                   "k": K, "r": R, "r2": R2, "R": 1, "leaf": LEAF, "subpel": Q, "eps": EPS,
                   "band_rows": args.band_rows, "pipelined_sweep_pairs": bool(args.pipeline)},
        "roofline": roof,
        "quality": {"F_inlier_rate_epe_lt_3px": round(rate, 4), "kept_fraction": round(keep, 4),
                    "occluded_fraction": round(float(pair.occluded.mean()), 4)},
    }
    if not args.no_secondary:
        line["kernels"] = kernel_table(ff, run, torch, W, H, C, img=img1)
        if args.pipeline and len(each) >= 3 * per_field:
            line["level1_sweep"] = level1_sweep(each, per_field, args.steps, W, H, args.band_rows)
            line["level1_sweep"]["latency_floor"] = latency_floor(ff, torch, dev, line["level1_sweep"])
        line["secondary"] = secondary(ff, torch, dev, pair, skewed, args.steps)
    if batch_pairs is not None:
        line["batch"] = bench_batch(args, ff, batch_pairs, torch, dev, steps=5)
    if eval_pairs is not None:
        line["learned_proposal"] = bench_learned(ff, pair, img1, img2, eval_pairs, torch, dev, value, rate)
    if sift_workloads is not None:
        line["sift_flow"] = bench_sift(ff, torch, dev, sift_workloads, steps=5)
        if sift_cpu is not None:
            line["sift_flow"]["cpu_baseline"] = sift_cpu
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def kernel_table(ff, run, torch, W, H, C, img=None):
    """Every kernel class of the step against its own bound: algorithmic
    bytes per launch over the measured launch time, against the HBM peak.
    In the step the two images' descriptors share the GPU; the descriptor
    classes are also timed for one image alone (`alone_*`)."""
    ab = algorithmic_bytes(W, H, C)
    classes = ["lab", "smooth", "census", "wht", "descriptors", "tree", "seed", "level_entry", "random_search",
               "filter"]
    t = class_times(ff, run, torch, classes)
    alone = {}
    if img is not None:
        d = ff.ff_desc_init(W, H, C, K, Q, (R, R2))
        blob = torch.empty(d.bytes, dtype=torch.uint8, device=img.device)
        alone = class_times(ff, lambda: ff.ff_compute_descriptors(d, img, blob), torch,
                            ["lab", "smooth", "census", "wht", "descriptors"], reps=10)
    table = {}
    for c in classes:
        ms, per = t[c]
        row = {"avg_launch_ms": round(ms, 4), "launches_per_step": round(per, 2)}
        if per == 0 and c == "descriptors":
            row["note"] = ("in the step the descriptors are two calls per image, Lab8 + WHT and then levels + "
                           "census, with the kd-trees started between them: see the lab, smooth, census and wht "
                           "rows; the whole call is timed alone")
            if c in alone:
                gba = ab[c] / (alone[c][0] / 1000.0) / 1e9
                row.update(bound="hbm", algorithmic_bytes=ab[c], alone_ms=round(alone[c][0], 4),
                           alone_GBps=round(gba, 1), alone_frac=round(gba / HBM_PEAK_GBS, 4))
        elif per == 0:
            row["note"] = "no launch of its own: runs inside the pipelined sweep launches"
        elif c in ab:
            gbs = ab[c] / (ms / 1000.0) / 1e9
            row.update(bound="hbm", algorithmic_bytes=ab[c], GBps=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
            if c in alone:
                gba = ab[c] / (alone[c][0] / 1000.0) / 1e9
                row.update(alone_ms=round(alone[c][0], 4), alone_GBps=round(gba, 1),
                           alone_frac=round(gba / HBM_PEAK_GBS, 4))
        else:
            row.update(bound="alu/latency")
        table[c] = row
    return table


def level1_sweep(each, per_field, steps, W, H, bh):
    """The last propagation launch of each field is level 1's single sweep
    (pipelined schedule): its time per wavefront step.  A band starts
    skew + 2 steps after the band above (the skew of its rows plus two steps
    of hand-off lookahead) and runs Gw + skew steps."""
    sweeps = [each[s * 3 * per_field + f * per_field + per_field - 1] for s in range(steps) for f in range(3)]
    ms = statistics.median(sweeps)
    bands = (H + bh - 1) // bh
    skew = bh - 1 + (bh - 1) // 4
    wave_steps = W + skew + (skew + 2) * (bands - 1)
    return {"median_ms": round(ms, 4), "wavefront_steps": wave_steps,
            "ns_per_step": round(ms * 1e6 / wave_steps, 1),
            "cycles_per_step_at_2.4GHz": round(ms * 1e-3 * CLOCK_GHZ * 1e9 / wave_steps, 0)}


def load_round_trip_ns(ff, torch, dev, n_ints, hops=20000, reps=5):
    """One dependent global load's round trip (ns), median of `reps` timed
    walks of a cycle over the first word of every 128-byte line of an
    n_ints buffer (warmed by two passes over it first)."""
    nxt = torch.from_numpy(ff.load_cycle(n_ints)).to(dev)
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    lines = n_ints // 32
    res = []
    for _ in range(reps):
        ff.ff_probe_load_latency(nxt, 2 * lines, hops, out)
        torch.cuda.synchronize()
        res.append(out[0].item() * 10.0 / hops)
    return statistics.median(res)


def latency_floor(ff, torch, dev, sweep):
    """The sweep's latency floor: a step's result decides the next step's
    target addresses, so every wavefront step costs at least one dependent
    round trip to the cache that holds the census words (L2 for a cycle of
    1 MB, L1 for one of 16 KB, both measured here on one thread)."""
    l1 = load_round_trip_ns(ff, torch, dev, 4096)
    l2 = load_round_trip_ns(ff, torch, dev, 1 << 18)
    floor_ms = sweep["wavefront_steps"] * l2 * 1e-6
    return {"l1_round_trip_ns": round(l1, 1), "l2_round_trip_ns": round(l2, 1),
            "l2_round_trip_cycles_at_2.4GHz": round(l2 * CLOCK_GHZ, 0),
            "floor_ms_one_l2_round_trip_per_step": round(floor_ms, 4),
            "floor_over_measured": round(floor_ms / sweep["median_ms"], 4),
            "note": "the level-1 sweep's wavefront steps x one dependent L2 round trip, against its measured time"}


def secondary(ff, torch, dev, pair, skewed, steps):
    """The paper's fast variant (r = 6, one backward field, section 4.2),
    the benchmark step replayed from a HIP graph, the skewed-motion recipe,
    and the path through the region filter and the sparsification (sections
    3.4, 3.5)."""
    from synth import pairs
    H, W, C = pair.img1.shape
    res = {}
    i1, i2 = torch.from_numpy(pair.img1).to(dev), torch.from_numpy(pair.img2).to(dev)

    def measure(m, a, b, p):
        run = lambda: m.run(a, b, seed=p.seed)
        run()
        ms, _, out = time_steps(run, torch, steps)
        assert all(s == 0 for s in m.status()), m.status()
        return ms, out

    fast = ff.PairMatcher(W, H, C, r=6, r2=6, k=K, subpel=Q, eps=EPS, n_bwd=1)
    ms, out = measure(fast, i1, i2, pair)
    res["fast_variant"] = {"workload": "the benchmark pair with r = 6 and one backward field (section 4.2)",
                           "Mpixel_per_s": round(W * H / ms / 1e3, 3), "ms_per_pair": round(ms, 4),
                           "F_inlier_rate_epe_lt_3px": round(pairs.inlier_rate(out["F"].cpu().numpy(), pair, Q), 4)}
    del fast
    # the same step captured in one HIP graph (the three field streams forked
    # from and joined to the capturing stream) and replayed: no launch gaps
    # between a field's dependent kernels; outputs checked against eager
    mg = ff.PairMatcher(W, H, C, r=R, r2=R2, k=K, subpel=Q, eps=EPS)
    out = mg.run(i1, i2, seed=pair.seed)
    torch.cuda.synchronize()
    eager = {k: out[k].clone() for k in ("F", "B1", "B2", "filtered")}
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=gs):
        gout = mg.run(i1, i2, seed=pair.seed)
    g.replay()
    ms, _, _ = time_steps(g.replay, torch, steps)
    assert all(s == 0 for s in mg.status()), mg.status()
    same = all(torch.equal(gout[k], eager[k]) for k in eager)
    res["graph_replay"] = {"workload": "the benchmark step captured in one HIP graph and replayed",
                           "Mpixel_per_s": round(W * H / ms / 1e3, 3), "ms_per_pair": round(ms, 4),
                           "equals_eager": same}
    del g, mg
    m = ff.PairMatcher(W, H, C, r=R, r2=R2, k=K, subpel=Q, eps=EPS)
    s1, s2 = torch.from_numpy(skewed.img1).to(dev), torch.from_numpy(skewed.img2).to(dev)
    ms, out = measure(m, s1, s2, skewed)
    res["skewed_motion_recipe"] = {
        "workload": "seed 1000 with layer translations 200 u v^2 per axis (u, v ~ U(-1, 1)): mostly small motions",
        "Mpixel_per_s": round(W * H / ms / 1e3, 3), "ms_per_pair": round(ms, 4),
        "F_inlier_rate_epe_lt_3px": round(pairs.inlier_rate(out["F"].cpu().numpy(), skewed, Q), 4),
        "occluded_fraction": round(float(skewed.occluded.mean()), 4)}
    del m
    mf = ff.PairMatcher(W, H, C, r=R, r2=R2, k=K, subpel=Q, eps=EPS, region_s=SPARSE_S, sparse_e=SPARSE_E)
    ms, out = measure(mf, i1, i2, pair)
    ab = algorithmic_bytes(W, H, C)
    run = lambda: mf.run(i1, i2, seed=pair.seed)
    t = class_times(ff, run, torch, ["region", "sparsify"])
    kept = out["keep_region"].float().mean().item()
    res["with_region_filter_and_sparsification"] = {
        "workload": f"the benchmark step followed by the region filter (s = {SPARSE_S}) and the sparsification "
                    f"(e = {SPARSE_E})",
        "Mpixel_per_s": round(W * H / ms / 1e3, 3), "ms_per_pair": round(ms, 4),
        "kept_after_region_filter": round(kept, 4), "samples": int((out["pick"] >= 0).sum().item()),
        "kernels": {c: {"avg_launch_ms": round(t[c][0], 4), "algorithmic_bytes": ab[c],
                        "GBps": round(ab[c] / (t[c][0] / 1000.0) / 1e9, 1),
                        "frac": round(ab[c] / (t[c][0] / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)} for c in t}}
    return res


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
        m = ff.PairMatcher(W, H, 3, r=R, r2=R2, k=K, subpel=Q, eps=EPS, use_kdtree=use_tree)

        def once():
            pf, pb = proposal.proposals_both_ways(net, b1, b2)
            return m.run(img1, img2, seed=HEADLINE_SEED, proposal=(pf[0], pb[0]))

        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        assert m.status() == [0, 0, 0], m.status()
        res["pair"][mode] = {"Mpixel_per_s": round(W * H / ms / 1e3, 3),
                             "inlier_F": round(pairs.inlier_rate(out["F"].cpu().numpy(), pair, Q), 4)}
    res["network"] = network_kernels(ff, net, eval_pairs, torch, dev)
    ev = proposal.evaluate(net, eval_pairs, reps=3, log=lambda s: None)
    res["batch"] = {"workload": f"{len(eval_pairs)} held-out 1024x436 layered pairs (seeds {LEARNED_SEED0}.."
                                f"{LEARNED_SEED0 + len(eval_pairs) - 1}) in one batched call",
                    **{m: {"Mpixel_per_s": round(ev[m]["mpx_s"], 3), "inlier_F": round(ev[m]["inlier_F"], 4),
                           "inlier_filtered": round(ev[m]["inlier_filtered"], 4)}
                       for m in ("plain", "plain+learned", "learned")},
                    "network_alone_at_seed_points": round(ev["network_only_seed_points"], 4)}
    return res


FRONTIER = (("plain", 8), ("plain", 4), ("plain", 16), ("plain", 32), ("plain", 64), ("plain+learned", 4),
            ("plain+learned", 8), ("plain+learned", 16), ("plain+learned", 32), ("plain+learned", 64),
            ("learned", 8))


def bench_frontier(args, ff, pair, eval_pairs, torch, dev, steps=10):
    """The learned proposal as a trade: for each kd-tree leaf size l (a
    larger leaf: a shallower tree, more seed candidates per point) with and
    without the network's candidate, and the network alone (no tree), the
    whole step's throughput on the benchmark pair (network forward inside the
    timed region where used) and the EPE < 3 px rate of F over the benchmark
    pair and the held-out pairs (seeds 4000..), each matched on its own."""
    from paper_1508_05151_amd import proposal
    from synth import pairs
    net = proposal.load(WEIGHTS)
    H, W = pair.img1.shape[:2]
    held = [pair] + list(eval_pairs)
    imgs = [(torch.from_numpy(p.img1).to(dev), torch.from_numpy(p.img2).to(dev)) for p in held]
    rows = []
    for mode, leaf in FRONTIER:
        m = ff.PairMatcher(W, H, 3, r=R, r2=R2, k=K, subpel=Q, eps=EPS, leaf=leaf,
                           use_kdtree=0 if mode == "learned" else 1)

        def once(i1, i2, seed):
            prop = None
            if mode != "plain":
                pf, pb = proposal.proposals_both_ways(net, i1.unsqueeze(0), i2.unsqueeze(0))
                prop = (pf[0], pb[0])
            return m.run(i1, i2, seed=seed, proposal=prop)

        i1, i2 = imgs[0]
        once(i1, i2, HEADLINE_SEED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            once(i1, i2, HEADLINE_SEED)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        rates = []
        for p, (a, b) in zip(held, imgs):
            out = once(a, b, p.seed)
            rates.append(pairs.inlier_rate(out["F"].cpu().numpy(), p, Q))
        assert m.status() == [0, 0, 0], m.status()
        rows.append({"mode": mode, "leaf": leaf, "ms_per_pair": round(ms, 4),
                     "Mpixel_per_s": round(W * H / ms / 1e3, 3), "inlier_F_benchmark_pair": round(rates[0], 4),
                     "inlier_F_mean": round(float(sum(rates) / len(rates)), 4)})
        del m
    base = rows[0]
    line = {"metric": "learned-proposal frontier: whole-step Mpixel/s against the EPE < 3 px rate of F",
            "unit": "Mpixel/s", "n_gpus": 1, "steps": steps, "dtype": "int32 (network bf16)", "data": "synthetic",
            "config": {"workload": f"the benchmark pair (seed {HEADLINE_SEED}) timed; the rate over it and "
                                   f"{len(eval_pairs)} held-out layered 1024x436 pairs (seeds {LEARNED_SEED0}..)",
                       "k": K, "r": R, "r2": R2, "subpel": Q, "eps": EPS},
            "rows": rows,
            "dominating_plain_l8": [r for r in rows[1:] if r["Mpixel_per_s"] > base["Mpixel_per_s"]
                                    and r["inlier_F_mean"] >= base["inlier_F_mean"]]}
    print(json.dumps(line), flush=True)


NET_LAYERS = ((6, 32, 2, 1), (32, 32, 2, 1), (32, 32, 2, 1), (32, 32, 1, 4), (32, 32, 1, 8), (32, 2, 1, 1))
BF16_PEAK_TFLOPS = 2500.0    # dense bf16 MFMA


def net_flops(W, H):
    """Multiply-adds x 2 of one forward pass (the convolutions' products)."""
    f = 0
    for ci, co, st, _ in NET_LAYERS:
        W, H = (W + st - 1) // st, (H + st - 1) // st
        f += 2 * 9 * ci * co * W * H
    return f


def network_kernels(ff, net, eval_pairs, torch, dev, reps=10):
    """The network's forward pass over the batch (both directions, as the
    learned modes run it) and one training step of the batch, against the
    dense bf16 MFMA peak."""
    import numpy as np
    from paper_1508_05151_amd import proposal
    H, W = eval_pairs[0].img1.shape[:2]
    i1 = torch.from_numpy(np.stack([p.img1 for p in eval_pairs])).to(dev)
    i2 = torch.from_numpy(np.stack([p.img2 for p in eval_pairs])).to(dev)
    B = i1.shape[0]
    proposal.proposals_both_ways(net, i1, i2)
    torch.cuda.synchronize()
    ff.ff_profile_begin("proposal", reps + 2)
    for _ in range(reps):
        proposal.proposals_both_ways(net, i1, i2)
    torch.cuda.synchronize()
    tot, n, _ = ff.ff_profile_end()
    fwd_ms = tot / max(n, 1)
    flops = net_flops(W, H) * 2 * B
    hc, wc = ff.seed_grid(W, H)
    labels = torch.zeros((B, hc, wc), dtype=torch.int32, device=dev)
    g = ff.ProposalNet(net.params.detach().clone(), device=dev)
    g.gradient(i1, i2, labels)
    torch.cuda.synchronize()
    ff.ff_profile_begin("train", reps + 2)
    for _ in range(reps):
        g.gradient(i1, i2, labels)
    torch.cuda.synchronize()
    tot, n, _ = ff.ff_profile_end()
    tr_ms = tot / max(n, 1)
    achieved = flops / (fwd_ms / 1000.0) / 1e12
    return {"forward_both_directions_ms": round(fwd_ms, 4), "pairs": B,
            "forward_gflop": round(flops / 1e9, 3), "forward_TFLOPs": round(achieved, 2),
            "forward_frac_of_bf16_peak": round(achieved / BF16_PEAK_TFLOPS, 4),
            "train_step_ms": round(tr_ms, 4),
            "note": "3x3 convolutions of 32 channels at 1/2 to 1/8 resolution: memory- and latency-bound, "
                    "about 40 FLOP per byte of activations"}


def bench_batch(args, ff, prs, torch, dev, steps=None):
    """64 pairs of mixed sizes: descriptors of all 128 images, one
    ff_match_batch call for all 192 fields, 64 consistency filters -- the
    whole batch captured in one HIP graph; against the same pairs run one
    pair per launch sequence (PairMatcher, three streams per pair)."""
    steps = steps or args.steps
    shapes = [(p.img1.shape[1], p.img1.shape[0]) for p in prs]
    i1 = [torch.from_numpy(p.img1).to(dev) for p in prs]
    i2 = [torch.from_numpy(p.img2).to(dev) for p in prs]
    seeds = [p.seed for p in prs]
    total_px = sum(w * h for w, h in shapes)
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
    for _ in range(max(args.warmup, 1)):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert m.status() == 0
    ms_batch = (t1 - t0) * 1000.0 / steps
    # one pair per launch sequence, same pairs (buffers allocated up front)
    singles = [ff.PairMatcher(w, h, 3, r=R, r2=R2, k=K, subpel=Q, eps=EPS) for (w, h) in shapes]
    for i, sm in enumerate(singles):
        sm.run(i1[i], i2[i], seed=seeds[i], pair_id=i)
    torch.cuda.synchronize()
    reps = max(1, steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        for i, sm in enumerate(singles):
            sm.run(i1[i], i2[i], seed=seeds[i], pair_id=i)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1000.0 / reps
    same = all(torch.equal(singles[i].flow[f], m.out[i][f][0]) and torch.equal(singles[i].cost[f], m.out[i][f][1])
               for i in range(len(prs)) for f in ("F", "B1", "B2")) and \
        all(torch.equal(singles[i].keep, m.out[i]["keep"]) and torch.equal(singles[i].filtered, m.out[i]["filtered"])
            for i in range(len(prs)))
    del singles
    return {
        "metric": "batched matching of mixed-size pairs: Mpixel/s and pairs/s, one batched call vs one pair "
                  "per launch",
        "value": round(total_px / (ms_batch / 1000.0) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1, "steps": steps,
        "ms_per_step": round(ms_batch, 3),
        "pairs_per_s": round(len(prs) / (ms_batch / 1000.0), 2),
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{len(prs)} layered pairs of mixed sizes (320x240 to 1242x375, 2-8 layers, seeds "
                               f"3000..{3000 + len(prs) - 1}), {total_px} px per batch; descriptors, all fields in "
                               f"one ff_match_batch call, filters; whole batch replayed from one HIP graph",
                   "band_rows": best_bh, "pipelined_sweep_pairs": bool(best_pipe),
                   "autotune": "band height x sweep-pair pipelining, fastest of 6 on this batch"},
        "one_pair_per_launch": {"ms_per_batch": round(ms_single, 3),
                                "Mpixel_per_s": round(total_px / (ms_single / 1000.0) / 1e6, 3),
                                "pairs_per_s": round(len(prs) / (ms_single / 1000.0), 2)},
        "speedup_vs_one_pair_per_launch": round(ms_single / ms_batch, 3),
        "batch_equals_one_pair_path": bool(same),
    }


OUTLIER_EPS = (0.5, 1, 1.5, 2, 2.5, 3, 4, 5, 6, 8, 10, 15, 20)


def bench_outliers(args, ff, prs, torch, dev, outlier_px=5.0, s=SPARSE_S):
    """Figure 6 of the paper (section 4.1) on synthetic ground truth: for each
    epsilon, the share of outliers (end-point error above 5 px) and of
    inliers that a filter removes, for the one-way check (F against B1), the
    two-way check (B1 and B2) and the two-way check followed by the region
    filter (s = 50).  Over every pixel whose F is set (occluded ones
    included: their ground truth is defined), summed over the pairs."""
    import numpy as np
    H, W = prs[0].img1.shape[:2]
    m = ff.PairMatcher(W, H, 3, r=R, r2=R2, k=K, subpel=Q, eps=EPS)
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


ABLATION = (
    ("k=3 (paper's setting)", dict(k=3)),
    ("k=2", dict(k=2)),
    ("k=1", dict(k=1)),
    ("k=0 (no hierarchy)", dict(k=0)),
    ("k=3, l=4", dict(k=3, leaf=4)),
    ("k=3, l=16", dict(k=3, leaf=16)),
    ("k=3, R=2", dict(k=3, R=2)),
    ("k=3, r=6, one backward field (fast variant)", dict(k=3, r=6, r2=6, n_bwd=1)),
)


def bench_ablation(args, ff, workloads, torch, dev):
    """The measures of Table 1 (section 4.1) on synthetic ground truth for
    the settings the paper varies: the share of F's flows within 3 px of the
    truth, the end-point error bounded at 10 px per flow (EPE10) and the raw
    end-point error, over non-occluded pixels, plus the kept share and the
    throughput of the whole path.  An empty flow counts as wrong, with an
    error of 10 px in EPE10 and left out of EPE.  One table per workload."""
    tables = {name: ablation_rows(ff, prs, torch, dev) for name, prs in workloads.items()}
    line = {"experiment": "Table 1's measures over the search settings on synthetic ground truth",
            "workload": f"{args.outlier_pairs} pairs per workload, non-occluded pixels; throughput of the whole "
                        f"path per pair",
            "tables": tables}
    print(json.dumps(line), flush=True)


def ablation_rows(ff, prs, torch, dev):
    import numpy as np
    H, W, C = prs[0].img1.shape if prs[0].img1.ndim == 3 else (*prs[0].img1.shape, 1)
    eps = 1 if C == 1 else EPS
    rows = []
    for name, kw in ABLATION:
        kk, r, r2, nb = kw.get("k", K), kw.get("r", R), kw.get("r2", R2), kw.get("n_bwd", 2)
        m = ff.PairMatcher(W, H, C, r=r, r2=r2, k=kk, subpel=Q, eps=eps, n_bwd=nb, leaf=kw.get("leaf", LEAF),
                           R=kw.get("R", 1))
        ok = n = 0
        e10 = e = 0.0
        n_set = kept = 0
        ms_tot = 0.0
        for p in prs:
            i1, i2 = torch.from_numpy(p.img1).to(dev), torch.from_numpy(p.img2).to(dev)
            run = lambda: m.run(i1, i2, seed=p.seed)
            run()
            run()
            ms, _, out = time_steps(run, torch, 5)
            assert all(st == 0 for st in m.status())
            ms_tot += ms
            F = out["F"].cpu().numpy()
            u = F.astype(np.int64) & 0xFFFFFFFF
            dx = (((u & 0xFFFF) ^ 0x8000) - 0x8000) / Q
            dy = ((((u >> 16) & 0xFFFF) ^ 0x8000) - 0x8000) / Q
            valid = F != ff.FF_EMPTY
            nocc = ~p.occluded
            epe = np.hypot(dx - p.flow[..., 0], dy - p.flow[..., 1])
            ok += int((valid & nocc & (epe < 3.0)).sum())
            n += int(nocc.sum())
            e10 += float(np.where(valid, np.minimum(epe, 10.0), 10.0)[nocc].sum())
            e += float(epe[valid & nocc].sum())
            n_set += int((valid & nocc).sum())
            kept += int(out["keep"].sum().item())
        del m
        rows.append({"setting": name, "le3px_pct": round(100.0 * ok / n, 3), "EPE10": round(e10 / n, 4),
                     "EPE": round(e / max(n_set, 1), 4), "kept_pct": round(100.0 * kept / (len(prs) * W * H), 3),
                     "Mpixel_per_s": round(len(prs) * W * H / ms_tot / 1e3, 3)})
    return rows


if __name__ == "__main__":
    main()
