"""Training and evaluation of the learned coarse-flow proposal.

Labels: the plain method's forward field after the two-way consistency filter
(section 3.4), read at the seed grid points (8 gx, 8 gy) of a 3-level
hierarchy; points the filter removed stay unlabelled.  The network is trained
with its own HIP forward/backward/Adam kernels (``ff.ProposalNet``) on pairs
generated on the device in bulk (``synth.gpu_pairs``), and evaluated on
seeded NumPy pairs whose seeds the training set never uses.

Three matching modes are compared (``evaluate``):
  plain          kd-tree seeds only (the paper's method);
  plain+learned  kd-tree seeds plus the network's flow as one more candidate;
  learned        the network's flow as the only seed candidate (no kd-tree).
The backward fields take the network's flow of the swapped pair.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import ff

W_DEF, H_DEF = 1024, 436
TRAIN_SEED0 = 1_000_000


def labels_from_filtered(filtered, k=3):
    """Seed-grid labels (packed 1/Q px, EMPTY where filtered out)."""
    s = 1 << k
    return filtered[..., ::s, ::s].contiguous()


def make_dataset(n_pairs, seed0=TRAIN_SEED0, batch=16, W=W_DEF, H=H_DEF, device="cuda", log=print):
    """Generate n_pairs layered pairs on the device and label them with the
    plain method.  Returns (img1, img2, labels) device tensors."""
    from synth import gpu_pairs
    n_pairs = (n_pairs + batch - 1) // batch * batch
    img1 = torch.empty((n_pairs, H, W, 3), dtype=torch.uint8, device=device)
    img2 = torch.empty_like(img1)
    hc, wc = ff.seed_grid(W, H)
    labels = torch.empty((n_pairs, hc, wc), dtype=torch.int32, device=device)
    matcher = ff.BatchMatcher([(W, H)] * batch)
    t0 = time.time()
    last = t0
    for b0 in range(0, n_pairs, batch):
        seeds = list(range(seed0 + b0, seed0 + b0 + batch))
        i1, i2, _ = gpu_pairs.layered_batch(seeds, W, H, device=device)
        img1[b0:b0 + batch] = i1
        img2[b0:b0 + batch] = i2
        out = matcher.run([img1[b0 + j] for j in range(batch)], [img2[b0 + j] for j in range(batch)], seeds=seeds)
        for j in range(batch):
            labels[b0 + j] = labels_from_filtered(out[j]["filtered"])
        if time.time() - last > 20:
            torch.cuda.synchronize()
            last = time.time()
            log(f"dataset {b0 + batch}/{n_pairs} pairs, {last - t0:.0f} s")
    torch.cuda.synchronize()
    if matcher.status() != 0:
        raise ff.FFError(matcher.status(), "labelling match")
    lab = labels.cpu().numpy()
    log(f"dataset ready: {n_pairs} pairs in {time.time() - t0:.0f} s, "
        f"{(lab != ff.FF_EMPTY).mean():.3f} of seed points labelled")
    return img1, img2, labels


def train(net, data, epochs=2, batch=16, lr_max=2e-3, lr_min=5e-5, warmup=100, seed=0, log=print,
          log_every=50):
    """Adam with linear warm-up and cosine decay over all steps."""
    img1, img2, labels = data
    n = img1.shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    g = torch.Generator().manual_seed(seed)
    hist = []
    t0 = time.time()
    step = 0
    for ep in range(epochs):
        order = torch.randperm(n, generator=g)
        for s in range(steps_per_epoch):
            idx = order[s * batch:(s + 1) * batch].to(img1.device)
            if step < warmup:
                lr = lr_max * (step + 1) / warmup
            else:
                u = (step - warmup) / max(total - warmup, 1)
                lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * u))
            loss = net.train_step(img1.index_select(0, idx).contiguous(), img2.index_select(0, idx).contiguous(),
                                  labels.index_select(0, idx).contiguous(), lr)
            step += 1
            if step % log_every == 0 or step == total:
                lv = float(loss.item())
                hist.append((step, lv))
                log(f"step {step}/{total} epoch {ep} lr {lr:.2e} loss {lv:.4f} ({lv * ff.NET_FLOW_SCALE:.2f} px) "
                    f"{time.time() - t0:.0f} s")
    return hist


def save(net, path, meta):
    from safetensors.torch import save_file
    save_file({"params": net.params.detach().cpu().contiguous()}, path,
              metadata={k: json.dumps(v) for k, v in meta.items()})


def load(path, device="cuda", subpel=4):
    from safetensors.torch import load_file
    sd = load_file(path)
    return ff.ProposalNet(sd["params"], device=device, subpel=subpel)


def proposals_both_ways(net, img1, img2):
    """Network flow of (img1 -> img2) and of the swapped pair, batched."""
    B = img1.shape[0]
    both1 = torch.cat([img1, img2], 0)
    both2 = torch.cat([img2, img1], 0)
    p = net.forward(both1, both2)
    return p[:B], p[B:]


def evaluate(net, eval_pairs, modes=("plain", "plain+learned", "learned"), reps=3, log=print):
    """Per mode: Mpx/s of the whole path (descriptors, network where used,
    three fields, filter) over the batch, and the EPE < 3 px rate of F and of
    the filtered field against ground truth (non-occluded pixels)."""
    from synth import pairs as P
    dev = "cuda"
    shapes = [(p.img1.shape[1], p.img1.shape[0]) for p in eval_pairs]
    assert len(set(shapes)) == 1
    W, H = shapes[0]
    i1 = torch.from_numpy(np.stack([p.img1 for p in eval_pairs])).to(dev)
    i2 = torch.from_numpy(np.stack([p.img2 for p in eval_pairs])).to(dev)
    B = len(eval_pairs)
    seeds = [p.seed for p in eval_pairs]
    res = {}
    for mode in modes:
        m = ff.BatchMatcher(shapes, use_kdtree=0 if mode == "learned" else 1)
        l1 = [i1[j] for j in range(B)]
        l2 = [i2[j] for j in range(B)]

        def once():
            props = None
            if mode != "plain":
                pf, pb = proposals_both_ways(net, i1, i2)
                props = [(pf[j], pb[j]) for j in range(B)]
            return m.run(l1, l2, seeds=seeds, proposals=props)

        out = once()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            out = once()
        t1.record()
        torch.cuda.synchronize()
        if m.status() != 0:
            raise ff.FFError(m.status(), f"evaluate {mode}")
        ms = t0.elapsed_time(t1) / reps
        rate_f = float(np.mean([P.inlier_rate(out[j]["F"][0].cpu().numpy(), eval_pairs[j], 4)
                                for j in range(B)]))
        rate_flt = float(np.mean([P.inlier_rate(out[j]["filtered"].cpu().numpy(), eval_pairs[j], 4)
                                  for j in range(B)]))
        res[mode] = dict(ms=ms, mpx_s=B * W * H / ms / 1e3, inlier_F=rate_f, inlier_filtered=rate_flt)
        log(f"{mode:14s} {ms:8.2f} ms  {res[mode]['mpx_s']:7.2f} Mpx/s  EPE<3 F {rate_f:.4f}  "
            f"filtered {rate_flt:.4f}")
    # the network alone, before any search: EPE < 3 px at the seed points
    pf, _ = proposals_both_ways(net, i1, i2)
    torch.cuda.synchronize()
    pf = pf.cpu().numpy()
    ok = tot = 0
    for j, p in enumerate(eval_pairs):
        f = pf[j].astype(np.int64) & 0xFFFFFFFF
        dx = (((f & 0xFFFF) ^ 0x8000) - 0x8000) / 4.0
        dy = ((((f >> 16) & 0xFFFF) ^ 0x8000) - 0x8000) / 4.0
        gt = p.flow[::8, ::8]
        vis = ~p.occluded[::8, ::8]
        e = np.hypot(dx - gt[..., 0], dy - gt[..., 1])
        ok += int(((e < 3.0) & vis).sum())
        tot += int(vis.sum())
    res["network_only_seed_points"] = ok / max(tot, 1)
    log(f"network alone at the seed points: EPE<3 {res['network_only_seed_points']:.4f}")
    return res


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="train the learned proposal on the GPU")
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--eval-pairs", type=int, default=16)
    ap.add_argument("--out", default="")
    ap.add_argument("--log", default="")
    a = ap.parse_args(argv)
    logf = open(a.log, "w") if a.log else None

    def log(s):
        print(s, flush=True)
        if logf:
            logf.write(s + "\n")
            logf.flush()

    ff.ff_init()
    t0 = time.time()
    data = make_dataset(a.pairs, batch=a.batch, log=log)
    net = ff.ProposalNet(seed=a.init_seed)
    hist = train(net, data, epochs=a.epochs, batch=a.batch, lr_max=a.lr, log=log)
    del data
    torch.cuda.empty_cache()
    meta = dict(pairs=a.pairs, epochs=a.epochs, batch=a.batch, lr=a.lr, init_seed=a.init_seed,
                train_seed0=TRAIN_SEED0, final_loss=hist[-1][1], seconds=round(time.time() - t0, 1),
                recipe="layered 1024x436, 6 layers, translations U(+-200) px (synth.gpu_pairs, motion=uniform)")
    if a.out:
        save(net, a.out, meta)
        log(f"saved {a.out}")
    if a.eval_pairs:
        from synth import pairs as P
        ev = [P.layered_pair(seed=4000 + i) for i in range(a.eval_pairs)]
        res = evaluate(net, ev, log=log)
        log(json.dumps(res))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
