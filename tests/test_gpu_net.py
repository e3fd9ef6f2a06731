"""GPU parity of the learned proposal's kernels against the float64 oracle:
forward output and its rounding to packed proposals, the parameter gradient of
the masked L1 loss, Adam, run-to-run determinism, checkpoint/resume, and the
proposal's use as a seed candidate (bit-exact with the oracle's match).

Tolerances.  Both sides multiply the same bf16 values exactly; they differ in
the accumulation (fp32 on the matrix cores, fp64 here: relative <= K * 2^-24
of the sum of |products|, K <= 2^19 terms) and, through that, in an
occasional bf16 rounding of a stored activation or gradient that falls on the
other side of a boundary (one bf16 ulp, 2^-8 relative, at that element) or a
ReLU decision at z ~ 0 taken the other way.  Each element is measured
against its magnitude -- the sum of |factor| x |factor| over the products it
sums (the oracle computes it with the same arithmetic on absolute values):

* forward: every output element within 2^-6 of its magnitude (two ulps of
  each factor of the last layer's products) and the RMS difference below one
  ulp (2^-8) of the RMS output;
* gradient with every ReLU clearly active (biases chosen so that no
  pre-activation comes near zero): every weight and bias gradient within
  2^-6 of its magnitude, the same two-ulp argument;
* gradient with realistic weights: a ReLU decision taken the other way keeps
  or drops a whole product term, so an element may be off by a share of its
  magnitude; every element within a quarter of it, and each layer within
  2^-6 in relative L2 with cosine >= 0.9999.

The L1 loss's gradient takes a sign per labelled point; the gradient tests
place their labels farther from the oracle's output than the forward error,
so both sides take the same sign."""
import sys

import numpy as np
import pytest

from oracle import ffo
from oracle import net_oracle as N
from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = 4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff as _ff
    _ff.ff_init()
    return _ff


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _theta(seed):
    rng = np.random.default_rng(100 + seed)
    th = N.init_params(seed).astype(np.float64)
    # non-zero biases so that the bias paths are exercised
    o = 0
    for ci, co, _, _, _ in N.LAYERS:
        o += co * ci * 9
        th[o:o + co] = rng.normal(0, 0.05, co)
        o += co
    return th.astype(np.float32)


def _theta_active(seed, x, margin=0.25):
    """Parameters whose every ReLU layer has a positive bias large enough
    that, on input x, every pre-activation stays at least `margin` above
    zero (bias = margin - the smallest bias-free pre-activation, layer by
    layer on the oracle's own activations): then no ReLU decision, forward or
    backward, can fall differently on the two sides, and only the bf16
    rounding of the stored tensors differs."""
    th = _theta(seed).astype(np.float64)
    a = x
    o = 0
    for (ci, co, st, d, relu), (W, _) in zip(N.LAYERS, N.split_params(th.copy())):
        o += co * ci * 9
        if relu:
            z = N.conv(a, N.bf16(W), np.zeros(co), st, d)
            th[o:o + co] = margin - z.min()
            a = N.bf16(np.maximum(z + th[o:o + co], 0.0))
        o += co
    return th.astype(np.float32)


def _batch(seed, B, W, H):
    ps = [pairs.layered_pair(seed=seed + i, W=W, H=H, nlayers=3) for i in range(B)]
    return np.stack([p.img1 for p in ps]), np.stack([p.img2 for p in ps]), ps


def _elem_bound(ref):
    return 2.0 ** -5 * np.abs(ref).max()


CASES = [("b2_61x45", 2, 61, 45), ("b1_97x37", 1, 97, 37), ("b1_1024x436", 1, 1024, 436)]


@pytest.mark.parametrize("name,B,W,H", CASES, ids=[c[0] for c in CASES])
def test_forward_matches_oracle(ff, name, B, W, H):
    _say("forward", name)
    th = _theta(0)
    i1, i2, _ = _batch(50, B, W, H)
    net = ff.ProposalNet(th, subpel=Q)
    hc, wc = ff.seed_grid(W, H)
    flow = torch.empty((B, hc, wc, 2), dtype=torch.float32, device="cuda")
    prop = net.forward(_dev(i1), _dev(i2), flow_out=flow)
    torch.cuda.synchronize()
    got = flow.cpu().numpy().astype(np.float64)
    x = N.input_tensor(i1, i2)
    ref, acts = N.forward(th.astype(np.float64), x, keep=True)
    assert got.shape == ref.shape == (B, hc, wc, 2)
    err = np.abs(got - ref)
    rms = np.sqrt((err ** 2).mean())
    mag = N.forward_magnitude(th.astype(np.float64), acts)
    _say("  max err", float(err.max()), "max |ref|", float(np.abs(ref).max()), "rms err", rms,
         "rms ref", float(np.sqrt((ref ** 2).mean())), "max err / magnitude", float((err / mag).max()))
    assert (err <= 2.0 ** -6 * mag).all(), float((err / mag).max())
    assert rms <= 2.0 ** -8 * np.sqrt((ref ** 2).mean()), rms
    # the packed proposal is exactly the rounding of the returned flow
    assert np.array_equal(prop.cpu().numpy(), N.proposal_q(got, Q))


def _labels(rng, B, hc, wc):
    fx = rng.integers(-160, 160, (B, hc, wc))
    fy = rng.integers(-80, 80, (B, hc, wc))
    lab = ffo.pack(fx, fy)
    lab[rng.random((B, hc, wc)) < 0.3] = ffo.EMPTY
    px = np.stack([fx, fy], -1).astype(np.float64) / Q
    px[lab == ffo.EMPTY] = np.nan
    return lab.astype(np.int32), px


GCASES = [("b2_61x45", 2, 61, 45), ("b1_200x120", 1, 200, 120), ("b1_1024x436", 1, 1024, 436)]


def _clear_labels(rng, out):
    """Labels (1/Q px, 30% unlabelled) placed away from the oracle's output
    by more than the forward element bound plus half a label quantum, so the
    sign of out - label (a discrete decision of the L1 gradient) is the same
    on both sides."""
    q = 1.0 / (Q * N.FLOW_SCALE)
    d = _elem_bound(out) + q + rng.uniform(0, 1.5, out.shape)
    t = out + np.where(rng.random(out.shape) < 0.5, -d, d)
    f = np.clip(np.rint(t * N.FLOW_SCALE * Q), -32767, 32767).astype(np.int64)
    lab = ffo.pack(f[..., 0], f[..., 1])
    lab[rng.random(out.shape[:3]) < 0.3] = ffo.EMPTY
    px = f.astype(np.float64) / Q
    px[lab == ffo.EMPTY] = np.nan
    return lab.astype(np.int32), px


@pytest.mark.parametrize("name,B,W,H", GCASES, ids=[c[0] for c in GCASES])
def test_gradient_matches_oracle(ff, name, B, W, H):
    _say("gradient", name)
    th = _theta(1)
    i1, i2, _ = _batch(70, B, W, H)
    x = N.input_tensor(i1, i2)
    th64 = th.astype(np.float64)
    out, acts = N.forward(th64, x, keep=True)
    lab, lab_px = _clear_labels(np.random.default_rng(3), out)
    rloss, gout = N.masked_l1(out, lab_px)
    rg, mag = N.backward(th64, acts, gout, magnitude=True)
    net = ff.ProposalNet(th, subpel=Q)
    loss, g = net.gradient(_dev(i1), _dev(i2), _dev(lab))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - rloss) <= 1e-4 * rloss
    o = 0
    for li, (ci, co, _, _, _) in enumerate(N.LAYERS):
        n = co * ci * 9 + co
        a, b = g[o:o + n], rg[o:o + n]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        ratio = np.abs(a - b) / np.maximum(mag[o:o + n], 1e-30)
        _say(f"  layer {li}: rel {rel:.2e} cos {cos:.8f} max err/magnitude {ratio.max():.3e} "
             f"p99.9 {np.quantile(ratio, 0.999):.3e}")
        # element by element: a ReLU decision at z ~ 0 taken differently on
        # the two sides drops or keeps a whole product term, so with
        # realistic weights an element can be off by a share of its
        # magnitude; no element by more than a quarter of it
        assert ratio.max() <= 0.25, (li, float(ratio.max()))
        assert rel <= 2.0 ** -6 and cos >= 0.9999, (li, rel, cos)
        o += n


def test_gradient_deterministic_and_adam(ff):
    th = _theta(2)
    B, W, H = 2, 128, 96
    i1, i2, _ = _batch(90, B, W, H)
    hc, wc = ff.seed_grid(W, H)
    lab, _ = _labels(np.random.default_rng(4), B, hc, wc)
    i1, i2, lab = _dev(i1), _dev(i2), _dev(lab)
    net = ff.ProposalNet(th, subpel=Q)
    _, g1 = net.gradient(i1, i2, lab)
    _, g2 = net.gradient(i1, i2, lab)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    # three Adam steps: compare with the oracle's update fed the same gradients
    m = np.zeros(N.param_count())
    v = np.zeros(N.param_count())
    ref = th.astype(np.float64)
    lr = 1e-3
    gbuf = torch.empty_like(net.params)
    for step in range(1, 4):
        _say("adam step", step)
        net.step = step
        ff.ff_proposal_train_step(net.params, net.m, net.v, step, lr, i1, i2, lab, net.workspace(B, W, H), Q, gbuf, net.loss)
        torch.cuda.synchronize()
        gg = gbuf.cpu().numpy().astype(np.float64)
        ref, m, v = N.adam_step(ref, m, v, gg, step, lr)
        got = net.params.cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max()), step


def test_checkpoint_resume_identical(ff, tmp_path):
    th = _theta(3)
    B, W, H = 2, 96, 64
    i1, i2, _ = _batch(110, B, W, H)
    hc, wc = ff.seed_grid(W, H)
    lab, _ = _labels(np.random.default_rng(5), B, hc, wc)
    i1, i2, lab = _dev(i1), _dev(i2), _dev(lab)
    a = ff.ProposalNet(th, subpel=Q)
    for _ in range(4):
        a.train_step(i1, i2, lab, 2e-3)
    b = ff.ProposalNet(th, subpel=Q)
    for _ in range(2):
        b.train_step(i1, i2, lab, 2e-3)
    torch.cuda.synchronize()
    path = tmp_path / "ckpt.pt"
    torch.save(b.state_dict(), path)
    c = ff.ProposalNet(subpel=Q)
    c.load_state_dict(torch.load(path, weights_only=True))
    for _ in range(2):
        c.train_step(i1, i2, lab, 2e-3)
    torch.cuda.synchronize()
    assert torch.equal(a.params, c.params) and torch.equal(a.m, c.m) and torch.equal(a.v, c.v)
    assert not torch.equal(a.params, torch.from_numpy(th).cuda())


def test_proposal_as_seed_candidate_matches_oracle(ff):
    """The network's rounded flow, injected at the seed grid, gives the same
    field as the oracle's match with that proposal (with and without the
    kd-tree candidates)."""
    th = _theta(4)
    p = pairs.square_pair(3)
    H, W = p.img1.shape[:2]
    net = ff.ProposalNet(th, subpel=Q)
    prop = net.forward(_dev(p.img1), _dev(p.img2))[0].contiguous()
    torch.cuda.synchronize()
    pn = prop.cpu().numpy()
    k, r = 3, 8
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    d = ff.ff_desc_init(W, H, 3, k, Q, (r,))
    b1 = torch.empty(d.bytes, dtype=torch.uint8, device="cuda")
    b2 = torch.empty_like(b1)
    ff.ff_compute_descriptors(d, _dev(p.img1), b1)
    ff.ff_compute_descriptors(d, _dev(p.img2), b2)
    for use_tree in (1, 0):
        _say("learned proposal, use_kdtree", use_tree)
        prm = ff.ff_default_params(k=k, seed=9, use_kdtree=use_tree)
        ws = torch.empty(ff.ff_match_workspace_bytes(d, d, r, prm), dtype=torch.uint8, device="cuda")
        F = torch.empty((H, W), dtype=torch.int32, device="cuda")
        Cc = torch.empty_like(F)
        ff.ff_match_field(d, b1, d, b2, r, prm, prop, F, Cc, ws)
        torch.cuda.synchronize()
        assert ff.ff_read_status(ws) == 0
        oF, oC = ffo.match_field(o1, o2, r, k=k, seed=9, use_kdtree=bool(use_tree), proposal=pn)
        assert np.array_equal(F.cpu().numpy(), oF) and np.array_equal(Cc.cpu().numpy(), oC)


@pytest.mark.parametrize("name,B,W,H", GCASES, ids=[c[0] for c in GCASES])
def test_gradient_elementwise_without_relu_decisions(ff, name, B, W, H):
    """Element by element: with every ReLU clearly active, both sides
    multiply bf16 tensors that differ at most by the bf16 rounding of the
    stored activations and gradients, so each weight's (bias's) gradient, a
    sum of products over pixels, differs by at most two bf16 ulps of each
    factor (2^-7 + 2^-7 relative) of its magnitude S = sum |x| |g| (sum |g|),
    plus fp32 accumulation (K 2^-24 S, K <= 2^19 pixels): |err| <= 2^-6 S."""
    _say("gradient element-wise", name)
    i1, i2, _ = _batch(130, B, W, H)
    x = N.input_tensor(i1, i2)
    th = _theta_active(5, x)
    th64 = th.astype(np.float64)
    out, acts = N.forward(th64, x, keep=True)
    # every pre-activation of the ReLU layers well above zero
    for li, (ci, co, st, d, relu) in enumerate(N.LAYERS):
        if relu:
            W_, b_ = N.split_params(th64)[li]
            z = N.conv(acts[li], N.bf16(W_), b_, st, d)
            assert z.min() > 0.05, (li, z.min())
    lab, lab_px = _clear_labels(np.random.default_rng(6), out)
    _, gout = N.masked_l1(out, lab_px)
    rg, mag = N.backward(th64, acts, gout, magnitude=True)
    net = ff.ProposalNet(th, subpel=Q)
    _, g = net.gradient(_dev(i1), _dev(i2), _dev(lab))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ratio = np.abs(g - rg) / np.maximum(mag, 1e-30)
    o = 0
    for li, (ci, co, _, _, _) in enumerate(N.LAYERS):
        n = co * ci * 9 + co
        _say(f"  layer {li}: max err/magnitude {ratio[o:o + n].max():.3e}")
        o += n
    assert ratio.max() <= 2.0 ** -6, float(ratio.max())
