"""GPU parity of the weighted (learned) BP: forward, loss, adjoint, Adam.

Forward messages and the per-frame adjoint follow the oracle's operation order,
so they are compared bit for bit with the oracle's float build (given the same
d loss / d lambda); the frame sum of the weight gradient is accumulated in
double in frame order on both sides, so it matches too.  The loss gradient
itself (computed in double on the GPU) and the end-to-end gradient are
compared with the double build within tolerance.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1609_09358_amd import binding as PB
from paper_1609_09358_amd import inputs

pytestmark = pytest.mark.gpu
POLY = {0: 0, 8: 0x07, 16: 0x1021, 24: 0x864CFB}


def frames(N, K, c, ebn0, B, seed):
    code = PB.PolarCode(N, K, c, 0, 2.5)
    info = inputs.info_bits(B, K, seed)
    u, x = O.encode_batch(info, K, c, POLY[c], code.frozen)
    llr = O.channel_llr(x, inputs.noise(B, N, seed), O.sigma2(ebn0, K / N))
    return code, u, llr


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_w(T, n, N, seed, lo=0.5, hi=1.5):
    return np.random.default_rng(seed).uniform(lo, hi, (T, 2, n, N)).astype(np.float32)


@pytest.mark.parametrize("N,K,c,T", [(16, 8, 0, 3), (128, 64, 0, 5), (256, 128, 8, 10), (1024, 512, 24, 4)])
@pytest.mark.parametrize("variant", [2, 3])
def test_forward_bit_exact(N, K, c, T, variant):
    n = N.bit_length() - 1
    B = 21
    code, u, llr = frames(N, K, c, 1.5, B, seed=N + T)
    W = rand_w(T, n, N, seed=T)
    out = PB.wbp_forward(code, dev(llr), dev(W), variant=variant, save=True)
    lam = host(out["llr_u"])
    saved = host(out["saved"])
    for f in range(B):
        ref = O.bp_frame(llr[f], code.frozen, max_iter=T, stop=0, W=W.astype(np.float64), save=True, prec="f32")
        assert np.array_equal(lam[f], ref["llr_u"].astype(np.float32))
        assert np.array_equal(saved[f], ref["save"].astype(np.float32))


def test_unit_weights_equal_plain_bp():
    N, K, c, T = 1024, 512, 16, 7
    code, u, llr = frames(N, K, c, 2.0, 32, seed=4)
    W = np.ones((T, 2, 10, N), np.float32)
    a = PB.wbp_forward(code, dev(llr), dev(W))
    b = PB.bp_decode_batch(code, dev(llr), max_iter=T, stop=0, soft=True)
    assert np.array_equal(host(a["llr_u"]), host(b["llr_u"]))
    assert np.array_equal(host(a["u_hat"]), host(b["u_hat"]))


@pytest.mark.parametrize("N,K,c,T", [(16, 8, 0, 3), (128, 64, 0, 4), (256, 128, 8, 10), (1024, 512, 24, 3)])
@pytest.mark.parametrize("variant", [2, 3])
def test_backward_bit_exact_given_dlam(N, K, c, T, variant):
    n = N.bit_length() - 1
    B = 19
    code, u, llr = frames(N, K, c, 1.0, B, seed=7 * N + T)
    W = rand_w(T, n, N, seed=N)
    llr_d, W_d = dev(llr), dev(W)
    fw = PB.wbp_forward(code, llr_d, W_d, variant=variant, save=True)
    _, dlam = PB.wbp_bce(code, fw["llr_u"], dev(u))
    dW, dllr = PB.wbp_backward(code, llr_d, W_d, fw["saved"], dlam, variant=variant, want_dllr=True)
    dlam_h = host(dlam).astype(np.float64)
    ref_dW, ref_dllr = O.wbp_backward(llr, code.frozen, T, W.astype(np.float64), dlam_h, prec="f32")
    assert np.array_equal(host(dW), ref_dW.astype(np.float32))
    assert np.array_equal(host(dllr), ref_dllr.astype(np.float32))
    assert np.abs(ref_dW).sum() > 0


@pytest.mark.parametrize("T", [3, 10])
def test_end_to_end_gradient(T):
    """Loss and weight gradient at N = 256 (the training workload's code).

    Against the float oracle the forward decisions are identical, the adjoint
    is linear in d loss / d lambda, and that vector differs only through the
    device's and the host's double exp (at most an ulp after rounding to
    float), so the gradients agree to float rounding at any T.  Against the
    double oracle, fp32 rounding of the messages grows with every iteration
    (min/clip decisions flip on near-ties), so that comparison is made at
    T = 3 only, as for plain BP."""
    N, K, c, B = 256, 128, 8, 64
    n = 8
    code, u, llr = frames(N, K, c, 2.0, B, seed=99)
    W = rand_w(T, n, N, seed=5, lo=0.8, hi=1.2)
    llr_d, W_d = dev(llr), dev(W)
    fw = PB.wbp_forward(code, llr_d, W_d, save=True)
    loss, dlam = PB.wbp_bce(code, fw["llr_u"], dev(u))
    dW, _ = PB.wbp_backward(code, llr_d, W_d, fw["saved"], dlam)
    g = host(dW).astype(np.float64)
    tot = float(host(loss).astype(np.float64).sum())
    l32, g32 = O.wbp_grad(llr, code.frozen, u, T, W.astype(np.float64), prec="f32")
    assert abs(tot - l32) <= 1e-5 * max(1.0, abs(l32))
    assert np.max(np.abs(g - g32)) <= 1e-5 * np.abs(g32).max()
    if T <= 3:
        l64, g64 = O.wbp_grad(llr, code.frozen, u, T, W.astype(np.float64))
        assert abs(tot - l64) <= 1e-5 * max(1.0, abs(l64))
        assert np.max(np.abs(g - g64)) <= 1e-4 * np.abs(g64).max()


def test_adam_matches_oracle():
    rng = np.random.default_rng(3)
    w = rng.normal(size=5000).astype(np.float32)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    wd, md, vd = dev(w), dev(m), dev(v)
    w64, m64, v64 = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 6):
        g = rng.normal(size=5000).astype(np.float32)
        PB.polar_adam_step(wd, dev(g), md, vd, step)
        O.adam_step(w64, g.astype(np.float64), m64, v64, step)
    np.testing.assert_allclose(host(wd), w64, rtol=1e-5, atol=1e-6)


def test_autograd_function():
    N, K, c, T, B = 256, 128, 8, 4, 16
    code, u, llr = frames(N, K, c, 2.0, B, seed=12)
    W = torch.ones((T, 2, 8, N), device="cuda", requires_grad=True)
    llr_d = dev(llr)
    loss = PB.WeightedBPLoss.apply(llr_d, W, dev(u), code)
    loss.backward()
    fw = PB.wbp_forward(code, llr_d, W.detach(), save=True)
    _, dlam = PB.wbp_bce(code, fw["llr_u"], dev(u))
    dW, _ = PB.wbp_backward(code, llr_d, W.detach(), fw["saved"], dlam)
    assert torch.equal(W.grad, dW)
    assert float(loss) > 0


@pytest.mark.parametrize("N,K,c,T", [(64, 32, 0, 4), (256, 128, 8, 10), (1024, 512, 24, 3)])
def test_multi_loss_backward_bit_exact_given_dlam(N, K, c, T):
    """Loss after every iteration: the adjoint takes one d loss / d LLR(u) per
    iteration and matches the oracle's float build bit for bit."""
    n = N.bit_length() - 1
    B = 11
    code, u, llr = frames(N, K, c, 1.0, B, seed=3 * N + T)
    W = rand_w(T, n, N, seed=N + 1)
    llr_d, W_d = dev(llr), dev(W)
    fw = PB.wbp_forward(code, llr_d, W_d, save=True)
    _, dlam = PB.wbp_bce_multi(code, fw["saved"], dev(u), T)
    assert tuple(dlam.shape) == (B, T, N)
    dW, dllr = PB.wbp_backward(code, llr_d, W_d, fw["saved"], dlam, want_dllr=True)
    ref_dW, ref_dllr = O.wbp_backward(llr, code.frozen, T, W.astype(np.float64), host(dlam).astype(np.float64),
                                      prec="f32")
    assert np.array_equal(host(dW), ref_dW.astype(np.float32))
    assert np.array_equal(host(dllr), ref_dllr.astype(np.float32))


@pytest.mark.parametrize("T", [3, 10])
def test_multi_loss_end_to_end_vs_oracle(T):
    N, K, c, B = 256, 128, 8, 48
    code, u, llr = frames(N, K, c, 2.0, B, seed=123 + T)
    W = rand_w(T, 8, N, seed=9, lo=0.8, hi=1.2)
    llr_d, W_d = dev(llr), dev(W)
    fw = PB.wbp_forward(code, llr_d, W_d, save=True)
    loss, dlam = PB.wbp_bce_multi(code, fw["saved"], dev(u), T)
    dW, _ = PB.wbp_backward(code, llr_d, W_d, fw["saved"], dlam)
    g = host(dW).astype(np.float64)
    tot = float(host(loss).astype(np.float64).sum())
    l32, g32 = O.wbp_grad(llr, code.frozen, u, T, W.astype(np.float64), multi=True, prec="f32")
    assert abs(tot - l32) <= 1e-5 * max(1.0, abs(l32))
    assert np.max(np.abs(g - g32)) <= 1e-5 * np.abs(g32).max()
    if T <= 3:
        l64, g64 = O.wbp_grad(llr, code.frozen, u, T, W.astype(np.float64), multi=True)
        assert abs(tot - l64) <= 1e-5 * max(1.0, abs(l64))
        assert np.max(np.abs(g - g64)) <= 1e-4 * np.abs(g64).max()


@pytest.mark.parametrize("N,K,c,T", [(64, 32, 0, 6), (1024, 512, 24, 12)])
@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("lo,hi", [(0.8, 1.1), (0.5, 1.0), (-1.0, 1.0)])
def test_per_stage_weights_equal_expanded_per_node_weights(N, K, c, T, variant, lo, hi):
    """One weight per stage column (scalar loads) decodes exactly like the
    same weights repeated over the column's nodes, with early stopping.  With
    every weight within [-1, 1] (the ranges ending at 1.0, which also hold
    weights of exactly 1 and -1 and, in the last, negative ones) the
    per-stage kernel leaves out the clips that cannot act; above 1 it keeps
    them."""
    n = N.bit_length() - 1
    code, u, llr = frames(N, K, c, 2.0, 40, seed=N + T + variant)
    w = np.random.default_rng(T).uniform(lo, hi, (T, 2, n)).astype(np.float32)
    if hi == 1.0:
        w[0, 0, 0], w[1, 1, n - 1] = 1.0, -1.0 if lo < 0 else 1.0
    Ws = torch.from_numpy(w).cuda()
    Wn = Ws[..., None].expand(T, 2, n, N).contiguous()
    a = PB.bp_decode_batch(code, dev(llr), max_iter=T, stop=1, weights=Ws, variant=variant, soft=True)
    b = PB.bp_decode_batch(code, dev(llr), max_iter=T, stop=1, weights=Wn, variant=variant, soft=True)
    for key in ("u_hat", "llr_u", "iters", "ok"):
        assert torch.equal(a[key], b[key]), key
    ha = PB.HybridDecoder(code, max_iter=T, L=8, weights=Ws)(dev(llr))
    hb = PB.HybridDecoder(code, max_iter=T, L=8, weights=Wn)(dev(llr))
    assert torch.equal(ha["info"], hb["info"])


@pytest.mark.parametrize("layout,lo,hi", [("node", 0.75, 1.05), ("column", 0.75, 1.0), ("column", 0.7, 1.25)])
@pytest.mark.parametrize("stop", [0, 1])
@pytest.mark.parametrize("variant", [0, 2])
def test_weighted_bp_decode_vs_f32_oracle(layout, lo, hi, stop, variant):
    """bp_decode_batch with learned weights (one per node, or one per stage
    column) at N = 1024, T = 20 -- the benchmark's decoder when the weights are
    per column within [0, 1], where the kernel leaves out the clip that cannot
    act -- against the oracle's float build: soft outputs LLR(u), iteration
    counts, verdicts and decisions bit for bit."""
    N, K, c, T, B = 1024, 512, 24, 20, 24
    n = 10
    code, u, llr = frames(N, K, c, 2.0, B, seed=900 + int(10 * hi) + stop)
    rng = np.random.default_rng(int(100 * lo) + stop)
    shape = (T, 2, n, N) if layout == "node" else (T, 2, n)
    w = rng.uniform(lo, hi, shape).astype(np.float32)
    if hi == 1.0:
        w.reshape(-1)[:3] = 1.0
    Wn = w if layout == "node" else np.repeat(w[..., None], N, axis=3)
    out = PB.bp_decode_batch(code, dev(llr), max_iter=T, stop=stop, weights=dev(w), variant=variant, soft=True)
    ref = O.bp_batch(llr, code.frozen, c, POLY[c], max_iter=T, stop=stop, W=Wn.astype(np.float64), prec="f32",
                     soft=True)
    assert np.array_equal(host(out["iters"]), ref["iters"])
    assert np.array_equal(host(out["ok"]), ref["ok"])
    assert np.array_equal(host(out["u_hat"]), ref["u_hat"])
    assert np.array_equal(host(out["llr_u"]), ref["llr_u"].astype(np.float32))
    if stop == 1:
        assert 0 < ref["ok"].sum() < B


@pytest.mark.parametrize("N,K,c,T", [(64, 32, 0, 4), (256, 128, 8, 10), (1024, 512, 24, 3)])
def test_frame_loss_backward_bit_exact_given_dlam(N, K, c, T):
    """The frame-failure surrogate's d loss / d LLR(u) per iteration feeds the
    same adjoint: bit-exact with the oracle's float build given that input."""
    n = N.bit_length() - 1
    B = 13
    code, u, llr = frames(N, K, c, 1.5, B, seed=5 * N + T)
    W = rand_w(T, n, N, seed=N + 2, lo=0.6, hi=1.2)
    llr_d, W_d = dev(llr), dev(W)
    fw = PB.wbp_forward(code, llr_d, W_d, save=True)
    _, dlam = PB.wbp_frame_loss(code, fw["saved"], dev(u), T)
    assert tuple(dlam.shape) == (B, T, N)
    dW, dllr = PB.wbp_backward(code, llr_d, W_d, fw["saved"], dlam, want_dllr=True)
    ref_dW, ref_dllr = O.wbp_backward(llr, code.frozen, T, W.astype(np.float64), host(dlam).astype(np.float64),
                                      prec="f32")
    assert np.array_equal(host(dW), ref_dW.astype(np.float32))
    assert np.array_equal(host(dllr), ref_dllr.astype(np.float32))


@pytest.mark.parametrize("T,ebn0", [(3, 0.5), (10, 1.5), (20, 2.5)])
@pytest.mark.parametrize("kind,fw_c", [(2, 0.0), (3, 0.0), (3, 40.0)])
def test_frame_loss_end_to_end_vs_oracle(T, ebn0, kind, fw_c):
    """Frame-level losses and their weight gradients at N = 256 against the
    oracle: the frame-failure loss (kind 2) and the expected-iterations loss
    with and without a fail weight (kind 3).  The loss per frame and the
    gradient agree to float rounding with the float build at any T and with
    the double build at T = 3.  The Eb/N0 is chosen so that a good part of the
    frames sit between 'always right' and 'never right', where these losses
    have a gradient."""
    N, K, c, B = 256, 128, 8, 64
    code, u, llr = frames(N, K, c, ebn0, B, seed=77 + T)
    W = rand_w(T, 8, N, seed=11, lo=0.8, hi=1.1)
    llr_d, W_d = dev(llr), dev(W)
    fw = PB.wbp_forward(code, llr_d, W_d, save=True)
    if kind == 2:
        loss, dlam = PB.wbp_frame_loss(code, fw["saved"], dev(u), T)
    else:
        loss, dlam = PB.wbp_iteration_loss(code, fw["saved"], dev(u), T, fw_c)
    dW, _ = PB.wbp_backward(code, llr_d, W_d, fw["saved"], dlam)
    g = host(dW).astype(np.float64)
    per = host(loss).astype(np.float64)
    top = 1.0 if kind == 2 else T - 1 + fw_c
    assert np.all((per >= 0) & (per <= top / B * (1 + 1e-6)))
    tot = float(per.sum())
    l32, g32 = O.wbp_grad(llr, code.frozen, u, T, W.astype(np.float64), kind=kind, fail_weight=fw_c, prec="f32")
    assert abs(tot - l32) <= 1e-5 * max(1e-3, abs(l32))
    assert np.abs(g32).max() > 0
    assert np.max(np.abs(g - g32)) <= 1e-5 * np.abs(g32).max()
    if T <= 3:
        l64, g64 = O.wbp_grad(llr, code.frozen, u, T, W.astype(np.float64), kind=kind, fail_weight=fw_c)
        assert abs(tot - l64) <= 1e-5 * max(1e-3, abs(l64))
        assert np.max(np.abs(g - g64)) <= 1e-4 * np.abs(g64).max()


def test_column_weights_and_gradient():
    """Column layout: the spread weights repeat each column's weight over its
    N nodes exactly; the column gradient is the per-node gradient summed over
    each column (double accumulation, compared with the oracle's per-node
    gradient summed in double)."""
    N, K, c, T, B = 1024, 512, 24, 4, 9
    n = 10
    code, u, llr = frames(N, K, c, 2.0, B, seed=31)
    wc = np.random.default_rng(4).uniform(0.7, 1.0, (T, 2, n)).astype(np.float32)
    Wn = PB.wbp_column_weights(code, dev(wc))
    assert np.array_equal(host(Wn), np.repeat(wc[..., None], N, axis=3))
    llr_d = dev(llr)
    fw = PB.wbp_forward(code, llr_d, Wn, save=True)
    _, dlam = PB.wbp_bce_multi(code, fw["saved"], dev(u), T)
    dW, _ = PB.wbp_backward(code, llr_d, Wn, fw["saved"], dlam)
    gc = host(PB.wbp_column_grad(code, dW)).astype(np.float64)
    _, g32 = O.wbp_grad(llr, code.frozen, u, T, np.repeat(wc[..., None], N, axis=3).astype(np.float64), kind=1,
                        prec="f32")
    ref = g32.sum(axis=3)
    assert np.abs(ref).max() > 0
    assert np.max(np.abs(gc - ref)) <= 1e-5 * np.abs(ref).max()


def test_bounded_adam_is_adam_then_projection():
    rng = np.random.default_rng(8)
    w = rng.uniform(-0.2, 1.2, 3000).astype(np.float32)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    wd, md, vd = dev(w), dev(m), dev(v)
    w64, m64, v64 = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 5):
        g = rng.normal(size=3000).astype(np.float32)
        PB.polar_adam_step_bounded(wd, dev(g), md, vd, step, lr=0.05, lo=0.0, hi=1.0)
        O.adam_step(w64, g.astype(np.float64), m64, v64, step, lr=0.05)
        np.clip(w64, 0.0, 1.0, out=w64)
    got = host(wd)
    assert got.min() >= 0.0 and got.max() <= 1.0
    assert (got == 0.0).sum() > 0 and (got == 1.0).sum() > 0
    np.testing.assert_allclose(got, w64, rtol=1e-5, atol=1e-6)
    with pytest.raises(PB.PolarError):
        PB.polar_adam_step_bounded(wd, dev(g), md, vd, 5, lo=1.0, hi=0.0)


def _mcnemar_z(only_a, only_b):
    """z statistic of McNemar's paired test: how many standard deviations the
    discordant counts lie apart (b wrong where a is right vs the reverse)."""
    return (only_a - only_b) / max(1.0, np.sqrt(only_a + only_b))


def test_training_lowers_bp_failures_of_learned_hybrid_front_end():
    """What the gradient-trained network gains over the method without it, on
    the learned hybrid's front end (N = 1024, K = 512, CRC-24, T = 20, one
    weight per stage column within [0, 1], frame-failure loss, Adam through
    the library's forward and adjoint kernels): on held-out frames at 2.5 dB
    the trained BP hands far fewer frames to the list decoder than plain
    min-sum BP with the same T (w = 1), beyond both 95% Clopper-Pearson
    intervals; and training from the normalized min-sum scale alpha = 0.94
    (every weight equal) lowers the failures further, by McNemar's paired test
    on the same frames."""
    from scipy.stats import beta

    from paper_1609_09358_amd import train_wbp as TW

    N, K, c, T = 1024, 512, 24, 20
    code = PB.PolarCode(N, K, c, POLY[c], 2.5)
    held = TW.Trainer(code, 1, 16, seed=60606)
    _, _, llr = held.frames(1 << 16, ebn0=2.5)
    M = llr.shape[0]

    def fails(W):
        o = PB.bp_decode_batch(code, llr, max_iter=T, stop=1, weights=W)
        return o["ok"] == 0

    def cp(k):
        lo = 0.0 if k == 0 else beta.ppf(0.025, k, M - k + 1)
        hi = 1.0 if k == M else beta.ppf(0.975, k + 1, M - k)
        return lo, hi

    f1 = fails(torch.ones((T, 2, code.n), device="cuda"))
    tr = TW.Trainer(code, T, 1024, lr=1e-2, ebn0=(2.5, 2.5), seed=5, layout="column", loss="frame",
                    bounds=(0.0, 1.0), w0=1.0)
    for _ in range(200):
        tr.train_step()
    assert float(tr.W.min()) >= 0.0 and float(tr.W.max()) <= 1.0
    ft = fails(tr.W)
    k1, kt = int(f1.sum()), int(ft.sum())
    assert cp(kt)[1] < cp(k1)[0], (kt, k1)
    assert kt < 0.3 * k1

    fa = fails(torch.full((T, 2, code.n), 0.94, device="cuda"))
    tr2 = TW.Trainer(code, T, 1024, lr=3e-3, ebn0=(2.5, 2.5), seed=6, layout="column", loss="frame",
                     bounds=(0.0, 1.0), w0=0.94)
    for _ in range(300):
        tr2.train_step()
    fb = fails(tr2.W)
    z = _mcnemar_z(int((fa & ~fb).sum()), int((fb & ~fa).sum()))
    assert z > 3.0, (int(fa.sum()), int(fb.sum()), z)


def test_c4_bce_training_lowers_fer():
    """The learned BP of its configuration (N = 256, K = 128, CRC-8, T = 10,
    per-edge weights from 1, Adam lr 1e-3 on the final-iteration BCE over
    Eb/N0 uniform in [1, 4] dB, batches of 4096, 1e6 training frames): on
    1e5 held-out frames at 3 dB its frame error rate is lower than that of the
    untrained decoder (plain min-sum BP, 10 iterations, re-encoding stop), by
    McNemar's paired test on the same frames."""
    from paper_1609_09358_amd import train_wbp as TW

    tr, hist = TW.train(256, 128, 8, 10, frames=1_000_000, batch=4096, lr=1e-3, ebn0=(1.0, 4.0), design=2.5,
                        seed=1, log_every=1 << 30, verbose=False)
    assert hist[-1][1] < hist[0][1]
    code = tr.code
    info, _, llr = TW.Trainer(code, 1, 16, seed=31337).frames(100_000, ebn0=3.0)
    a = PB.bp_decode_batch(code, llr, max_iter=10, stop=1)
    b = PB.bp_decode_batch(code, llr, max_iter=10, stop=1, weights=tr.W)
    ea = (TW.info_of(code, a["u_hat"]) != info).any(dim=1)
    eb = (TW.info_of(code, b["u_hat"]) != info).any(dim=1)
    z = _mcnemar_z(int((ea & ~eb).sum()), int((eb & ~ea).sum()))
    assert z > 3.0, (int(ea.sum()), int(eb.sum()), z)
