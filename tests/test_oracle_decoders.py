"""Pins of the oracle's decoders (BP, SC, CA-SCL, hybrid, weighted BP, Adam).

References used here share no code with the oracle: brute-force enumeration
of tiny codes (exact and max-log posteriors, maximum-likelihood codewords),
closed forms, noiseless inputs, symmetry of the code, central finite
differences, and the decoders' known relations (SCL with L = 1 is SC).
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_1609_09358_amd import inputs
from tests import _bruteforce as BF


def _frame(N, K, c, poly, ebn0, seed, design=2.0, B=1):
    k = K + c
    fr = O.ga_frozen(N, k, design, K / N)
    info = inputs.info_bits(B, K, seed)
    u, x = O.encode_batch(info, K, c, poly, fr)
    z = inputs.noise(B, N, seed)
    llr = O.channel_llr(x, z, O.sigma2(ebn0, K / N))
    return fr, info, u, x, llr


# ------------------------------------------------------------------ BP

def _n2_posteriors(l, prior, exact):
    """Posterior LLRs of u_0, u_1 for one PE (N = 2) by enumeration.

    Costs: a bit b with LLR v costs b * v (up to a b-independent constant)."""
    cost = {}
    for u0, u1 in itertools.product([0, 1], repeat=2):
        x0, x1 = u0 ^ u1, u1
        cost[(u0, u1)] = prior[0] * u0 + prior[1] * u1 + l[0] * x0 + l[1] * x1
    out = []
    for pos in (0, 1):
        c0 = [v for key, v in cost.items() if key[pos] == 0]
        c1 = [v for key, v in cost.items() if key[pos] == 1]
        if exact:
            out.append(np.log(np.exp(-np.array(c0)).sum()) - np.log(np.exp(-np.array(c1)).sum()))
        else:
            out.append(min(c1) - min(c0))
    return np.array(out)


@pytest.mark.parametrize("rule", [0, 1])
def test_bp_single_pe_equals_enumeration(rule):
    """N = 2 has no cycles: after one iteration (and at the fixed point) the
    BP outputs LLR(u_i) = L_1 + R_1 are the exact (rule 1) or max-log
    (rule 0, min-sum) posteriors, for every frozen pattern."""
    rng = np.random.default_rng(3 + rule)
    for fr in ([0, 0], [1, 0], [0, 1], [1, 1]):
        fr = np.array(fr, np.uint8)
        for _ in range(50):
            l = rng.uniform(-5, 5, 2).astype(np.float32)
            ref = _n2_posteriors(l.astype(np.float64), 20.0 * fr, exact=bool(rule))
            for iters in (1, 2, 3):
                got = O.bp_frame(l, fr, max_iter=iters, stop=0, rule=rule)["llr_u"]
                np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)


def test_bp_repetition_code_closed_form():
    """Frozen = [1, 0]: after one iteration LLR(u_1) = l_0 + l_1."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        l = rng.uniform(-8, 8, 2).astype(np.float32)
        out = O.bp_frame(l, np.array([1, 0], np.uint8), max_iter=1, stop=0)
        assert abs(out["llr_u"][1] - (float(l[0]) + float(l[1]))) < 1e-12


@pytest.mark.parametrize("N,K", [(128, 64), (1024, 512)])
def test_bp_noiseless_decodes_in_one_iteration(N, K):
    fr = O.ga_frozen(N, K, 2.0, K / N)
    info = inputs.info_bits(4, K, seed=N)
    u, x = O.encode_batch(info, K, 0, 0, fr)
    llr = (4.0 * (1.0 - 2.0 * x)).astype(np.float32)
    for prec in ("f64", "f32"):
        out = O.bp_batch(llr, fr, max_iter=100, stop=1, prec=prec)
        assert np.array_equal(out["u_hat"], u)
        assert np.all(out["iters"] == 1) and np.all(out["ok"] == 1)


def test_bp_codeword_symmetry():
    """Flipping the LLR signs along a codeword x = u G maps every BP message by
    the same sign pattern, so decode(llr * (1 - 2x)) = decode(llr) XOR u."""
    N, K = 128, 64
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.5, seed=21, B=64)
    other = O.encode_batch(inputs.info_bits(64, K, 99), K, 0, 0, fr)
    u2, x2 = other
    base = O.bp_batch(llr, fr, max_iter=30, stop=0, prec="f32")
    flip = O.bp_batch(llr * (1.0 - 2.0 * x2), fr, max_iter=30, stop=0, prec="f32")
    same = np.all((flip["u_hat"] ^ u2) == base["u_hat"], axis=1)
    assert same.mean() >= 0.95


@pytest.mark.slow
def test_bp_fer_is_sane_and_monotone():
    """Rate-1/2, N = 128: FER falls with Eb/N0 and BP is within a small factor
    of SC (polar BP and SC perform alike at this length)."""
    N, K, B = 128, 64, 600
    fer_bp, fer_sc = [], []
    for e in (1.0, 2.0, 3.0):
        fr, info, u, x, llr = _frame(N, K, 0, 0, e, seed=int(10 * e), B=B)
        out = O.bp_batch(llr, fr, max_iter=100, stop=1)
        fer_bp.append(np.mean(np.any(out["u_hat"] != u, axis=1)))
        sc = np.array([O.sc_frame(llr[f], fr) for f in range(B)])
        fer_sc.append(np.mean(np.any(sc != u, axis=1)))
    assert fer_bp[0] > fer_bp[1] > fer_bp[2]
    assert fer_bp[2] < 0.05
    for a, b in zip(fer_bp, fer_sc):
        assert a < 3 * b + 0.02


def test_bp_stop_rules():
    N, K, c, poly = 256, 128, 8, 0x07
    fr, info, u, x, llr = _frame(N, K, c, poly, 2.5, seed=8, design=2.5, B=32)
    g = O.bp_batch(llr, fr, c, poly, max_iter=60, stop=1)
    r = O.bp_batch(llr, fr, c, poly, max_iter=60, stop=2)
    n = O.bp_batch(llr, fr, c, poly, max_iter=7, stop=0)
    assert np.all(n["iters"] == 7)
    for f in range(32):
        # a frame stopped early by the re-encoding check is a codeword
        if g["iters"][f] < 60:
            xh = O.polar_transform(g["u_hat"][f])
            again = O.bp_frame(llr[f], fr, c, poly, max_iter=int(g["iters"][f]), stop=0)
            assert np.array_equal(xh, (again["llr_x"] < 0).astype(np.uint8))
        # ok means the CRC over the decided info bits holds
        if g["ok"][f]:
            free = np.where(fr == 0)[0]
            b = g["u_hat"][f][free]
            assert np.array_equal(O.crc(b[:K], c, poly), b[K:])
        assert r["iters"][f] <= 60


def _read_n4_golden():
    g = {"iters": {}, "stop1": {}}
    path = os.path.join(os.path.dirname(__file__), "golden", "bp_n4_minsum.txt")
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        if line[0] == "iter":
            g["iters"].setdefault(int(line[1]), {})[line[2]] = np.array([float(v) for v in line[3:]])
        elif line[0] == "stop1":
            g["stop1"][line[1]] = np.array([int(v) for v in line[2:]])
        else:
            g[line[0]] = np.array([float(v) for v in line[1:]])
    return g


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bp_n4_worked_example(prec):
    """Messages of two BP iterations on N = 4, worked by hand from the PE
    equations of Sec. II-B in the paper's sweep order (R over stages 2..n+1,
    then L over n..1): tests/golden/bp_n4_minsum.txt.  Fixes the schedule, the
    port mapping, the clipping of a computed sum and the re-encoding stop."""
    g = _read_n4_golden()
    fr = g["frozen"].astype(np.uint8)
    llr = g["llr"].astype(np.float32)
    for T in (1, 2):
        r = O.bp_frame(llr, fr, max_iter=T, stop=0, llr_max=float(g["llr_max"][0]), save=True, prec=prec)
        want = g["iters"][T]
        sv = r["save"][T - 1]  # [dir][column][node]: R row s+1 / L row s
        np.testing.assert_array_equal(sv[0][0], want["R1"])
        np.testing.assert_array_equal(sv[0][1], want["R2"])
        np.testing.assert_array_equal(sv[1][1], want["L1"])
        np.testing.assert_array_equal(sv[1][0], want["L0"])
        np.testing.assert_array_equal(r["llr_u"], want["llr_u"])
        np.testing.assert_array_equal(r["llr_x"], want["llr_x"])
    r = O.bp_frame(llr, fr, max_iter=2, stop=1, prec=prec)
    assert r["iters"] == g["stop1"]["iters"][0]
    np.testing.assert_array_equal(r["u_hat"], g["stop1"]["u_hat"])
    assert r["ok"] == g["stop1"]["ok"][0]


def test_bp_f32_and_f64_agree():
    N, K = 1024, 512
    fr, info, u, x, llr = _frame(N, K, 16, 0x1021, 2.5, seed=5, design=2.5, B=8)
    a = O.bp_frame(llr[0], fr, max_iter=3, stop=0, prec="f64")["llr_u"]
    b = O.bp_frame(llr[0], fr, max_iter=3, stop=0, prec="f32")["llr_u"]
    np.testing.assert_allclose(b, a, rtol=1e-4, atol=1e-4)


# ------------------------------------------------------------------ SC / SCL

def test_sc_n2_closed_form():
    rng = np.random.default_rng(2)
    for _ in range(50):
        l = rng.uniform(-6, 6, 2).astype(np.float32)
        fr = np.zeros(2, np.uint8)
        u = O.sc_frame(l, fr)
        f = np.sign(l[0]) * np.sign(l[1]) * min(abs(l[0]), abs(l[1]))
        u0 = int(f < 0)
        lam1 = float(l[1]) + (1 - 2 * u0) * float(l[0])
        assert u[0] == u0 and u[1] == int(lam1 < 0)


def test_sc_repetition_code_is_ml():
    """Only u_{N-1} free: the code is the repetition code, SC decides by the
    sign of the LLR sum (the last row of G is all ones)."""
    rng = np.random.default_rng(6)
    fr = np.ones(64, np.uint8)
    fr[-1] = 0
    for _ in range(50):
        l = rng.normal(0.3, 2.0, 64).astype(np.float32)
        assert O.sc_frame(l, fr)[-1] == int(l.astype(np.float64).sum() < 0)


@pytest.mark.parametrize("N,K", [(64, 32), (256, 128), (1024, 528)])
@pytest.mark.parametrize("rule", [0, 1])
def test_scl_list_one_is_sc(N, K, rule):
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.5, seed=N + rule, B=6)
    for prec in ("f64", "f32"):
        for f in range(6):
            sc = O.sc_frame(llr[f], fr, rule=rule, prec=prec)
            scl = O.scl_frame(llr[f], fr, 1, rule=rule, prec=prec)["u_hat"]
            assert np.array_equal(sc, scl)


@pytest.mark.parametrize("N,k", [(8, 4), (16, 5), (16, 3)])
@pytest.mark.parametrize("rule", [0, 1])
def test_scl_full_list_is_ml(N, k, rule):
    """With L = 2^k no path is ever pruned: SCL returns the ML codeword."""
    fr = O.ga_frozen(N, k, 1.0, k / N)
    rng = np.random.default_rng(N * 10 + k + rule)
    L = 2 ** k
    ties = 0
    for _ in range(150):
        info = rng.integers(0, 2, k).astype(np.uint8)
        u, x = O.encode_batch(info[None], k, 0, 0, fr)
        llr = O.channel_llr(x, rng.standard_normal((1, N)), O.sigma2(-1.0, k / N))[0]
        ml = BF.ml_minsum if rule == 0 else BF.ml_exact
        u_ml, best, met = ml(llr.astype(np.float64), fr)
        if np.sum(np.abs(met - best) <= 1e-9 * max(1.0, abs(best))) > 1:
            ties += 1
            continue
        got = O.scl_frame(llr, fr, L, rule=rule)["u_hat"]
        assert np.array_equal(got, u_ml.astype(np.uint8))
    assert ties < 10


@pytest.mark.parametrize("rule", [0, 1])
def test_scl_path_metric_is_codeword_metric(rule):
    """Every complete path's metric equals the metric of its re-encoded
    codeword: sum |llr_j| over disagreeing positions (min-sum) or
    sum ln(1 + e^{-(1-2x_j) llr_j}) (exact)."""
    N, K, L = 256, 128, 8
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.0, seed=31, B=4)
    for f in range(4):
        out = O.scl_frame(llr[f], fr, L, rule=rule, all_paths=True)
        l64 = llr[f].astype(np.float64)
        for q in range(out["n_paths"]):
            xq = O.polar_transform(out["all_u"][q]).astype(np.int64)
            if rule == 0:
                ref = np.sum(np.abs(l64) * (xq != (l64 < 0)))
            else:
                ref = np.sum(np.logaddexp(0.0, -(1 - 2 * xq) * l64))
            assert abs(out["all_pm"][q] - ref) <= 1e-9 * max(1.0, ref)


# ------------------------------------------------------------------ decision-aided SCL (Sec. II-A)

@pytest.mark.parametrize("rule", [0, 1])
def test_decision_aided_everywhere_is_sc(rule):
    """With every non-frozen position decision-aided no path ever branches, so
    the list decoder is SC whatever L."""
    N, K = 256, 128
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.0, seed=51 + rule, B=5)
    da = (fr == 0).astype(np.uint8)
    for prec in ("f64", "f32"):
        for f in range(5):
            sc = O.sc_frame(llr[f], fr, rule=rule, prec=prec)
            for L in (1, 4, 32):
                got = O.scl_frame(llr[f], fr, L, rule=rule, prec=prec, da=da)
                assert np.array_equal(got["u_hat"], sc) and got["n_paths"] == 1


def test_decision_aided_nowhere_is_plain_scl():
    N, K, c, poly = 256, 120, 8, 0x07
    fr, info, u, x, llr = _frame(N, K, c, poly, 1.0, seed=52, B=6)
    a = O.scl_batch(llr, fr, 8, c, poly)
    b = O.scl_batch(llr, fr, 8, c, poly, da=np.zeros(N, np.uint8))
    assert all(np.array_equal(a[k], b[k]) for k in ("u_hat", "crc_ok", "pm"))


@pytest.mark.parametrize("rule", [0, 1])
def test_decision_aided_path_metrics_are_codeword_metrics(rule):
    """Decision-aided positions take the hard decision, so every surviving
    path's metric is still its re-encoded codeword's metric, and each of those
    positions agrees with the hard decision of its path's LLR (the decoded
    codeword is consistent with the decisions)."""
    N, K, L, n_da = 256, 128, 8, 40
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.0, seed=53 + rule, B=4)
    da = O.decision_aided_mask(N, fr, n_da, 2.0, K / N)
    for f in range(4):
        out = O.scl_frame(llr[f], fr, L, rule=rule, all_paths=True, da=da)
        l64 = llr[f].astype(np.float64)
        for q in range(out["n_paths"]):
            xq = O.polar_transform(out["all_u"][q]).astype(np.int64)
            if rule == 0:
                ref = np.sum(np.abs(l64) * (xq != (l64 < 0)))
            else:
                ref = np.sum(np.logaddexp(0.0, -(1 - 2 * xq) * l64))
            assert abs(out["all_pm"][q] - ref) <= 1e-9 * max(1.0, ref)


def test_decision_aided_mask_is_most_reliable():
    N, K, c, design = 1024, 512, 16, 2.5
    fr = O.ga_frozen(N, K + c, design, K / N)
    m = O.ga_means(N, O.sigma2(design, K / N))
    prev = np.zeros(N, np.uint8)
    for n_da in (0, 1, 50, 300, K + c):
        da = O.decision_aided_mask(N, fr, n_da, design, K / N)
        assert da.sum() == n_da and np.all(da <= (fr == 0)) and np.all(prev <= da)
        if 0 < n_da < K + c:
            rest = (fr == 0) & (da == 0)
            assert m[da == 1].min() >= m[rest].max()
        prev = da
    assert np.array_equal(prev, (fr == 0).astype(np.uint8))


def test_scl_crc_selection_rule():
    N, K, c, poly, L = 128, 56, 8, 0x07, 8
    fr, info, u, x, llr = _frame(N, K, c, poly, 0.5, seed=77, design=2.0, B=40)
    free = np.where(fr == 0)[0]
    picked_non_best = 0
    for f in range(40):
        out = O.scl_frame(llr[f], fr, L, c, poly, all_paths=True)
        oks = []
        for q in range(out["n_paths"]):
            b = out["all_u"][q][free]
            oks.append(np.array_equal(O.crc(b[:K], c, poly), b[K:]))
        oks = np.array(oks)
        pm = out["all_pm"]
        if oks.any():
            cand = np.where(oks)[0]
            q = cand[np.argmin(pm[cand])]
            assert out["crc_ok"] == 1
        else:
            q = int(np.argmin(pm))
            assert out["crc_ok"] == 0
        assert np.array_equal(out["u_hat"], out["all_u"][q])
        picked_non_best += int(q != int(np.argmin(pm)))
    assert picked_non_best > 0  # the CRC changed the choice at least once


def test_scl_noiseless_and_list_ordering():
    N, K, c, poly = 1024, 512, 16, 0x1021
    fr = O.ga_frozen(N, K + c, 2.5, 0.5)
    info = inputs.info_bits(2, K, seed=12)
    u, x = O.encode_batch(info, K, c, poly, fr)
    llr = (3.0 * (1.0 - 2.0 * x)).astype(np.float32)
    for f in range(2):
        out = O.scl_frame(llr[f], fr, 8, c, poly, all_paths=True)
        assert np.array_equal(out["u_hat"], u[f]) and out["crc_ok"] == 1 and out["pm"] == 0.0


@pytest.mark.slow
def test_scl_fer_not_worse_than_sc():
    N, K, c, poly, B = 256, 120, 8, 0x07, 300
    fr, info, u, x, llr = _frame(N, K, c, poly, 1.5, seed=41, B=B)
    sc = np.array([O.sc_frame(llr[f], fr) for f in range(B)])
    scl = O.scl_batch(llr, fr, 8, c, poly)["u_hat"]
    assert np.sum(np.any(scl != u, 1)) <= np.sum(np.any(sc != u, 1))


# ------------------------------------------------------------------ hybrid

@pytest.mark.parametrize("stop", [1, 2])
@pytest.mark.parametrize("rule", [0, 1])
def test_hybrid_is_bp_else_scl(rule, stop):
    """Hybrid of Sec. III, frame by frame: BP's information bits where BP ends
    with its verdict ok (re-encoding stop, or the CRC stop that Sec. II-B
    allows in its place), the list decoder's elsewhere."""
    N, K, c, poly, L = 256, 120, 8, 0x07, 4
    fr, info, u, x, llr = _frame(N, K, c, poly, 1.5, seed=51, B=24)
    h = O.hybrid_batch(llr, fr, K, c, poly, max_iter=40, L=L, rule=rule, stop=stop)
    bp = O.bp_batch(llr, fr, c, poly, max_iter=40, stop=stop, rule=rule)
    sl = O.scl_batch(llr, fr, L, c, poly)
    free = np.where(fr == 0)[0]
    assert 0 < h["used_scl"].sum() < 24
    for f in range(24):
        src = bp["u_hat"][f] if bp["ok"][f] else sl["u_hat"][f]
        assert h["used_scl"][f] == 1 - bp["ok"][f]
        assert np.array_equal(h["info"][f], src[free[:K]])


# ------------------------------------------------------------------ weighted BP

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_wbp_unit_weights_is_plain_bp(prec):
    N, K, T = 256, 128, 6
    n = 8
    fr, info, u, x, llr = _frame(N, K, 0, 0, 2.0, seed=61, B=3)
    W = np.ones((T, 2, n, N))
    for f in range(3):
        a = O.bp_frame(llr[f], fr, max_iter=T, stop=0, W=W, save=True, prec=prec)
        b = O.bp_frame(llr[f], fr, max_iter=T, stop=0, save=True, prec=prec)
        assert np.array_equal(a["save"], b["save"])
        assert np.array_equal(a["llr_u"], b["llr_u"])


@pytest.mark.parametrize("N,T", [(8, 2), (16, 3), (32, 2)])
def test_wbp_gradient_matches_finite_differences(N, T):
    """Central differences on the double oracle at random weights in
    [0.5, 1.5] (away from the min and clip kinks)."""
    n = N.bit_length() - 1
    K = N // 2
    rng = np.random.default_rng(N + T)
    fr = O.ga_frozen(N, K, 0.0, 0.5)
    info = rng.integers(0, 2, (3, K)).astype(np.uint8)
    u, x = O.encode_batch(info, K, 0, 0, fr)
    llr = O.channel_llr(x, rng.standard_normal((3, N)), O.sigma2(0.0, 0.5))
    W = rng.uniform(0.5, 1.5, (T, 2, n, N))
    loss, dW, dl = O.wbp_grad(llr, fr, u, T, W, want_dllr=True)
    eps = 1e-6
    flat = W.reshape(-1)
    idx = rng.choice(flat.size, size=min(flat.size, 80), replace=False)
    bad = 0
    for q in idx:
        wp = flat.copy(); wp[q] += eps
        wm = flat.copy(); wm[q] -= eps
        lp, _ = O.wbp_grad(llr, fr, u, T, wp)
        lm, _ = O.wbp_grad(llr, fr, u, T, wm)
        fd = (lp - lm) / (2 * eps)
        if abs(fd - dW.reshape(-1)[q]) > 1e-6 + 1e-5 * abs(fd):
            bad += 1
    assert bad <= 1, bad
    # gradient with respect to the channel LLRs, perturbing float32 inputs
    # by a float64 step through a wrapper that keeps the double precision
    nz = np.abs(dW).sum()
    assert nz > 0


def test_wbp_loss_value():
    """Loss is the mean binary cross-entropy of P(u_i = 1) = sigmoid(-lam_i)
    over the non-frozen positions."""
    N, K, T = 64, 32, 4
    n = 6
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.0, seed=71, B=5)
    W = np.ones((T, 2, n, N))
    loss, _ = O.wbp_grad(llr, fr, u, T, W)
    lam = O.bp_batch(llr, fr, max_iter=T, stop=0, soft=True)["llr_u"]
    p1 = 1.0 / (1.0 + np.exp(lam))
    free = fr == 0
    bce = -(u * np.log(p1) + (1 - u) * np.log(1 - p1))
    assert abs(loss - bce[:, free].mean()) < 1e-9


def test_wbp_multi_loss_is_sum_of_truncated_final_losses():
    """The first t iterations of a T-iteration decoder are a t-iteration
    decoder, so the loss after every iteration is the sum of the final-iteration
    losses of the truncated decoders, and its weight gradient the sum of their
    gradients (padded with zeros for the later iterations)."""
    N, K, T = 64, 32, 5
    n = 6
    rng = np.random.default_rng(17)
    fr, info, u, x, llr = _frame(N, K, 0, 0, 1.0, seed=72, B=4)
    W = rng.uniform(0.6, 1.4, (T, 2, n, N))
    k = int((fr == 0).sum())
    s = 1.0 / (4 * k)
    loss_m, dW_m, dl_m = O.wbp_grad(llr, fr, u, T, W, scale=s, multi=True, want_dllr=True)
    loss_s, dW_s, dl_s = 0.0, np.zeros_like(W), np.zeros_like(dl_m)
    for t in range(1, T + 1):
        lt, gt, dlt = O.wbp_grad(llr, fr, u, t, W[:t], scale=s, want_dllr=True)
        loss_s += lt
        dW_s[:t] += gt
        dl_s += dlt
    assert abs(loss_m - loss_s) <= 1e-12 * max(1.0, abs(loss_s))
    assert np.allclose(dW_m, dW_s, rtol=1e-9, atol=1e-15)
    assert np.allclose(dl_m, dl_s, rtol=1e-9, atol=1e-15)
    assert np.abs(dW_m[0]).sum() > 0


def test_wbp_multi_loss_gradient_matches_finite_differences():
    N, T = 16, 3
    n = 4
    K = 8
    rng = np.random.default_rng(5)
    fr = O.ga_frozen(N, K, 0.0, 0.5)
    info = rng.integers(0, 2, (3, K)).astype(np.uint8)
    u, x = O.encode_batch(info, K, 0, 0, fr)
    llr = O.channel_llr(x, rng.standard_normal((3, N)), O.sigma2(0.0, 0.5))
    W = rng.uniform(0.5, 1.5, (T, 2, n, N))
    loss, dW = O.wbp_grad(llr, fr, u, T, W, multi=True)
    eps = 1e-6
    flat = W.reshape(-1)
    bad = 0
    for q in rng.choice(flat.size, size=60, replace=False):
        wp = flat.copy(); wp[q] += eps
        wm = flat.copy(); wm[q] -= eps
        fd = (O.wbp_grad(llr, fr, u, T, wp, multi=True)[0] - O.wbp_grad(llr, fr, u, T, wm, multi=True)[0]) / (2 * eps)
        if abs(fd - dW.reshape(-1)[q]) > 1e-6 + 1e-5 * abs(fd):
            bad += 1
    assert bad <= 1, bad


def test_wbp_channel_gradient_matches_finite_differences():
    """d loss / d llr against central differences on the double oracle.  The
    LLRs are rounded to multiples of 2^-12 and perturbed by +-2^-12, so every
    perturbed input is an exact float32 (the oracle's input type); a few
    channel LLRs lie beyond the clipping level, where the loss does not depend
    on them (the clip at load has derivative 0)."""
    N, T, K = 16, 3, 8
    n = 4
    rng = np.random.default_rng(23)
    fr = O.ga_frozen(N, K, 0.0, 0.5)
    info = rng.integers(0, 2, (3, K)).astype(np.uint8)
    u, x = O.encode_batch(info, K, 0, 0, fr)
    llr = O.channel_llr(x, rng.standard_normal((3, N)), O.sigma2(0.0, 0.5)).astype(np.float64)
    llr[0, 3] = 25.0
    llr[1, 9] = -23.5
    llr[2, 0] = 20.75
    # the last node with a wrong-signed LLR beyond the clip: without the clip at
    # load its adjoint would be -1/24 here (the sums it enters stay unclipped)
    llr[:, N - 1] = 22.0 * (2.0 * x[:, N - 1] - 1.0)
    h = 2.0 ** -12
    llr = (np.round(llr / h) * h).astype(np.float32)
    W = rng.uniform(0.5, 1.5, (T, 2, n, N))
    s = 1.0 / (3 * K)
    _, _, dl = O.wbp_grad(llr, fr, u, T, W, scale=s, want_dllr=True)
    assert np.all(dl[np.abs(llr) > 20] == 0)
    bad = 0
    for f in range(3):
        for i in range(N):
            lp = llr[f:f + 1].copy(); lp[0, i] += np.float32(h)
            lm = llr[f:f + 1].copy(); lm[0, i] -= np.float32(h)
            assert float(lp[0, i]) - float(llr[f, i]) == h and float(llr[f, i]) - float(lm[0, i]) == h
            fd = (O.wbp_grad(lp, fr, u[f:f + 1], T, W, scale=s)[0]
                  - O.wbp_grad(lm, fr, u[f:f + 1], T, W, scale=s)[0]) / (2 * h)
            if abs(fd - dl[f, i]) > 1e-6 + 1e-4 * abs(fd):
                bad += 1
    assert bad <= 1, bad
    assert np.count_nonzero(dl) >= 30


def test_adam_first_step_closed_form():
    """Step 1: m_hat = g, v_hat = g^2, so each weight moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    g = rng.normal(size=100)
    w = np.ones(100)
    m = np.zeros(100)
    v = np.zeros(100)
    O.adam_step(w, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(w, 1.0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _truncated_S(llr, fr, u, W, T):
    """S_t per frame: the BCE sum over the non-frozen bits of LLR(u) from a
    separate t-iteration decode (no early stop), t = 1..T."""
    free = fr == 0
    S = np.zeros((llr.shape[0], T))
    for t in range(1, T + 1):
        lam = O.bp_batch(llr, fr, max_iter=t, stop=0, W=W[:t], soft=True)["llr_u"]
        z = np.where(u == 1, 1.0, -1.0) * lam
        S[:, t - 1] = np.logaddexp(0.0, z)[:, free].sum(axis=1)
    return S


def test_wbp_frame_loss_value():
    """Loss kind 2 is the mean over frames of prod_t (1 - exp(-S_t)), S_t the
    BCE sum of LLR(u) after iteration t, here taken from separate truncated
    decodes; frames decoded right early get a loss near 0, frames that stay
    wrong a loss near 1."""
    N, K, T = 64, 32, 5
    n = 6
    rng = np.random.default_rng(19)
    fr, info, u, x, llr = _frame(N, K, 0, 0, 0.5, seed=74, B=6)
    W = rng.uniform(0.6, 1.2, (T, 2, n, N))
    loss = O.wbp_grad(llr, fr, u, T, W, kind=2)[0]
    S = _truncated_S(llr, fr, u, W, T)
    ref = np.mean(np.prod(1.0 - np.exp(-S), axis=1))
    assert abs(loss - ref) <= 1e-12 * max(1.0, ref)
    # the loss of one frame is the probability, bits independent, that no
    # iteration's decisions are all right
    per = [O.wbp_grad(llr[f:f + 1], fr, u[f:f + 1], T, W, kind=2, scale=1.0)[0] for f in range(6)]
    assert np.all((np.array(per) >= 0) & (np.array(per) <= 1))
    # noiseless frames: every iteration right with high probability
    clean = np.where(x == 0, 8.0, -8.0).astype(np.float32)
    assert O.wbp_grad(clean, fr, u, T, W, kind=2)[0] < 1e-6


def test_wbp_frame_loss_single_iteration_closed_form():
    """T = 1: 1 - exp(-S) with S the final-iteration BCE sum; its gradient is
    exp(-S) times the BCE gradient (chain rule through the outer function)."""
    N, K = 32, 16
    n = 5
    rng = np.random.default_rng(3)
    fr, info, u, x, llr = _frame(N, K, 0, 0, 0.0, seed=75, B=1)
    W = rng.uniform(0.6, 1.2, (1, 2, n, N))
    l2, g2 = O.wbp_grad(llr, fr, u, 1, W, kind=2, scale=1.0)
    l0, g0 = O.wbp_grad(llr, fr, u, 1, W, kind=0, scale=1.0)
    assert abs(l2 - (1.0 - np.exp(-l0))) <= 1e-14
    np.testing.assert_allclose(g2, np.exp(-l0) * g0, rtol=1e-12, atol=1e-300)


def test_wbp_frame_loss_gradient_matches_finite_differences():
    """Weight and channel-LLR gradients of the frame-failure loss against
    central differences on the double oracle (channel LLRs on a 2^-12 grid,
    perturbed by +-2^-12, so every input stays an exact float32)."""
    N, T, K = 16, 3, 8
    n = 4
    rng = np.random.default_rng(29)
    fr = O.ga_frozen(N, K, 0.0, 0.5)
    info = rng.integers(0, 2, (3, K)).astype(np.uint8)
    u, x = O.encode_batch(info, K, 0, 0, fr)
    llr = O.channel_llr(x, rng.standard_normal((3, N)), O.sigma2(-1.0, 0.5)).astype(np.float64)
    h = 2.0 ** -12
    llr = (np.round(llr / h) * h).astype(np.float32)
    W = rng.uniform(0.5, 1.5, (T, 2, n, N))
    loss, dW, dl = O.wbp_grad(llr, fr, u, T, W, kind=2, want_dllr=True)
    assert 0.05 < loss < 0.95
    eps = 1e-6
    flat = W.reshape(-1)
    bad = 0
    for q in rng.choice(flat.size, size=60, replace=False):
        wp = flat.copy(); wp[q] += eps
        wm = flat.copy(); wm[q] -= eps
        fd = (O.wbp_grad(llr, fr, u, T, wp, kind=2)[0] - O.wbp_grad(llr, fr, u, T, wm, kind=2)[0]) / (2 * eps)
        if abs(fd - dW.reshape(-1)[q]) > 1e-7 + 1e-5 * abs(fd):
            bad += 1
    assert bad <= 1, bad
    assert np.abs(dW).max() > 1e-4
    bad = 0
    for f in range(3):
        for i in range(N):
            lp = llr.copy(); lp[f, i] += np.float32(h)
            lm = llr.copy(); lm[f, i] -= np.float32(h)
            fd = (O.wbp_grad(lp, fr, u, T, W, kind=2)[0] - O.wbp_grad(lm, fr, u, T, W, kind=2)[0]) / (2 * h)
            if abs(fd - dl[f, i]) > 1e-6 + 1e-4 * abs(fd):
                bad += 1
    assert bad <= 1, bad
    assert np.count_nonzero(dl) >= 30


def test_wbp_iteration_loss_value():
    """Loss kind 3: sum over u < T of P_u plus c P_T, P_u = prod_{t<=u}
    (1 - exp(-S_t)) with S_t from separate truncated decodes; noiseless frames
    cost nothing, hopeless ones T - 1 + c."""
    N, K, T, c = 64, 32, 5, 7.5
    n = 6
    rng = np.random.default_rng(23)
    fr, info, u, x, llr = _frame(N, K, 0, 0, 0.5, seed=76, B=6)
    W = rng.uniform(0.6, 1.2, (T, 2, n, N))
    loss = O.wbp_grad(llr, fr, u, T, W, kind=3, fail_weight=c)[0]
    S = _truncated_S(llr, fr, u, W, T)
    P = np.cumprod(1.0 - np.exp(-S), axis=1)
    ref = np.mean(P[:, :-1].sum(axis=1) + c * P[:, -1])
    assert abs(loss - ref) <= 1e-12 * max(1.0, ref)
    # noiseless frames at the clip level, plain min-sum: every iteration is
    # right with certainty, so nothing is left to pay
    ones = np.ones_like(W)
    clean = np.where(x == 0, 20.0, -20.0).astype(np.float32)
    assert O.wbp_grad(clean, fr, u, T, ones, kind=3, fail_weight=c)[0] < 1e-6
    wrong = np.where(x == 0, -20.0, 20.0).astype(np.float32)  # every channel value points the wrong way
    lw = O.wbp_grad(wrong, fr, u, T, ones, kind=3, fail_weight=c)[0]
    assert abs(lw - (T - 1 + c)) < 1e-6


def test_wbp_iteration_loss_affine_in_fail_weight():
    """The fail-weight term is the kind-2 loss: L(c1) - L(c2) = (c1 - c2) F for
    the value and the gradient; at T = 1 the loss is c F exactly."""
    N, K, T = 32, 16, 4
    n = 5
    rng = np.random.default_rng(6)
    fr, info, u, x, llr = _frame(N, K, 0, 0, 0.0, seed=77, B=3)
    W = rng.uniform(0.6, 1.2, (T, 2, n, N))
    l1, g1 = O.wbp_grad(llr, fr, u, T, W, kind=3, fail_weight=9.0)
    l2, g2 = O.wbp_grad(llr, fr, u, T, W, kind=3, fail_weight=2.0)
    lf, gf = O.wbp_grad(llr, fr, u, T, W, kind=2)
    assert abs((l1 - l2) - 7.0 * lf) <= 1e-12 * max(1.0, abs(l1))
    np.testing.assert_allclose(g1 - g2, 7.0 * gf, rtol=1e-9, atol=1e-14 * np.abs(g1).max())
    W1 = W[:1]
    l3, g3 = O.wbp_grad(llr, fr, u, 1, W1, kind=3, fail_weight=3.0)
    l4, g4 = O.wbp_grad(llr, fr, u, 1, W1, kind=2)
    assert abs(l3 - 3.0 * l4) <= 1e-14
    np.testing.assert_allclose(g3, 3.0 * g4, rtol=1e-12, atol=1e-300)


def test_wbp_iteration_loss_gradient_matches_finite_differences():
    """Weight and channel-LLR gradients of the iteration loss against central
    differences on the double oracle (LLRs on a 2^-12 grid perturbed by
    +-2^-12, exact float32 inputs)."""
    N, T, K, c = 16, 3, 8, 5.0
    n = 4
    rng = np.random.default_rng(31)
    fr = O.ga_frozen(N, K, 0.0, 0.5)
    info = rng.integers(0, 2, (3, K)).astype(np.uint8)
    u, x = O.encode_batch(info, K, 0, 0, fr)
    llr = O.channel_llr(x, rng.standard_normal((3, N)), O.sigma2(-1.0, 0.5)).astype(np.float64)
    h = 2.0 ** -12
    llr = (np.round(llr / h) * h).astype(np.float32)
    W = rng.uniform(0.5, 1.5, (T, 2, n, N))
    loss, dW, dl = O.wbp_grad(llr, fr, u, T, W, kind=3, fail_weight=c, want_dllr=True)
    assert 0.05 < loss < T - 1 + c - 0.05
    eps = 1e-6
    flat = W.reshape(-1)
    bad = 0
    for q in rng.choice(flat.size, size=60, replace=False):
        wp = flat.copy(); wp[q] += eps
        wm = flat.copy(); wm[q] -= eps
        fd = (O.wbp_grad(llr, fr, u, T, wp, kind=3, fail_weight=c)[0]
              - O.wbp_grad(llr, fr, u, T, wm, kind=3, fail_weight=c)[0]) / (2 * eps)
        if abs(fd - dW.reshape(-1)[q]) > 1e-7 + 1e-5 * abs(fd):
            bad += 1
    assert bad <= 1, bad
    assert np.abs(dW).max() > 1e-4
    bad = 0
    for f in range(3):
        for i in range(N):
            lp = llr.copy(); lp[f, i] += np.float32(h)
            lm = llr.copy(); lm[f, i] -= np.float32(h)
            fd = (O.wbp_grad(lp, fr, u, T, W, kind=3, fail_weight=c)[0]
                  - O.wbp_grad(lm, fr, u, T, W, kind=3, fail_weight=c)[0]) / (2 * h)
            if abs(fd - dl[f, i]) > 1e-6 + 1e-4 * abs(fd):
                bad += 1
    assert bad <= 1, bad
    assert np.count_nonzero(dl) >= 30
