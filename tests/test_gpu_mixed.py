"""GPU parity of the ragged mixed-code hybrid (polar_mixed_*).

The workload mixes twelve codes, N in {256, 512, 1024, 2048} and rates
{1/4, 1/2, 3/4}, CRC-16, frozen sets by Gaussian approximation at 2 dB, with
a per-frame Eb/N0 uniform in [1, 3] dB and the frames in random order.  The
mixed decoder runs the same BP and CA-SCL arithmetic as the single-code
hybrid, so every frame must match the single-code decoder bit for bit, and a
sample of frames the oracle's float build; the hipGraph replay must match the
eager call on every replay.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1609_09358_amd import binding as PB
from paper_1609_09358_amd import inputs

pytestmark = pytest.mark.gpu
CRC16 = 0x1021


def make_codes(Ns=(256, 512, 1024, 2048), rates=(0.25, 0.5, 0.75)):
    return [PB.PolarCode(N, int(N * r), 16, 0, 2.0) for N in Ns for r in rates]


def mixed_batch(plan, B, seed, lo=1.0, hi=3.0):
    """Ragged batch laid out densely in frame order (host arrays)."""
    codes = plan.codes
    cf = inputs.choice(B, codes, seed).astype(np.int32)
    ebn0 = inputs.ebn0_uniform(B, lo, hi, seed)
    llr_off, out_off, tot, totk = plan.layout(cf)
    llr = np.zeros(tot, np.float32)
    info = np.zeros(totk, np.uint8)
    for c, code in enumerate(codes):
        idx = np.where(cf == c)[0]
        if len(idx) == 0:
            continue
        bits = inputs.info_bits(len(idx), code.K, seed * 100 + c)
        _, x = O.encode_batch(bits, code.K, 16, CRC16, code.frozen)
        z = inputs.noise(len(idx), code.N, seed * 100 + c)
        s2 = np.array([O.sigma2(e, code.K / code.N) for e in ebn0[idx]])
        rows = O.channel_llr(x, z, s2)
        for j, f in enumerate(idx):
            llr[llr_off[f]:llr_off[f] + code.N] = rows[j]
            info[out_off[f]:out_off[f] + code.K] = bits[j]
    return cf, llr_off, out_off, llr, info


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(plan, cf, llr_off, out_off, llr, totk, graph=False):
    B = len(cf)
    info_hat = torch.full((totk,), 7, dtype=torch.uint8, device="cuda")
    used = torch.full((B,), 9, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    plan(dev(llr), dev(cf), dev(llr_off), dev(out_off), info_hat, used, stats, graph=graph)
    torch.cuda.synchronize()
    return info_hat.cpu().numpy(), used.cpu().numpy(), stats.cpu().numpy()


def test_mixed_matches_single_code_hybrid_and_oracle():
    codes = make_codes()
    it, L, B = 60, 8, 700
    plan = PB.MixedPlan(codes, max_frames=1024, max_iter=it, L=L)
    cf, llr_off, out_off, llr, info = mixed_batch(plan, B, seed=5)
    info_hat, used, st = run(plan, cf, llr_off, out_off, llr, len(info))
    assert st[0] == B and st[1] + st[2] == B and st[2] == used.sum()
    assert 0 < used.sum() < B
    rng = np.random.default_rng(1)
    for c, code in enumerate(codes):
        idx = np.where(cf == c)[0]
        rows = np.stack([llr[llr_off[f]:llr_off[f] + code.N] for f in idx])
        one = PB.HybridDecoder(code, max_iter=it, L=L)(dev(rows))
        got = np.stack([info_hat[out_off[f]:out_off[f] + code.K] for f in idx])
        assert np.array_equal(got, one["info"].cpu().numpy()), f"code {c}"
        assert np.array_equal(used[idx], one["used_scl"].cpu().numpy()), f"code {c}"
        # a few frames of each code, failed ones first, against the oracle
        pick = np.concatenate([np.where(used[idx] == 1)[0][:2], rng.choice(len(idx), 2, replace=False)])
        ref = O.hybrid_batch(rows[pick], code.frozen, code.K, 16, CRC16, it, L, prec="f32")
        assert np.array_equal(got[pick], ref["info"]), f"code {c}"
        assert np.array_equal(used[idx][pick], ref["used_scl"]), f"code {c}"
    fer = np.mean([np.any(info_hat[out_off[f]:out_off[f] + codes[cf[f]].K] != info[out_off[f]:out_off[f] + codes[cf[f]].K])
                   for f in range(B)])
    assert fer < 0.4  # rate-3/4 codes near 1 dB fail often; hard decisions alone fail almost always


def test_mixed_graph_replays_match_eager():
    """Captured once, replayed with two different batches in turn (other
    buffers, other sizes), eager work and synchronizations in between."""
    codes = make_codes(Ns=(256, 1024), rates=(0.5, 0.75))
    plan = PB.MixedPlan(codes, max_frames=512, max_iter=40, L=4)
    batches = [mixed_batch(plan, 300, seed=11), mixed_batch(plan, 157, seed=12)]
    eager = [run(plan, cf, lo, oo, llr, len(info)) for cf, lo, oo, llr, info in batches]
    for rep in range(4):
        cf, lo, oo, llr, info = batches[rep % 2]
        g = run(plan, cf, lo, oo, llr, len(info), graph=True)
        e = eager[rep % 2]
        assert np.array_equal(g[0], e[0]) and np.array_equal(g[1], e[1]) and np.array_equal(g[2], e[2]), rep
        # eager decoding between replays
        e2 = run(plan, cf, lo, oo, llr, len(info))
        assert np.array_equal(e2[0], e[0])


def test_mixed_edge_cases():
    codes = make_codes(Ns=(256,), rates=(0.5,))
    plan = PB.MixedPlan(codes, max_frames=64, max_iter=20, L=2)
    cf, lo, oo, llr, info = mixed_batch(plan, 10, seed=3)
    # an out-of-range code id is skipped: its output and flag stay untouched
    cf_bad = cf.copy()
    cf_bad[4] = 5
    info_hat, used, st = run(plan, cf_bad, lo, oo, llr, len(info))
    ok_rows = [f for f in range(10) if f != 4]
    ref, ref_used, _ = run(plan, cf, lo, oo, llr, len(info))
    for f in ok_rows:
        assert np.array_equal(info_hat[oo[f]:oo[f] + 128], ref[oo[f]:oo[f] + 128])
    assert np.all(info_hat[oo[4]:oo[4] + 128] == 7) and used[4] == 9 and st[0] == 9
    # empty call, and more frames than the plan holds
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    e64 = torch.empty(0, dtype=torch.int64, device="cuda")
    ef = torch.empty(0, dtype=torch.float32, device="cuda")
    eu = torch.empty(0, dtype=torch.uint8, device="cuda")
    plan(ef, e, e64, e64, eu)
    big = torch.zeros(65, dtype=torch.int32, device="cuda")
    big64 = torch.zeros(65, dtype=torch.int64, device="cuda")
    with pytest.raises(PB.PolarError):
        plan(torch.zeros(256, device="cuda"), big, big64, big64, torch.zeros(65 * 128, dtype=torch.uint8,
                                                                              device="cuda"))


def test_autotuned_plan_decodes_identically():
    """The tuner picks layouts and an LDS budget; decoding results do not
    depend on them."""
    from paper_1609_09358_amd import autotune
    from paper_1609_09358_amd import mixed_workload as MW
    codes = MW.make_codes(Ns=(256, 1024), rates=(0.5,))
    batch = MW.ragged_batch(codes, 400, seed=21)
    base = PB.MixedPlan(codes, max_frames=400, max_iter=50, L=8)
    out0 = torch.empty(batch["total_info_bits"], dtype=torch.uint8, device="cuda")
    args = (batch["llr"], batch["code_of_frame"], batch["llr_off"], batch["out_off"])
    base(*args, out0)
    try:
        tuned = autotune.tune_mixed(codes, [rows for _, rows in batch["per_code"]], 50, 8)
        assert all(v in PB.polar_bp_variants(c.N) for v, c in zip(tuned["variants"], codes))
        plan = PB.MixedPlan(codes, max_frames=400, max_iter=50, L=8, variants=tuned["variants"])
        out1 = torch.empty_like(out0)
        plan(*args, out1, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out0, out1)
        # whole-plan tuning (longest bucket's layout, LDS budget)
        used = torch.empty(400, dtype=torch.uint8, device="cuda")
        out2 = torch.empty_like(out0)
        tp = autotune.tune_mixed_plan(codes, args + (out2, used), 50, 8, tuned["variants"], budgets=(0, 16384), reps=2)
        assert all(v in PB.polar_bp_variants(c.N) for v, c in zip(tp["variants"], codes))
        plan2 = PB.MixedPlan(codes, max_frames=400, max_iter=50, L=8, variants=tp["variants"])
        out3 = torch.empty_like(out0)
        plan2(*args, out3, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out0, out3)
    finally:
        PB.polar_set_scl_lds_budget(0)


def test_mixed_short_codes_take_their_own_branch():
    """Codes shorter than 32 bits form one group each; codes of one block
    length share a group (one BP kernel and one list decoder, each frame with
    its own code).  Every frame must match the single-code hybrid."""
    from paper_1609_09358_amd import mixed_workload as MW
    codes = [PB.PolarCode(16, 4, 8, 0, 2.0), PB.PolarCode(8, 2, 0, 0, 2.0),
             PB.PolarCode(256, 64, 8, 0, 2.0), PB.PolarCode(256, 160, 8, 0, 2.0)]
    it, L, B = 30, 4, 500
    batch = MW.ragged_batch(codes, B, seed=31)
    plan = PB.MixedPlan(codes, max_frames=B, max_iter=it, L=L)
    info_hat = torch.full((batch["total_info_bits"],), 7, dtype=torch.uint8, device="cuda")
    used = torch.full((B,), 9, dtype=torch.uint8, device="cuda")
    plan(batch["llr"], batch["code_of_frame"], batch["llr_off"], batch["out_off"], info_hat, used, graph=True)
    torch.cuda.synchronize()
    oo = batch["out_off"].cpu().numpy()
    got_all, used_all = info_hat.cpu().numpy(), used.cpu().numpy()
    for c, code in enumerate(codes):
        ids, rows = batch["per_code"][c]
        if ids.numel() == 0:
            continue
        one = PB.HybridDecoder(code, max_iter=it, L=L)(rows.contiguous())
        idx = ids.cpu().numpy()
        got = np.stack([got_all[oo[f]:oo[f] + code.K] for f in idx])
        assert np.array_equal(got, one["info"].cpu().numpy()), f"code {c}"
        assert np.array_equal(used_all[idx], one["used_scl"].cpu().numpy()), f"code {c}"
