"""Benchmark: decoded information throughput of the learned hybrid decoder.

Workload (synthetic, seeded): polar code N = 1024, K = 512 information bits
plus CRC-24, frozen set by Gaussian approximation at 2.5 dB; uniform random
information bits, BPSK over AWGN at Eb/N0 = 2.5 dB (rate K/N).

One step is one hybrid decode of a resident batch of frames: weighted
(learned) min-sum BP with at most T = 20 iterations, stopping as soon as the
CRC of its decided information bits holds (Sec. II-B allows the CRC in place
of the re-encoding check), device-side compaction of the frames it did not
finish,
CA-SCL with list size 32 on them (with the decision aiding of Sec. II-A on the
320 most reliable information positions: on 39192 frames the learned BP
failed at 2.5 dB it made the same frame errors as plain CA-SCL for every count
up to 320), merge.  Steps run through the two-stream
pipeline (BP and compaction of step j + 1 overlap the CA-SCL and merge of
step j, the asynchronous scheduling of Sec. III); the single-stream time is
reported beside.  The LLRs are in HBM before the timed region starts; host
transfers are excluded.

The learned decoder has one weight per (iteration, sweep direction, stage
column), shared by the column's nodes.  Its weights are trained before timing
(untimed, seeded, on frames drawn apart from the timed ones): the normalized
min-sum scale with the fewest BP failures on validation frames is the start,
then Adam on the frame-failure loss (the probability, bits taken as
independent, that no iteration decides the whole frame right) runs through the
library's own forward and adjoint kernels, each weight kept within [0, 1] (a
learned weight never amplifies a message).  The derivative-free coordinate
search on the failure rate is reported beside it for comparison.  The plain
hybrid (unweighted BP, at most 200 iterations, then CA-SCL with list size 32
and no decision aiding) decodes the same
frames for comparison; the throughput counts only if the learned decoder's
frame error rate does not exceed the upper 95% Clopper-Pearson bound of the
plain decoder's on a common set of frames.

Printed: one JSON line with the throughput, a roofline entry for the kernel
that takes most of the step's time (measured with HIP events on the stream
the kernels run on), and the CPU oracle timed on a bounded sample of the same
workload on the host cores.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures
HBM_PEAK_GBS = 8000.0
# fp32 vector: 157.3 TFLOP/s counting a fused multiply-add as two operations,
# i.e. 128 single-precision lane operations per CU per clock at 2.4 GHz, the
# peak for the BP kernel's operations (add, multiply, fused multiply-add,
# med3, bit operation) counted one each.  A probe of independent add, fma or
# med3 chains, of one kind or mixed, issues at half that (38 T/s); the BP
# kernel measured above it (47.6 T VALU lane-instructions/s)
CU, FP32_LANES_PER_CU_CLOCK, CLOCK_GHZ = 256, 128, 2.4
VALU_PEAK_GOPS = CU * FP32_LANES_PER_CU_CLOCK * CLOCK_GHZ

POLY24 = 0x864CFB
# early stop of the learned BP: the CRC of the decided information bits (Sec.
# II-B allows it in place of the re-encoding check); the plain comparator
# keeps the re-encoding check
STOP = 2
# fine-tuning of the learned weights on the expected-iterations loss: a frame
# BP leaves to the list decoder counts as FAIL_WEIGHT BP iterations (the step's
# time model, the list decoder's frame latency over the chip's wave slots
# against BP's time per iteration, gives about 57; 40, 57 and 80 measured alike
# within noise, 40 the fastest)
FAIL_WEIGHT = 40.0
ITER_SCHEDULE = ((1e-3, 1500),)

# HBM bytes per 65536-frame launch of the weighted BP kernel (one weight per
# stage column, CRC stop) as the per-kernel timing loop runs it (u_hat
# written), from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a device copy of
# known size; valid only for the kernel sources they were measured on (hash of
# the files below) and that stop rule
BP_TRAFFIC = {"bytes": 354132792, "frames": 65536, "stop": 2, "src_sha256_16": "7fbfbbecc642d8ec"}
BP_SOURCES = ("paper_1609_09358_amd/csrc/bp.hip", "paper_1609_09358_amd/csrc/bp_common.hpp",
              "paper_1609_09358_amd/csrc/bp_geom.hpp")


def bp_traffic(frames):
    import hashlib
    h = hashlib.sha256()
    for f in BP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if (h.hexdigest()[:16] != BP_TRAFFIC["src_sha256_16"] or frames != BP_TRAFFIC["frames"]
            or STOP != BP_TRAFFIC["stop"]):
        return None
    return BP_TRAFFIC["bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=65536, help="frames per step")
    ap.add_argument("--ebn0", type=float, default=2.5)
    ap.add_argument("--T", type=int, default=20, help="learned BP iterations")
    ap.add_argument("--L", type=int, default=32, help="list size")
    ap.add_argument("--train-frames", type=int, default=1_000_000, help="training frames of the N=256 learned BP")
    ap.add_argument("--fer-frames", type=int, default=1 << 20, help="frames per decoder for the FER comparison")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only the per-kernel timing loops of the learned BP and the list decoder (for profilers)")
    ap.add_argument("--profile-pipeline", action="store_true",
                    help="only the headline's tuning and its K pipelined steps (for kernel traces)")
    ap.add_argument("--skip-extras", action="store_true",
                    help="only the headline, its FER check and per-kernel timing (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    return ap.parse_args()


def cp_upper(k, n, conf=0.95):
    """Upper end of the two-sided Clopper-Pearson interval of k errors in n."""
    from scipy.stats import beta
    return 1.0 if k >= n else float(beta.ppf(1 - (1 - conf) / 2, k + 1, n - k))


def cp_lower(k, n, conf=0.95):
    """Lower end of the two-sided Clopper-Pearson interval of k errors in n."""
    from scipy.stats import beta
    return 0.0 if k <= 0 else float(beta.ppf((1 - conf) / 2, k, n - k + 1))


def host_cpu():
    """Host CPU description: model name, logical CPUs, CPUs this process may
    use, and the thread budget of the environment (OMP_NUM_THREADS)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    budget = os.environ.get("OMP_NUM_THREADS", "")
    return {"model": model, "nproc": os.cpu_count(), "usable": usable,
            "omp_num_threads": int(budget) if budget.isdigit() else None}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); frames are independent, so a multi-GPU "
              "run would shard the batch; it is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import inputs
    from paper_1609_09358_amd import train_wbp as TW

    torch.cuda.set_device(0)
    N, K, C, DESIGN, T, L, IMAX, DA = 1024, 512, 24, 2.5, args.T, args.L, 200, 320
    n = N.bit_length() - 1
    B = args.frames
    R = K / N
    sigma2 = 1.0 / (2.0 * R * 10.0 ** (args.ebn0 / 10.0))
    code = PB.PolarCode(N, K, C, POLY24, DESIGN, da_bits=DA)
    # the configured comparator: plain BP then plain CA-SCL (no decision aiding)
    code_plain = PB.PolarCode(N, K, C, POLY24, DESIGN, da_bits=0)
    assert np.array_equal(code_plain.frozen, code.frozen)
    log = lambda **kw: print(json.dumps(kw), file=sys.stderr, flush=True)

    # ---- learned weights (untimed, seeded, on frames drawn apart from the timed
    # ones): the normalized min-sum scale with the fewest BP failures on
    # validation frames, then Adam on the frame-failure loss through the
    # library's forward and adjoint kernels (one weight per stage column, kept
    # within [0, 1]), then Adam on the expected-iterations loss (the iterations
    # a frame runs plus FAIL_WEIGHT for a frame BP leaves to the list decoder:
    # the step's cost in BP iterations); beside it, for comparison, the
    # derivative-free coordinate search on the failure rate that fitted the
    # weights before
    t_fit = time.perf_counter()
    val_gen = TW.Trainer(code, 1, 16, seed=9358)
    _, _, val_llr = val_gen.frames(1 << 17, ebn0=args.ebn0)
    W0, alpha, rate0 = TW.fit_scale(code, val_llr, T, per_stage=True, stop=STOP)
    tr, seen = TW.train_front_end(code, T, alpha, args.ebn0)
    W_frame = tr.W.clone()
    tr2, seen2 = TW.train_front_end(code, T, W_frame, args.ebn0, schedule=ITER_SCHEDULE, loss="iter",
                                    fail_weight=FAIL_WEIGHT)
    W = tr2.W.clone()
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t_fit

    def val_stats(Wx):
        o = PB.bp_decode_batch(code, val_llr, max_iter=T, stop=STOP, weights=Wx)
        return {"bp_fail_rate": round(1.0 - float(o["ok"].float().mean()), 6),
                "mean_iterations": round(float(o["iters"].float().mean()), 4)}

    weights_info = {"layout": "per stage column [T][2][n]", "alpha": alpha,
                    "training": {"loss": "frame failure, then expected iterations with fail weight %g"
                                 % FAIL_WEIGHT, "optimizer": "Adam, projected onto [0, 1]",
                                 "schedule": "lr 3e-3 x 1500 steps, 1e-3 x 1000 steps; then lr 1e-3 x %d steps"
                                 % ITER_SCHEDULE[0][1], "batch": tr.B,
                                 "frames": seen + seen2, "seconds": round(fit_s, 1)},
                    "validation_frames": int(val_llr.shape[0]),
                    "val_plain_min_sum": val_stats(torch.ones_like(W)), "val_alpha": val_stats(W0),
                    "val_frame_loss": val_stats(W_frame), "val_trained": val_stats(W)}
    del W_frame
    if not (args.profile_kernels or args.profile_pipeline):
        t_s = time.perf_counter()
        Ws1, _ = TW.refine_blocks(code, val_llr, W0.clone(), wmax=1.0, stop=STOP)
        Ws, _ = TW.refine_blocks(code, val_llr, Ws1, per_column=True, wmax=1.0, stop=STOP)
        weights_info["val_coordinate_search"] = dict(val_stats(Ws), seconds=round(time.perf_counter() - t_s, 1))
        del Ws, Ws1
    log(stage="weights", **weights_info)
    del val_llr

    # ---- synthetic frames, resident in HBM (untimed)
    seed = 20161
    info = inputs.info_bits(B, K, seed)
    z = inputs.noise(B, N, seed, dtype=np.float32)
    info_d = torch.from_numpy(info).cuda()
    x_d = PB.polar_encode(code, info_d)
    llr = PB.polar_channel_awgn(x_d, torch.from_numpy(z).cuda(),
                                torch.full((B,), sigma2, dtype=torch.float32, device="cuda"))
    del x_d
    torch.cuda.synchronize()

    if args.profile_kernels:
        # only the per-kernel timing loops (for rocprofv3 runs): the BP kernel
        # and the list decoder as the roofline entry measures them
        kt = kernel_times(code, llr, W, T, L, max(3, args.steps // 2))
        kt.pop("bp_out")
        if args.copy_calibration:
            src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            kt["copy_calibration_bytes"] = src.numel() * 4
        w_unit = float(W.abs().max()) <= 1.0
        ops = (7.0 if w_unit else 8.0) * n * N * kt["iter_sum"]
        print(json.dumps(dict(kt, frames=B, grid_bp_workgroups=B, ops_per_pe_sweep=7 if w_unit else 8,
                              bp_ops_per_launch=ops, bp_Tops=round(ops / (kt["bp_ms"] * 1e-3) / 1e12, 4),
                              weights_max_abs=float(W.abs().max()))))
        return

    learned = PB.HybridDecoder(code, max_iter=T, L=L, stop=STOP, weights=W)
    plain = PB.HybridDecoder(code_plain, max_iter=IMAX, L=L, stop=1)
    learned_pipe = PB.HybridPipeline(code, max_iter=T, L=L, stop=STOP, weights=W)
    plain_pipe = PB.HybridPipeline(code_plain, max_iter=IMAX, L=L, stop=1)
    out = learned(llr)
    out_p = plain(llr)
    torch.cuda.synchronize()

    def run_steps(dec, o, steps, warmup):
        for _ in range(warmup):
            dec(llr, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dec(llr, out=o)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def run_pipe(pipe, o, steps, warmup):
        # consecutive batches of a call write different outputs (two buffers
        # alternate; batch j + 2 starts after batch j is merged)
        o2 = {"info": torch.empty_like(o["info"])}
        alt = lambda k: [o if i % 2 == 0 else o2 for i in range(k)]
        pipe([llr] * warmup, outs=alt(warmup))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pipe([llr] * steps, outs=alt(steps))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if args.profile_pipeline:
        # only the headline's pipelined steps (for rocprofv3 kernel traces): the
        # untimed tuning, then W + K steps of the learned hybrid, the last K timed
        from paper_1609_09358_amd import autotune
        occ = autotune.tune_pipeline(learned_pipe, llr)
        elapsed = run_pipe(learned_pipe, out, args.steps, args.warmup)
        print(json.dumps(dict(steps=args.steps, warmup=args.warmup, frames=B,
                              ms_per_step=round(1e3 * elapsed / args.steps, 4),
                              Gbps=round(B * K * args.steps / elapsed / 1e9, 3),
                              lds_budget=occ["lds_budget"], scl_wgs_per_cu=occ["scl_wgs_per_cu"],
                              bp_wgs_per_cu=occ["wgs_per_cu"])))
        return

    # ---- timed region: K learned-hybrid steps through the two-stream pipeline,
    # with the list decoder's LDS budget and the caps on BP and list-decoder
    # workgroups per CU that run it fastest (tuned beforehand, untimed)
    from paper_1609_09358_amd import autotune
    occ = autotune.tune_pipeline(learned_pipe, llr)
    elapsed = run_pipe(learned_pipe, out, args.steps, args.warmup)
    ms_step = 1e3 * elapsed / args.steps
    gbps = B * K * args.steps / elapsed / 1e9
    # the same steps on one stream, and the plain hybrid on the same frames
    gbps_single = B * K * args.steps / run_steps(learned, out, args.steps, args.warmup) / 1e9
    occ_p = autotune.tune_pipeline(plain_pipe, llr)
    gbps_plain = B * K * args.steps / run_pipe(plain_pipe, out_p, args.steps, args.warmup) / 1e9
    PB.polar_set_pipeline_bp_occupancy(0)
    PB.polar_set_pipeline_scl_occupancy(0)
    gbps_plain_single = B * K * args.steps / run_steps(plain, out_p, args.steps, args.warmup) / 1e9
    # the learned decoder's list-decoder settings for what follows (kernel timing)
    PB.polar_set_scl_lds_budget(occ["lds_budget"])

    # ---- statistics of one step of each
    def one(dec, o):
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        dec(llr, out=o, stats=st)
        torch.cuda.synchronize()
        return st.cpu().numpy()

    st = one(learned, out)
    st_p = one(plain, out_p)
    fer_batch = float(np.mean(np.any(out["info"].cpu().numpy() != info, axis=1)))

    # ---- FER of both on common frames (fresh, seeded, generated on the device)
    fer_gen = TW.Trainer(code, 1, 16, seed=4242)
    nf, err_l, err_p, only_l, only_p = 0, 0, 0, 0, 0
    while nf < args.fer_frames:
        b = min(B, args.fer_frames - nf)
        inf_f, _, llr_f = fer_gen.frames(b, ebn0=args.ebn0)
        el = (learned(llr_f)["info"] != inf_f).any(dim=1)
        ep = (plain(llr_f)["info"] != inf_f).any(dim=1)
        err_l += int(el.sum())
        err_p += int(ep.sum())
        only_l += int((el & ~ep).sum())
        only_p += int((ep & ~el).sum())
        nf += b
    fer_l, fer_p = err_l / nf, err_p / nf
    valid = fer_l <= cp_upper(err_p, nf)

    # ---- per-kernel durations with events on the launch stream
    kt = kernel_times(code, llr, W, T, L, max(3, args.steps // 2))
    bp_ms, scl_ms, nfail, iter_sum, bp_out = kt["bp_ms"], kt["scl_ms"], kt["scl_frames"], kt["iter_sum"], kt["bp_out"]

    # algorithmic work of the weighted BP kernel, per PE and sweep: the input
    # sum of the first output (1), the shared operand's sign moved onto the
    # weight (1), the two min-sum terms as clamps of one input to the other's
    # magnitude (2), the weight product of the first output (1), the weight
    # product plus addition of the second (1, fused), the clip of the second
    # (1) and that of the first (1) unless every weight is within [-1, 1],
    # where it cannot act = 7 or 8 single-lane operations; n*N/2 PEs and 2
    # sweeps per iteration
    w_unit = float(W.abs().max()) <= 1.0
    bp_ops = (7.0 if w_unit else 8.0) * n * N * iter_sum
    # algorithmic work of the SCL kernel: L * n * N / 2 f/g evaluations per frame
    scl_ops = float(L * n * N // 2) * nfail
    dominant = "bp_kernel" if bp_ms >= scl_ms else "scl_kernel"
    ach = bp_ops / (bp_ms * 1e-3) / 1e12 if dominant == "bp_kernel" else scl_ops / (scl_ms * 1e-3) / 1e12
    roofline = {
        "kernel": dominant,
        "bound": "alu",
        "achieved": round(ach, 4),
        "peak": round(VALU_PEAK_GOPS / 1e3, 2),
        "unit": "Tops/s",
        "frac": round(ach / (VALU_PEAK_GOPS / 1e3), 4),
        "traffic": bp_traffic(B) if dominant == "bp_kernel" else None,
    }
    gamma = float(st[2]) / B
    extra = {
        "valid_fer_le_plain": bool(valid),
        "fer_learned": fer_l,
        "fer_plain": fer_p,
        "fer_frames": nf,
        "fer_plain_cp95_upper": cp_upper(err_p, nf),
        "mcnemar_only_learned_wrong": only_l,
        "mcnemar_only_plain_wrong": only_p,
        "fer_timed_batch": fer_batch,
        "learned_single_stream_Gbps": round(gbps_single, 4),
        "pipeline_tuning": {"learned": occ, "plain": occ_p},
        "plain_hybrid_Gbps": round(gbps_plain, 4),
        "plain_single_stream_Gbps": round(gbps_plain_single, 4),
        "speedup_vs_plain": round(gbps / gbps_plain, 3),
        "bp_fail_rate": gamma,
        "bp_fail_rate_plain": float(st_p[2]) / B,
        "mean_bp_iterations": float(st[3]) / B,
        "mean_bp_iterations_plain": float(st_p[3]) / B,
        "kernel_ms": {"bp_kernel": round(bp_ms, 4), "scl_kernel": round(scl_ms, 4)},
        "bp_ops_per_pe_sweep": 7 if w_unit else 8,
        "weights_max_abs": round(float(W.abs().max()), 4),
        "scl_frames": nfail,
        "weights": weights_info,
        "eq1_theory_Gbps": None,
    }
    # eq. (1) of the paper with the measured parts
    if nfail:
        t_bp = B * K / (bp_ms * 1e-3) / 1e9
        t_scl = nfail * K / (scl_ms * 1e-3) / 1e9
        extra["eq1_theory_Gbps"] = round(t_bp * t_scl / (t_scl + gamma * t_bp), 3)

    if args.copy_calibration:
        src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = src.numel() * 4

    if not args.skip_extras:
        extra["scl_only"] = scl_only(code_plain, code, llr, L, gbps, gbps_plain)
        extra["c1_plain_bp"] = c1_plain_bp()
        extra["c3_mixed"] = c3_mixed(args.steps)
        extra["c4_learned_bp"] = c4_learned_bp(frames=args.train_frames)
        extra["scl_ranking_ab"] = scl_ranking_ab(code, llr, bp_out, W, T)
        extra["latency"] = latency_study(code, learned, T, W)
        extra["c5_other_points"] = c5_points(code, learned_pipe, plain_pipe, learned, plain, B)
        extra["c2_rules"] = c2_rules(args.frames, max(3, args.steps // 4))
        extra["c2_sweep"] = c2_sweep(args.frames, max(3, args.steps // 4))
        extra["paper_operating_point"] = paper_operating_point()

    cpu = None
    if not args.no_cpu:
        W_nodes = W[..., None].expand(T, 2, n, N).cpu().numpy().astype(np.float64)
        cpu = cpu_baseline(info, z, sigma2, code.frozen, N, K, C, L, T, W_nodes, args.cpu_seconds,
                           da=code.decision_aided)

    line = {
        "metric": "decoded info Gbit/s, N=1024 R=1/2 hybrid at FER≤plain, Eb/N0 2.5 dB",
        "value": round(gbps, 4),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"learned hybrid: weighted min-sum BP T={T} (CRC-24 stop) -> CA-SCL "
                        f"L={L} with {DA} decision-aided positions; N=1024 K=512 CRC-24, GA design 2.5 dB, "
                        f"BPSK/AWGN Eb/N0 {args.ebn0} dB; compared with plain hybrid BP i_max={IMAX} -> CA-SCL "
                        f"L={L} without decision aiding on the same frames",
            "frames_per_step": B,
            "ebn0_db": args.ebn0,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


def kernel_times(code, llr, W, T, L, reps):
    """Average durations (HIP events on the stream the kernels are launched
    on) of the learned BP kernel alone on the batch and of the list decoder
    alone on the frames that BP fails, each over `reps` launches after
    untimed ones for 60 ms (the clock's steady state); with the iteration sum
    of one BP launch (every launch decodes the same frames)."""
    import torch

    from paper_1609_09358_amd import binding as PB

    B, N = llr.shape
    stream = torch.cuda.current_stream()

    def timed(fn, warm_ms=60.0):
        # the clock needs a few tens of milliseconds of load to reach its
        # steady state after the host-side work before: untimed launches
        # until warm_ms have passed
        t_w = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        while (time.perf_counter() - t_w) * 1e3 < warm_ms:
            fn()
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps  # ms

    bp_out = dict(u_hat=torch.empty((B, N), dtype=torch.uint8, device="cuda"),
                  iters=torch.empty(B, dtype=torch.int32, device="cuda"),
                  ok=torch.empty(B, dtype=torch.uint8, device="cuda"))
    bp_ms = timed(lambda: PB.bp_decode_batch(code, llr, max_iter=T, stop=STOP, weights=W, out=bp_out))
    fail_ids = torch.nonzero(bp_out["ok"] == 0).flatten().to(torch.int32).contiguous()
    nfail = int(fail_ids.numel())
    scl_out = dict(u_hat=torch.empty((B, N), dtype=torch.uint8, device="cuda"),
                   crc_ok=torch.empty(B, dtype=torch.uint8, device="cuda"),
                   pm=torch.empty(B, dtype=torch.float32, device="cuda"))
    ws_bytes = PB.polar_workspace_size(code, max(nfail, 1), L)
    scl_ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    scl_ms = timed(lambda: PB.scl_decode_batch(code, llr, L, frame_ids=fail_ids, out=scl_out,
                                               workspace=scl_ws)) if nfail else 0.0
    return {"bp_ms": bp_ms, "scl_ms": scl_ms, "scl_frames": nfail, "iter_sum": int(bp_out["iters"].sum().item()),
            "timed_launches": reps, "bp_out": bp_out}


def scl_ranking_ab(code, llr, bp_out, W, T, reps=3):
    """List decoding with the pruned pseudo sort, a bitonic sort of the
    candidates (Sec. II-A describes both) and threshold selection, on the
    frames the learned BP failed in one batch (latency-bound) and on 8192
    frames (throughput-bound)."""
    import torch

    from paper_1609_09358_amd import binding as PB

    fail = torch.nonzero(bp_out["ok"] == 0).flatten().to(torch.int32).contiguous()
    many = torch.arange(8192, dtype=torch.int32, device="cuda")
    res = {}
    for L in (8, 32):
        for name, ids in (("failed_frames", fail), ("8192_frames", many)):
            row = {}
            for mode in (1, 2, 3):
                PB.polar_set_scl_ranking(mode)
                out = PB.scl_decode_batch(code, llr, L, frame_ids=ids)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    PB.scl_decode_batch(code, llr, L, frame_ids=ids, out=out)
                torch.cuda.synchronize()
                row[{1: "pseudo_sort_ms", 2: "bitonic_ms", 3: "threshold_ms"}[mode]] = \
                    round((time.perf_counter() - t0) / reps * 1e3, 3)
            res[f"L{L}_{name}"] = dict(frames=int(ids.numel()), **row)
    PB.polar_set_scl_ranking(0)
    return res


def c5_points(code, learned_pipe, plain_pipe, learned, plain, B, ebn0s=(2.0, 3.0), steps=10, fer_frames=1 << 20):
    """The learned hybrid at the other Eb/N0 points of its configuration (the
    weights fitted at 2.5 dB): pipelined throughput of both decoders on one
    resident batch, and their FER on common fresh frames with the
    Clopper-Pearson bound of the plain decoder's."""
    import torch

    from paper_1609_09358_amd import train_wbp as TW

    rows = []
    for e in ebn0s:
        gen = TW.Trainer(code, 1, 16, seed=int(100 * e) + 17)
        _, _, llr = gen.frames(B, ebn0=e)
        res = {"ebn0_db": e}
        for name, pipe in (("learned", learned_pipe), ("plain", plain_pipe)):
            pipe([llr] * 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pipe([llr] * steps)
            torch.cuda.synchronize()
            res[f"{name}_Gbps"] = round(B * code.K * steps / (time.perf_counter() - t0) / 1e9, 4)
        nf = el = ep = 0
        while nf < fer_frames:
            b = min(B, fer_frames - nf)
            inf_f, _, llr_f = gen.frames(b, ebn0=e)
            el += int((learned(llr_f)["info"] != inf_f).any(dim=1).sum())
            ep += int((plain(llr_f)["info"] != inf_f).any(dim=1).sum())
            nf += b
        res.update(fer_frames=nf, fer_learned=el / nf, fer_plain=ep / nf, fer_plain_cp95_upper=cp_upper(ep, nf),
                   valid_fer_le_plain=bool(el / nf <= cp_upper(ep, nf)))
        rows.append(res)
    return rows


def latency_study(code, learned, T, W, reps=20):
    """Decode-call latency of the learned hybrid (the latency of every frame
    in the call) for small batches over Eb/N0, median and worst over `reps`
    calls, in the spirit of the paper's latency figure; each with the call's
    kernels replayed as one captured graph (the default) and launched one by
    one."""
    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import train_wbp as TW

    gen = TW.Trainer(code, 1, 16, seed=5555)
    rows = []
    for e in (1.5, 2.5, 3.5):
        for B in (1, 64, 4096):
            _, _, llr = gen.frames(B, ebn0=e)
            row = {"ebn0_db": e, "frames": B}
            for mode, tag in ((1, "graph"), (0, "direct")):
                PB.polar_set_hybrid_graphs(mode)
                out = learned(llr)
                learned(llr, out=out)
                torch.cuda.synchronize()
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    learned(llr, out=out)
                    torch.cuda.synchronize()
                    ts.append((time.perf_counter() - t0) * 1e3)
                ts.sort()
                row[f"{tag}_median_ms"] = round(ts[len(ts) // 2], 4)
                row[f"{tag}_worst_ms"] = round(ts[-1], 4)
            PB.polar_set_hybrid_graphs(1)
            rows.append(row)
    return rows


def c1_plain_bp(reps=20):
    """Plain min-sum BP of its configuration: N=128, K=64, no CRC, GA at 2 dB,
    1000 frames at 2 dB, at most 100 iterations with the re-encoding stop.
    Throughput of one call on the 1000 resident frames (launch-bound) and on
    65536 frames of the same kind, mean iterations and FER (95%
    Clopper-Pearson interval)."""
    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import train_wbp as TW

    code = PB.PolarCode(128, 64, 0, 0, 2.0)
    gen = TW.Trainer(code, 1, 16, seed=128)
    res = {}
    for B in (1000, 65536):
        info, _, llr = gen.frames(B, ebn0=2.0)
        out = PB.bp_decode_batch(code, llr, max_iter=100, stop=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            PB.bp_decode_batch(code, llr, max_iter=100, stop=1, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        err = int((TW.info_of(code, out["u_hat"]) != info).any(dim=1).sum())
        res[f"frames_{B}"] = {"Gbps": round(B * 64 / dt / 1e9, 4), "ms": round(dt * 1e3, 4),
                              "mean_iterations": float(out["iters"].float().mean()), "fer": err / B,
                              "fer_cp95": [cp_lower(err, B), cp_upper(err, B)]}
    return res


def scl_only(code_plain, code_da, llr, L, learned_gbps, plain_gbps, reps=3):
    """List decoding of every frame (no BP), the decoder the paper's hybrid is
    compared with in Sec. IV: CA-SCL L on the same resident batch without and
    with decision aiding, and the hybrids' speed-up over it."""
    import torch

    from paper_1609_09358_amd import binding as PB

    B = llr.shape[0]
    res = {"frames": B}
    for name, c in (("plain", code_plain), ("decision_aided", code_da)):
        ws = torch.empty(max(PB.polar_workspace_size(c, B, L), 1), dtype=torch.uint8, device="cuda")
        out = PB.scl_decode_batch(c, llr, L, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            PB.scl_decode_batch(c, llr, L, out=out, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[f"scl_{name}_Gbps"] = round(B * c.K / dt / 1e9, 4)
    res["learned_hybrid_speedup"] = round(learned_gbps / res["scl_plain_Gbps"], 1)
    res["plain_hybrid_speedup"] = round(plain_gbps / res["scl_plain_Gbps"], 1)
    return res


def c4_learned_bp(frames=1_000_000, batch=4096, eval_frames=100_000):
    """Weighted BP N=256, K=128, CRC-8, T=10 trained with Adam (lr 1e-3) on the
    final-iteration BCE over Eb/N0 uniform in [1, 4] dB, from w = 1; frame
    error rates of the learned BP (10 iterations) and the plain BP (100
    iterations, the configured comparator, and 10) on the same fresh frames,
    all with the re-encoding stop, each with its 95% Clopper-Pearson interval."""
    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import train_wbp as TW

    t0 = time.perf_counter()
    tr, hist = TW.train(256, 128, 8, 10, frames=frames, batch=batch, lr=1e-3, ebn0=(1.0, 4.0), design=2.5, seed=1,
                        log_every=1 << 30, verbose=False)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    code = tr.code
    gen = TW.Trainer(code, 1, 16, seed=256)
    rows = []
    for e in (1.0, 2.0, 3.0, 4.0):
        info, _, llr = gen.frames(eval_frames, ebn0=e)
        row = {"ebn0_db": e}
        for name, w, it in (("learned_T10", tr.W, 10), ("plain_100_iterations", None, 100),
                            ("plain_10_iterations", None, 10)):
            o = PB.bp_decode_batch(code, llr, max_iter=it, stop=1, weights=w)
            err = int((TW.info_of(code, o["u_hat"]) != info).any(dim=1).sum())
            row[f"fer_{name}"] = err / eval_frames
            row[f"fer_{name}_cp95"] = [cp_lower(err, eval_frames), cp_upper(err, eval_frames)]
        rows.append(row)
    return {"train_frames": frames, "train_seconds": round(train_s, 2), "loss_first": hist[0][1],
            "loss_last": hist[-1][1], "eval_frames": eval_frames, "fer": rows}


def c2_rules(B, steps, ebn0=2.5):
    """Plain hybrid N=1024 K=512 CRC-16, i_max=200, L=8 at 2.5 dB with the
    min-sum rule and with the paper's exact rule, on the same frames."""
    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import train_wbp as TW

    code = PB.PolarCode(1024, 512, 16, 0, 2.5)
    info, _, llr = TW.Trainer(code, 1, 16, seed=1016).frames(B, ebn0=ebn0)
    res = {}
    for rule in (0, 1):
        dec = PB.HybridDecoder(code, max_iter=200, L=8, rule=rule)
        out = dec(llr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dec(llr, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        out = dec(llr, stats=st)
        torch.cuda.synchronize()
        s = st.cpu().numpy()
        res["exact" if rule else "min_sum"] = {
            "Gbps": round(B * 512 / dt / 1e9, 4), "ms": round(dt * 1e3, 3), "bp_fail_rate": float(s[2]) / B,
            "mean_bp_iterations": float(s[3]) / B,
            "fer": float((out["info"] != info).any(dim=1).float().mean()),
        }
    return res


def c2_sweep(B, steps, ebn0s=(1.5, 2.0, 2.5, 3.0), fer_frames=100_000):
    """The plain hybrid of its configuration (N=1024 K=512 CRC-16, GA at
    2.5 dB, min-sum BP i_max=200, CA-SCL L=8) over Eb/N0: single-stream and
    pipelined throughput on one resident batch, BP failure rate, mean
    iterations, and FER on 1e5 fresh frames per point."""
    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import train_wbp as TW

    code = PB.PolarCode(1024, 512, 16, 0, 2.5)
    dec = PB.HybridDecoder(code, max_iter=200, L=8)
    pipe = PB.HybridPipeline(code, max_iter=200, L=8)
    rows = []
    for e in ebn0s:
        gen = TW.Trainer(code, 1, 16, seed=int(100 * e) + 2)
        _, _, llr = gen.frames(B, ebn0=e)
        out = dec(llr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dec(llr, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        outs = [{"info": torch.empty((B, code.K), dtype=torch.uint8, device="cuda")} for _ in range(2)]
        pipe([llr] * 2, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pipe([llr] * steps, outs=[outs[i % 2] for i in range(steps)])
        torch.cuda.synchronize()
        dtp = (time.perf_counter() - t0) / steps
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        nf = err = 0
        while nf < fer_frames:
            b = min(B, fer_frames - nf)
            inf_f, _, llr_f = gen.frames(b, ebn0=e)
            err += int((dec(llr_f, stats=st)["info"] != inf_f).any(dim=1).sum())
            nf += b
        s = st.cpu().numpy()
        rows.append({"ebn0_db": e, "Gbps": round(B * code.K / dt / 1e9, 4),
                     "pipelined_Gbps": round(B * code.K / dtp / 1e9, 4),
                     "bp_fail_rate": float(s[2]) / float(s[0]), "mean_bp_iterations": float(s[3]) / float(s[0]),
                     "fer": err / nf, "fer_frames": nf})
    return rows


def paper_operating_point(B=16384, reps=3, da_bits=1024):
    """The paper's own hybrid configuration (Sec. III): N=4096, R=1/2, BP with
    the exact rule and i_max=50, CA-SCL L=32 (CRC-16 here) with decision
    aiding on the 1024 most reliable information positions (no frame-error
    change against plain CA-SCL at 1.25 and 1.5 dB on 8192 frames), over an
    Eb/N0 sweep; the paper reports at most 34 Mbit/s for it on its GPU."""
    import torch

    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import train_wbp as TW

    code = PB.PolarCode(4096, 2048, 16, 0, 2.5, da_bits=da_bits)
    dec = PB.HybridDecoder(code, max_iter=50, L=32, rule=1)
    gen = TW.Trainer(code, 1, 16, seed=4096)
    rows = []
    for e in (1.5, 2.0, 2.5, 3.0, 3.5):
        info, _, llr = gen.frames(B, ebn0=e)
        out = dec(llr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dec(llr, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        out = dec(llr, stats=st)
        torch.cuda.synchronize()
        s = st.cpu().numpy()
        rows.append({"ebn0_db": e, "Gbps": round(B * 2048 / dt / 1e9, 4), "bp_fail_rate": float(s[2]) / B,
                     "mean_bp_iterations": round(float(s[3]) / B, 3),
                     "fer": float((out["info"] != info).any(dim=1).float().mean())})
    # list decoding of every frame (the non-hybrid decoder of Sec. IV), on the
    # last point's frames: its time does not depend on the channel
    scl = {}
    for name, c in (("plain", PB.PolarCode(4096, 2048, 16, 0, 2.5)), ("decision_aided", code)):
        ws = torch.empty(max(PB.polar_workspace_size(c, B, 32), 1), dtype=torch.uint8, device="cuda")
        o = PB.scl_decode_batch(c, llr, 32, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        PB.scl_decode_batch(c, llr, 32, out=o, workspace=ws)
        torch.cuda.synchronize()
        scl[f"scl_only_{name}_Gbps"] = round(B * 2048 / (time.perf_counter() - t0) / 1e9, 4)
    for r in rows:
        r["speedup_vs_scl_only"] = round(r["Gbps"] / scl["scl_only_plain_Gbps"], 1)
    best = max(r["Gbps"] for r in rows)
    return {"frames": B, "da_bits": da_bits, "points": rows, "max_Gbps": best, "paper_max_Mbps": 34.0,
            "ratio_to_paper_max": round(best * 1e3 / 34.0, 1), **scl}


def c3_mixed(steps, B=4096, max_iter=200, L=8):
    """Ragged batch of twelve codes (N 256..2048, rates 1/4..3/4, CRC-16),
    Eb/N0 uniform in [1, 3] dB per frame: autotuned plan, eager launches and
    the replayed hipGraph, each timed over `steps` calls."""
    import torch

    from paper_1609_09358_amd import autotune
    from paper_1609_09358_amd import binding as PB
    from paper_1609_09358_amd import mixed_workload as MW

    codes = MW.make_codes()
    batch = MW.ragged_batch(codes, B, seed=3)
    tuned = autotune.tune_mixed(codes, [rows for _, rows in batch["per_code"]], max_iter, L)
    info_hat = torch.empty(batch["total_info_bits"], dtype=torch.uint8, device="cuda")
    used = torch.empty(B, dtype=torch.uint8, device="cuda")
    args = (batch["llr"], batch["code_of_frame"], batch["llr_off"], batch["out_off"], info_hat, used)
    # whole-plan choices: the longest bucket's BP layout, the list decoder's LDS budget
    tb = autotune.tune_mixed_plan(codes, args, max_iter, L, tuned["variants"])
    plan = PB.MixedPlan(codes, max_frames=B, max_iter=max_iter, L=L, variants=tb["variants"])
    res = {}
    for graph in (False, True):
        plan(*args, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan(*args, graph=graph)
        torch.cuda.synchronize()
        res["graph" if graph else "eager"] = (time.perf_counter() - t0) / steps
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    plan(*args, stats=stats, graph=True)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    fe = MW.frame_errors(batch, info_hat, codes)
    PB.polar_set_scl_lds_budget(0)
    bits = batch["total_info_bits"]
    return {
        "frames": B, "codes": len(codes), "info_bits": bits,
        "eager_ms": round(res["eager"] * 1e3, 3), "graph_ms": round(res["graph"] * 1e3, 3),
        "eager_Gbps": round(bits / res["eager"] / 1e9, 4), "graph_Gbps": round(bits / res["graph"] / 1e9, 4),
        "bp_fail_rate": float(st[2]) / B, "fer": fe / B, "variants": tb["variants"], "scl_lds_budget": tb["budget"],
        "plan_tuning_ms": tb["ms"],
    }


def cpu_baseline(info, z, sigma2, frozen, N, K, C, L, T, W64, target_s, da=None):
    """The oracle (double precision, as written) running the same learned
    hybrid on the first frames of the same workload on the host cores, one
    thread per slice."""
    import oracle as O

    # every CPU this process may use, within the environment's thread budget
    # (the CPU share the host grants when it sets OMP_NUM_THREADS)
    cpu = host_cpu()
    threads = cpu["usable"] if cpu["omp_num_threads"] is None else min(cpu["usable"], cpu["omp_num_threads"])
    threads = max(1, threads)
    fr = np.asarray(frozen, np.uint8)

    def llr_of(M):
        u, x = O.encode_batch(info[:M], K, C, POLY24, fr)
        return O.channel_llr(x, z[:M].astype(np.float64), sigma2)

    def dec(llr_part):
        return O.hybrid_batch(llr_part, fr, K, C, POLY24, T, L, W=W64, da=da, stop=STOP)

    # calibrate on a few frames, then size the sample for ~target_s seconds
    M0 = 4 * threads
    llr0 = llr_of(M0)
    chunks0 = np.array_split(np.arange(M0), threads)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda idx: dec(llr0[idx]), chunks0))
    per_frame = (time.perf_counter() - t0) / M0
    M = int(max(threads, min(len(info), target_s / max(per_frame, 1e-6))))
    M = max(threads, (M // threads) * threads)
    llr = llr_of(M)
    chunks = np.array_split(np.arange(M), threads)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        outs = list(ex.map(lambda idx: dec(llr[idx]), chunks))
    dt = time.perf_counter() - t0
    info_hat = np.concatenate([o["info"] for o in outs])
    # one core on a slice of the same frames
    M1 = max(1, min(M, int(M / threads)))
    t0 = time.perf_counter()
    dec(llr[:M1])
    dt1 = time.perf_counter() - t0
    return {
        "value": round(M * K / dt / 1e9, 6),
        "unit": "Gbit/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {M} frames of the same workload (same info bits and noise), double-precision oracle "
                  f"learned hybrid T={T} L={L} with the same weights, {dt:.1f} s; single core: first {M1} "
                  f"frames, {dt1:.1f} s",
        "value_single_core": round(M1 * K / dt1 / 1e9, 6),
        "fer": float(np.mean(np.any(info_hat != info[:M], axis=1))),
        "host": cpu,
    }


if __name__ == "__main__":
    main()
