"""Autotuner for the BP kernel layout.

For a block length N the library offers several register layouts
(`polar_bp_variants`): a variant r keeps 2^r nodes of every stage row per
thread, which fixes the threads per frame (N / 2^r), the frames per workgroup
(64 * 2^r / N when that exceeds 1), the window structure and hence the LDS
transpose buffers.  The tuner times each variant on a sample of the caller's
own frames with the caller's decoding parameters (events on the current
stream) and keeps the fastest; results are cached per process and optionally
in a JSON file.
"""
import json
import time
import os

import torch

from . import binding as PB

_CACHE = {}


def _key(code, max_iter, stop, weighted):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{dev}|N={code.N}|K={code.K}|c={code.crc_bits}|it={max_iter}|stop={stop}|w={int(weighted)}"


def tune_bp(code: PB.PolarCode, llr: torch.Tensor, max_iter: int, stop: int = 1, weights=None, reps: int = 3,
            sample: int = 16384, cache_file: str = "") -> dict:
    """Return {"variant": best, "ms": {variant: ms per call on the sample}}."""
    key = _key(code, max_iter, stop, weights is not None)
    if key in _CACHE:
        return _CACHE[key]
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as fh:
            disk = json.load(fh)
        if key in disk:
            _CACHE[key] = disk[key]
            return disk[key]
    sub = llr[: min(sample, llr.shape[0])].contiguous()
    B = sub.shape[0]
    out = dict(u_hat=torch.empty((B, code.N), dtype=torch.uint8, device=sub.device),
               iters=torch.empty(B, dtype=torch.int32, device=sub.device),
               ok=torch.empty(B, dtype=torch.uint8, device=sub.device))
    stream = torch.cuda.current_stream()
    timings = {}
    for v in PB.polar_bp_variants(code.N):
        PB.bp_decode_batch(code, sub, max_iter=max_iter, stop=stop, weights=weights, variant=v, out=out)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            PB.bp_decode_batch(code, sub, max_iter=max_iter, stop=stop, weights=weights, variant=v, out=out)
        e1.record(stream)
        e1.synchronize()
        timings[v] = e0.elapsed_time(e1) / reps
    best = min(timings, key=timings.get)
    res = {"variant": int(best), "ms": {int(k): round(v, 4) for k, v in timings.items()}}
    _CACHE[key] = res
    if cache_file:
        disk = {}
        if os.path.exists(cache_file):
            with open(cache_file) as fh:
                disk = json.load(fh)
        disk[key] = res
        with open(cache_file, "w") as fh:
            json.dump(disk, fh, indent=1)
    return res


def tune_scl_budget(code: PB.PolarCode, llr: torch.Tensor, L: int, budgets=(0, 8192, 12288, 20480, 40960),
                    reps: int = 2) -> dict:
    """Time the list decoder on the frames `llr` for each LDS budget
    (polar_set_scl_lds_budget; 0 = automatic) and leave the fastest set.
    Returns {"budget": best, "ms": {budget: ms per call}}."""
    stream = torch.cuda.current_stream()
    timings = {}
    for b in budgets:
        PB.polar_set_scl_lds_budget(b)
        out = PB.scl_decode_batch(code, llr, L)
        ws_bytes = PB.polar_workspace_size(code, llr.shape[0], L)
        ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=llr.device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            PB.scl_decode_batch(code, llr, L, out=out, workspace=ws)
        e1.record(stream)
        e1.synchronize()
        timings[b] = e0.elapsed_time(e1) / reps
    best = min(timings, key=timings.get)
    PB.polar_set_scl_lds_budget(best)
    return {"budget": int(best), "ms": {int(k): round(v, 4) for k, v in timings.items()}}


def tune_mixed(codes, llr_per_code, max_iter: int, L: int, scl_frames: int = 2048) -> dict:
    """Per-code BP layout for a mixed plan (each code timed on its own frames,
    `llr_per_code[c]` of shape [B_c][N_c]) and the list decoder's LDS budget
    (timed on the frames of the longest code).  Returns {"variants": [...],
    "budget": ..., "detail": ...}; the budget is left set, so create the plan
    afterwards."""
    variants, detail = [], {}
    for c, (code, llr) in enumerate(zip(codes, llr_per_code)):
        r = tune_bp(code, llr, max_iter=max_iter, stop=1)
        variants.append(r["variant"])
        detail[f"bp_code{c}_N{code.N}_K{code.K}"] = r
    c_big = max(range(len(codes)), key=lambda c: codes[c].N)
    sub = llr_per_code[c_big][:scl_frames].contiguous()
    b = tune_scl_budget(codes[c_big], sub, L)
    detail["scl"] = b
    return {"variants": variants, "budget": b["budget"], "detail": detail}


def tune_mixed_plan(codes, args, max_iter: int, L: int, variants, budgets=(0, 12288, 16384, 24576, 40960),
                    reps: int = 5) -> dict:
    """Whole-plan choices for a mixed plan, each timed on a batch (replayed
    graph; `args` = (llr, code_of_frame, llr_off, out_off, info_hat, used)):
    first the BP layout of the longest block length, whose bucket is the
    critical path (its failing frames run every iteration; a layout with more
    threads per frame shortens that chain even where it lowers throughput),
    then the list decoder's LDS budget (a smaller one fits more frames on a CU
    at once, a larger one keeps more tree levels in LDS).  Returns
    {"variants": [...], "budget": ..., "ms": {...}}; the budget is left set."""
    B = int(args[1].numel())

    def timed(var):
        plan = PB.MixedPlan(codes, max_frames=B, max_iter=max_iter, L=L, variants=var)
        plan(*args, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan(*args, graph=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    variants = list(variants)
    ms = {}
    nmax = max(c.N for c in codes)
    PB.polar_set_scl_lds_budget(0)
    best_v, best_t = None, None
    for v in PB.polar_bp_variants(nmax):
        var = [v if c.N == nmax else variants[i] for i, c in enumerate(codes)]
        t = timed(var)
        ms[f"variant_N{nmax}_{v}"] = round(t, 3)
        if best_t is None or t < best_t:
            best_v, best_t = v, t
    variants = [best_v if c.N == nmax else variants[i] for i, c in enumerate(codes)]
    best_b, best_bt = None, None
    for b in budgets:
        PB.polar_set_scl_lds_budget(b)
        t = timed(variants)
        ms[f"budget_{b}"] = round(t, 3)
        if best_bt is None or t < best_bt:
            best_b, best_bt = b, t
    PB.polar_set_scl_lds_budget(best_b)
    return {"variants": variants, "budget": best_b, "ms": ms}


def _time_pipe(pipe: PB.HybridPipeline, llr: torch.Tensor, steps: int) -> float:
    """ms per batch of the two-stream hybrid over `steps` batches of `llr`."""
    import time
    # two output buffers alternate: consecutive batches of a call must not share one
    out = [dict(info=torch.empty((llr.shape[0], pipe.code.K), dtype=torch.uint8, device=llr.device)) for _ in range(2)]
    alt = lambda k: [out[i % 2] for i in range(k)]
    pipe([llr] * 2, outs=alt(2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipe([llr] * steps, outs=alt(steps))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def tune_pipeline_occupancy(pipe: PB.HybridPipeline, llr: torch.Tensor, choices=(0, 4, 6, 8), steps: int = 6) -> dict:
    """Time the two-stream hybrid over `steps` batches of `llr` for each cap on
    BP workgroups per CU (polar_set_pipeline_bp_occupancy; 0 = none) and leave
    the fastest set.  Returns {"wgs_per_cu": best, "ms": {cap: ms per batch}}."""
    timings = {}
    for c in choices:
        PB.polar_set_pipeline_bp_occupancy(c)
        timings[c] = _time_pipe(pipe, llr, steps)
    best = min(timings, key=timings.get)
    PB.polar_set_pipeline_bp_occupancy(best)
    return {"wgs_per_cu": int(best), "ms": {int(k): round(v, 4) for k, v in timings.items()}}


def tune_pipeline(pipe: PB.HybridPipeline, llr: torch.Tensor, budgets=(0, 12288, 14336, 16384, 20480),
                  caps=(0, 4, 6, 8), scl_caps=(0, 4, 6), steps: int = 6) -> dict:
    """The two-stream hybrid's launch settings: first the list decoder's LDS
    budget per workgroup (polar_set_scl_lds_budget; 0 = the automatic share,
    a CU's LDS over the workgroups its registers allow) together with the cap
    on list-decoder workgroups per CU (polar_set_pipeline_scl_occupancy; 0 =
    all that fit), with no BP cap, then the cap on BP workgroups per CU with
    the best pair; each setting timed over `steps` batches of `llr` (the
    pairs as the best of three such runs: they differ by about 1 %) and the
    best left set.  The list decoder's LDS competes with the BP workgroups
    beside it: a larger budget keeps more of its state (the trace, then tree
    levels) out of the global slice, a smaller one or a cap on its grid leaves
    room for more BP workgroups.  Results are the same for every setting.
    Returns {"lds_budget": b, "scl_wgs_per_cu": s, "wgs_per_cu": c,
    "ms_budget_scl_cap": {"b/s": ms}, "ms_cap": {c: ms}}."""
    PB.polar_set_pipeline_bp_occupancy(0)
    tb = {}
    for b in budgets:
        PB.polar_set_scl_lds_budget(b)
        for c in scl_caps:
            PB.polar_set_pipeline_scl_occupancy(c)
            tb[(b, c)] = min(_time_pipe(pipe, llr, steps) for _ in range(3))
    best_b, best_s = min(tb, key=tb.get)
    PB.polar_set_scl_lds_budget(best_b)
    PB.polar_set_pipeline_scl_occupancy(best_s)
    occ = tune_pipeline_occupancy(pipe, llr, caps, steps)
    return {"lds_budget": int(best_b), "scl_wgs_per_cu": int(best_s), "wgs_per_cu": occ["wgs_per_cu"],
            "ms_budget_scl_cap": {f"{b}/{c}": round(v, 4) for (b, c), v in tb.items()}, "ms_cap": occ["ms"]}
