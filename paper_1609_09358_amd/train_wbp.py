"""Training of the weighted (learned) min-sum BP on the GPU.

Recipe (one step): draw a batch of random information bits and per-frame
Eb/N0 uniform in [lo, hi] dB, encode (polar_encode), BPSK/AWGN LLRs
(polar_channel_awgn), weighted BP forward with message saving (wbp_forward),
binary cross-entropy on the non-frozen bits (wbp_bce, or after every
iteration, wbp_bce_multi) or the frame-failure surrogate (wbp_frame_loss),
reverse-mode gradient (wbp_backward), Adam (polar_adam_step, or projected onto
a box, polar_adam_step_bounded).  Weights shared by a stage column are spread
over its nodes (wbp_column_weights) and their gradient summed back
(wbp_column_grad).  Every step of the decoder, its loss,
gradient and update runs in the library's kernels; torch supplies device
memory, the stream and the random draws of the workload.

The weights start at 1 (plain min-sum BP) unless told otherwise and are saved as float32 numpy
arrays [T][2][n][N] together with the Adam moments and the step count, so a
run can resume bit-exactly.
"""
import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import binding as PB


def sigma2_of(ebn0_db: torch.Tensor, rate: float) -> torch.Tensor:
    return 1.0 / (2.0 * rate * torch.pow(10.0, ebn0_db / 10.0))


class Trainer:
    """Gradient training of the weighted BP with the library's kernels.

    layout "node": one weight per edge output, W [T][2][n][N]; "column": one
    weight per stage column, W [T][2][n] (the learned hybrid's form), spread
    over the nodes by wbp_column_weights for the forward and adjoint, whose
    per-node gradient wbp_column_grad sums back per column.
    loss "bce": cross-entropy after the last iteration; "multi": summed over
    iterations; "frame": the frame-failure surrogate (probability that no
    iteration decides the whole frame right); "iter": the expected iterations
    of an early-stopping decoder plus fail_weight per frame left undecided
    after T.
    bounds (lo, hi): Adam projected onto that box (polar_adam_step_bounded).
    w0: the initial weight (1 = plain min-sum BP)."""

    def __init__(self, code: PB.PolarCode, T: int, batch: int, lr: float = 1e-3, ebn0=(1.0, 4.0), seed: int = 1,
                 llr_max: float = 20.0, multiloss: bool = False, layout: str = "node", loss: str = None,
                 bounds=None, w0: float = 1.0, fail_weight: float = 0.0):
        self.code, self.T, self.B, self.lr, self.ebn0, self.llr_max = code, T, batch, lr, ebn0, llr_max
        self.loss = loss or ("multi" if multiloss else "bce")
        assert self.loss in ("bce", "multi", "frame", "iter") and layout in ("node", "column")
        self.layout, self.bounds, self.fail_weight = layout, bounds, fail_weight
        dev = torch.device("cuda")
        node_shape = (T, 2, code.n, code.N)
        shape = node_shape if layout == "node" else (T, 2, code.n)
        self.W = torch.full(shape, float(w0), dtype=torch.float32, device=dev)
        self.m = torch.zeros(shape, dtype=torch.float32, device=dev)
        self.v = torch.zeros(shape, dtype=torch.float32, device=dev)
        self.step = 0
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        self.out = dict(llr_u=torch.empty((batch, code.N), dtype=torch.float32, device=dev),
                        u_hat=torch.empty((batch, code.N), dtype=torch.uint8, device=dev),
                        saved=torch.empty((batch,) + node_shape, dtype=torch.float32, device=dev))
        self.Wn = torch.empty(node_shape, dtype=torch.float32, device=dev) if layout == "column" else None
        self.dWc = torch.empty(shape, dtype=torch.float32, device=dev) if layout == "column" else None

    def frames(self, B=None, ebn0=None):
        """A fresh batch: (info [B][K], u [B][N], llr [B][N])."""
        B = B or self.B
        code = self.code
        info = torch.randint(0, 2, (B, code.K), generator=self.gen, device="cuda", dtype=torch.uint8)
        u, x = PB.polar_encode(code, info, want_u=True)
        lo, hi = self.ebn0 if ebn0 is None else (ebn0, ebn0)
        e = lo + (hi - lo) * torch.rand(B, generator=self.gen, device="cuda")
        z = torch.randn((B, code.N), generator=self.gen, device="cuda")
        llr = PB.polar_channel_awgn(x, z, sigma2_of(e, code.K / code.N).float().contiguous())
        return info, u, llr

    def node_weights(self) -> torch.Tensor:
        """The weights as the per-node kernels read them, [T][2][n][N]."""
        return self.W if self.layout == "node" else PB.wbp_column_weights(self.code, self.W, out=self.Wn)

    def train_step(self):
        _, u, llr = self.frames()
        Wn = self.node_weights()
        fw = PB.wbp_forward(self.code, llr, Wn, llr_max=self.llr_max, save=True, out=self.out)
        if self.loss == "multi":
            loss, dlam = PB.wbp_bce_multi(self.code, fw["saved"], u, self.T)
        elif self.loss == "frame":
            loss, dlam = PB.wbp_frame_loss(self.code, fw["saved"], u, self.T)
        elif self.loss == "iter":
            loss, dlam = PB.wbp_iteration_loss(self.code, fw["saved"], u, self.T, self.fail_weight)
        else:
            loss, dlam = PB.wbp_bce(self.code, fw["llr_u"], u)
        dW, _ = PB.wbp_backward(self.code, llr, Wn, fw["saved"], dlam, llr_max=self.llr_max)
        g = dW if self.layout == "node" else PB.wbp_column_grad(self.code, dW, out=self.dWc)
        self.step += 1
        if self.bounds is None:
            PB.polar_adam_step(self.W, g, self.m, self.v, self.step, lr=self.lr)
        else:
            PB.polar_adam_step_bounded(self.W, g, self.m, self.v, self.step, lr=self.lr, lo=self.bounds[0],
                                       hi=self.bounds[1])
        return loss

    def save(self, path):
        np.savez(path, W=self.W.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.array(self.step), rng=self.gen.get_state().cpu().numpy())

    def load(self, path):
        z = np.load(path)
        self.W.copy_(torch.from_numpy(z["W"]))
        self.m.copy_(torch.from_numpy(z["m"]))
        self.v.copy_(torch.from_numpy(z["v"]))
        self.step = int(z["step"])
        self.gen.set_state(torch.from_numpy(z["rng"]))


def train(N=256, K=128, crc_bits=8, T=10, frames=1_000_000, batch=4096, lr=1e-3, ebn0=(1.0, 4.0), design=2.5,
          seed=1, log_every=20, verbose=True):
    """Train and return (trainer, history); `frames` / `batch` steps."""
    code = PB.PolarCode(N, K, crc_bits, 0, design)
    tr = Trainer(code, T, batch, lr, ebn0, seed)
    steps = math.ceil(frames / batch)
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        loss = tr.train_step()
        if (s + 1) % log_every == 0 or s == 0 or s + 1 == steps:
            lv = float(loss.sum())
            hist.append((s + 1, lv))
            if verbose:
                print(json.dumps({"step": s + 1, "loss": lv, "s": round(time.perf_counter() - t0, 2)}), flush=True)
    torch.cuda.synchronize()
    return tr, hist


def train_front_end(code: PB.PolarCode, T: int, w0, ebn0: float, schedule=((3e-3, 1500), (1e-3, 1000)),
                    batch: int = 1024, seed: int = 5, loss: str = "frame", fail_weight: float = 0.0):
    """The learned hybrid's BP front end: one weight per stage column, from w0
    (a number for every weight, e.g. the normalized min-sum scale, or a
    [T][2][n] tensor), trained by Adam on the frame-failure loss (or the
    expected-iterations loss with fail_weight) at one Eb/N0, each weight kept
    within [0, 1]; schedule = ((lr, steps), ...).  Returns (trainer, frames
    seen)."""
    tr = Trainer(code, T, batch, lr=schedule[0][0], ebn0=(ebn0, ebn0), seed=seed, layout="column", loss=loss,
                 bounds=(0.0, 1.0), w0=1.0 if torch.is_tensor(w0) else w0, fail_weight=fail_weight)
    if torch.is_tensor(w0):
        tr.W.copy_(w0)
    seen = 0
    for lr, steps in schedule:
        tr.lr = lr
        for _ in range(steps):
            tr.train_step()
        seen += steps * batch
    return tr, seen


def bp_fail_rate(code: PB.PolarCode, llr: torch.Tensor, W: torch.Tensor, T: int, stop: int = 1, out=None) -> float:
    """Fraction of frames whose weighted BP verdict (re-encoding check and CRC)
    is not ok after at most T iterations: the frames a hybrid hands to SCL."""
    o = PB.bp_decode_batch(code, llr, max_iter=T, stop=stop, weights=W, out=out)
    return 1.0 - float(o["ok"].float().mean())


def bp_cost(code: PB.PolarCode, llr: torch.Tensor, W: torch.Tensor, T: int, fail_weight: float) -> float:
    """Mean BP iterations (a failed frame counts its T) plus fail_weight times
    the failure rate: a proxy for the hybrid's time per frame."""
    o = PB.bp_decode_batch(code, llr, max_iter=T, stop=1, weights=W)
    return float(o["iters"].float().mean()) + fail_weight * (1.0 - float(o["ok"].float().mean()))


def fit_scale(code: PB.PolarCode, llr: torch.Tensor, T: int, grid=None, per_stage: bool = False, stop: int = 1):
    """Normalized min-sum: the single weight alpha (every g term scaled by it)
    with the fewest BP failures on the frames `llr`; returns (W, alpha, rate)
    with W of shape [T][2][n][N], or [T][2][n] (one weight per stage column)."""
    grid = grid if grid is not None else [0.86 + 0.01 * i for i in range(15)]
    shape = (T, 2, code.n) if per_stage else (T, 2, code.n, code.N)
    best = None
    for a in grid:
        W = torch.full(shape, float(a), dtype=torch.float32, device=llr.device)
        r = bp_fail_rate(code, llr, W, T, stop=stop)
        if best is None or r < best[2]:
            best = (W, float(a), r)
    return best


def refine_blocks(code: PB.PolarCode, llr: torch.Tensor, W: torch.Tensor, factors=(0.96, 0.98, 1.02, 1.04),
                  sweeps: int = 1, per_column: bool = False, fail_weight=None, wmax=None, stop: int = 1):
    """Coordinate search on the BP failure rate itself (or, with fail_weight,
    on bp_cost): each block of weights -- one iteration and sweep direction,
    or (per_column) one iteration, direction and stage column -- in turn is
    scaled by the factor that lowers the objective on `llr` most, if any does.
    wmax: scaled weights are kept within [-wmax, wmax] (wmax = 1: the decoder
    never amplifies a check-node message, and the per-stage kernel then skips
    the clips that cannot act).  Returns (W, objective)."""
    T = W.shape[0]
    obj = (lambda w: bp_fail_rate(code, llr, w, T, stop=stop)) if fail_weight is None else \
          (lambda w: bp_cost(code, llr, w, T, fail_weight))
    cur = obj(W)
    blocks = [(t, d, s) for t in range(T) for d in range(2) for s in range(code.n)] if per_column else \
             [(t, d) for t in range(T) for d in range(2)]
    for _ in range(sweeps):
        for blk in blocks:
            base = W[blk].clone()
            best_f, best_r = None, cur
            for f in factors:
                W[blk] = base * f if wmax is None else (base * f).clamp(-wmax, wmax)
                r = obj(W)
                if r < best_r:
                    best_f, best_r = f, r
            W[blk] = base if best_f is None else (base * best_f if wmax is None else (base * best_f).clamp(-wmax, wmax))
            cur = best_r
    return W, cur


def info_of(code: PB.PolarCode, u_hat: torch.Tensor) -> torch.Tensor:
    """Information bits of decoded u vectors: the first K non-frozen positions
    (the CRC occupies the last c)."""
    idx = torch.as_tensor(code.info_pos[: code.K], dtype=torch.long, device=u_hat.device)
    return u_hat.index_select(1, idx)


def fer(decode, tr: Trainer, ebn0: float, frames: int, batch: int = 65536):
    """Frame error rate of `decode(llr) -> info_hat [B][K]` at one Eb/N0 on
    fresh frames from the trainer's generator."""
    err = 0
    done = 0
    while done < frames:
        b = min(batch, frames - done)
        info, _, llr = tr.frames(b, ebn0=ebn0)
        err += int((decode(llr) != info).any(dim=1).sum())
        done += b
    return err / frames


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--K", type=int, default=128)
    ap.add_argument("--crc", type=int, default=8)
    ap.add_argument("--T", type=int, default=10)
    ap.add_argument("--frames", type=int, default=1_000_000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    tr, _ = train(a.N, a.K, a.crc, a.T, a.frames, a.batch, a.lr)
    if a.out:
        tr.save(a.out)


if __name__ == "__main__":
    main()
