"""Synthetic ragged batch mixing several codes, generated on the device.

Twelve codes by default: N in {256, 512, 1024, 2048} times rates {1/4, 1/2,
3/4} (K = N R), CRC-16, frozen sets by Gaussian approximation at 2 dB.  Each
frame draws its code uniformly and its Eb/N0 uniformly in [lo, hi] dB; frames
are in random order.  Encoding and the channel run in the library's kernels;
torch supplies the seeded random draws and the gathers into the ragged layout.
"""
import numpy as np
import torch

from . import binding as PB


def make_codes(Ns=(256, 512, 1024, 2048), rates=(0.25, 0.5, 0.75), crc_bits=16, design_db=2.0):
    return [PB.PolarCode(N, int(N * r), crc_bits, 0, design_db) for N in Ns for r in rates]


def ragged_batch(codes, B, seed, lo=1.0, hi=3.0):
    """Returns dict(code_of_frame, llr_off, out_off, llr, info, per_code) with
    device tensors; per_code[c] = (frame ids, llr rows [B_c][N_c])."""
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    nc = len(codes)
    cf = torch.randint(0, nc, (B,), generator=g, device=dev, dtype=torch.int32)
    ebn0 = lo + (hi - lo) * torch.rand(B, generator=g, device=dev)
    Ns = torch.tensor([c.N for c in codes], device=dev, dtype=torch.int64)[cf.long()]
    Ks = torch.tensor([c.K for c in codes], device=dev, dtype=torch.int64)[cf.long()]
    llr_off = torch.cumsum(Ns, 0) - Ns
    out_off = torch.cumsum(Ks, 0) - Ks
    tot, totk = int(Ns.sum()), int(Ks.sum())
    llr = torch.empty(tot, dtype=torch.float32, device=dev)
    info = torch.empty(totk, dtype=torch.uint8, device=dev)
    per_code = []
    for c, code in enumerate(codes):
        ids = torch.nonzero(cf == c).flatten()
        nb = int(ids.numel())
        if nb == 0:
            per_code.append((ids, torch.empty((0, code.N), dtype=torch.float32, device=dev)))
            continue
        bits = torch.randint(0, 2, (nb, code.K), generator=g, device=dev, dtype=torch.uint8)
        x = PB.polar_encode(code, bits)
        z = torch.randn((nb, code.N), generator=g, device=dev)
        rate = code.K / code.N
        s2 = (1.0 / (2.0 * rate * torch.pow(10.0, ebn0[ids] / 10.0))).float().contiguous()
        rows = PB.polar_channel_awgn(x, z, s2)
        col = torch.arange(code.N, device=dev)
        llr[(llr_off[ids].unsqueeze(1) + col).flatten()] = rows.flatten()
        colk = torch.arange(code.K, device=dev)
        info[(out_off[ids].unsqueeze(1) + colk).flatten()] = bits.flatten()
        per_code.append((ids, rows))
    return dict(code_of_frame=cf, llr_off=llr_off.contiguous(), out_off=out_off.contiguous(), llr=llr, info=info,
                per_code=per_code, total_info_bits=totk)


def frame_errors(batch, info_hat, codes):
    """Number of frames with any information bit wrong."""
    cf = batch["code_of_frame"].cpu().numpy()
    oo = batch["out_off"].cpu().numpy()
    a = batch["info"].cpu().numpy()
    b = info_hat.cpu().numpy()
    Ks = np.array([c.K for c in codes])[cf]
    return int(sum(np.any(a[o:o + k] != b[o:o + k]) for o, k in zip(oo, Ks)))
