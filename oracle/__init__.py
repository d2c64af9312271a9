"""Python front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.

All arrays are numpy; bits are uint8 0/1, LLRs float32 (the GPU's input type),
outputs float64.  ``prec="f64"`` selects the double build (reference values),
``prec="f32"`` the float build (the paper's 32-bit precision, used for
bit-exact comparison of decisions).
"""
import ctypes as C

import numpy as np

from . import build as _build

_LIBS = {}

_u8p = C.POINTER(C.c_uint8)
_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)


def _lib(prec: str = "f64"):
    if prec not in _LIBS:
        _build.ensure_built()
        lib = C.CDLL(_build.LIBS[prec])
        lib.orc_sigma2.restype = C.c_double
        lib.orc_sigma2.argtypes = [C.c_double, C.c_double]
        lib.orc_ga_means.argtypes = [C.c_int, C.c_double, _f64p]
        lib.orc_ga_frozen.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _u8p, _f64p]
        lib.orc_crc.argtypes = [_u8p, C.c_int, C.c_int, C.c_uint32, _u8p]
        lib.orc_polar_transform.argtypes = [_u8p, C.c_int, _u8p]
        lib.orc_build_u.argtypes = [_u8p, C.c_int, C.c_int, C.c_uint32, _u8p, C.c_int, _u8p]
        lib.orc_encode_batch.argtypes = [_u8p, C.c_int64, C.c_int, C.c_int, C.c_uint32, _u8p,
                                         C.c_int, _u8p, _u8p]
        lib.orc_channel_llr.argtypes = [_u8p, _f64p, C.c_int64, C.c_double, _f32p]
        lib.orc_bp_frame.restype = C.c_int
        lib.orc_bp_frame.argtypes = [_f32p, C.c_int, _u8p, C.c_int, C.c_uint32, C.c_int, C.c_int,
                                     C.c_double, C.c_int, _f64p, _u8p, _f64p, _f64p, _u8p, _f64p]
        lib.orc_bp_batch.argtypes = [_f32p, C.c_int64, C.c_int, _u8p, C.c_int, C.c_uint32,
                                     C.c_int, C.c_int, C.c_double, C.c_int, _f64p, _u8p, _f64p,
                                     _i32p, _u8p]
        lib.orc_sc_frame.argtypes = [_f32p, C.c_int, _u8p, C.c_int, _u8p]
        lib.orc_scl_frame.restype = C.c_int
        lib.orc_scl_frame.argtypes = [_f32p, C.c_int, _u8p, _u8p, C.c_int, C.c_uint32, C.c_int,
                                      C.c_int, _u8p, _u8p, _f64p, _u8p, _f64p]
        lib.orc_scl_batch.argtypes = [_f32p, C.c_int64, C.c_int, _u8p, _u8p, C.c_int, C.c_uint32,
                                      C.c_int, C.c_int, _u8p, _u8p, _f64p]
        lib.orc_hybrid_batch.argtypes = [_f32p, C.c_int64, C.c_int, _u8p, _u8p, C.c_int, C.c_int,
                                         C.c_uint32, C.c_int, C.c_int, C.c_double, C.c_int, _f64p, C.c_int,
                                         _u8p, _u8p, _i32p]
        lib.orc_wbp_grad_frame.restype = C.c_double
        lib.orc_wbp_grad_batch.restype = C.c_double
        lib.orc_wbp_grad_batch.argtypes = [_f32p, C.c_int64, C.c_int, _u8p, _u8p, C.c_int,
                                           C.c_double, _f64p, C.c_double, C.c_int, C.c_double, _f64p, _f64p]
        lib.orc_wbp_backward_batch.argtypes = [_f32p, C.c_int64, C.c_int, _u8p, C.c_int, C.c_double, _f64p,
                                               _f64p, C.c_int, _f64p, _f64p]
        lib.orc_adam_step.argtypes = [_f64p, _f64p, _f64p, _f64p, C.c_int64, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_double]
        _LIBS[prec] = lib
    return _LIBS[prec]


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# code construction, CRC, encoder, channel
# --------------------------------------------------------------------------

def sigma2(ebn0_db: float, rate: float) -> float:
    """Noise variance of BPSK/AWGN at Eb/N0 for code rate `rate`."""
    return _lib().orc_sigma2(ebn0_db, rate)


def ga_means(N: int, sig2: float) -> np.ndarray:
    m = np.zeros(N, np.float64)
    _lib().orc_ga_means(N, sig2, _p(m, _f64p))
    return m


def ga_frozen(N: int, k: int, design_ebn0_db: float, rate: float) -> np.ndarray:
    """Frozen mask (1 = frozen) with the k most reliable positions left free."""
    fr = np.zeros(N, np.uint8)
    _lib().orc_ga_frozen(N, k, design_ebn0_db, rate, _p(fr, _u8p), None)
    return fr


def crc(bits, c: int, poly: int) -> np.ndarray:
    b = _u8(bits)
    out = np.zeros(c, np.uint8)
    _lib().orc_crc(_p(b, _u8p), len(b), c, poly, _p(out, _u8p))
    return out


def decision_aided_mask(N: int, frozen, n_da: int, design_ebn0_db: float, rate: float) -> np.ndarray:
    """The n_da most reliable non-frozen positions by Gaussian-approximation
    mean at the design point (equal means: the higher index counts as more
    reliable), as a 0/1 mask: the positions a decision-aided list decoder does
    not branch on (Sec. II-A)."""
    fr = _u8(frozen)
    m = ga_means(N, sigma2(design_ebn0_db, rate))
    cand = [i for i in range(N) if not fr[i]]
    cand.sort(key=lambda i: (m[i], i), reverse=True)
    mask = np.zeros(N, np.uint8)
    for i in cand[:n_da]:
        mask[i] = 1
    return mask


def polar_transform(u) -> np.ndarray:
    u = _u8(u)
    x = np.zeros_like(u)
    _lib().orc_polar_transform(_p(u, _u8p), len(u), _p(x, _u8p))
    return x


def build_u(info, K: int, c: int, poly: int, frozen) -> np.ndarray:
    info = _u8(info)
    fr = _u8(frozen)
    u = np.zeros(len(fr), np.uint8)
    _lib().orc_build_u(_p(info, _u8p), K, c, poly, _p(fr, _u8p), len(fr), _p(u, _u8p))
    return u


def encode_batch(info, K: int, c: int, poly: int, frozen):
    """info [B][K] -> (u [B][N], x [B][N])."""
    info = _u8(info).reshape(-1, K)
    fr = _u8(frozen)
    B, N = info.shape[0], len(fr)
    u = np.zeros((B, N), np.uint8)
    x = np.zeros((B, N), np.uint8)
    _lib().orc_encode_batch(_p(info, _u8p), B, K, c, poly, _p(fr, _u8p), N, _p(u, _u8p),
                            _p(x, _u8p))
    return u, x


def channel_llr(x, z, sig2) -> np.ndarray:
    """BPSK/AWGN LLRs (float32) of codewords x with unit-variance noise z.

    `sig2` is a scalar or one variance per frame (x, z of shape [B][N])."""
    x = _u8(x)
    z = _f64(z)
    out = np.zeros(x.shape, np.float32)
    lib = _lib()
    if np.ndim(sig2) == 0:
        lib.orc_channel_llr(_p(x, _u8p), _p(z, _f64p), x.size, float(sig2), _p(out, _f32p))
    else:
        s = np.asarray(sig2, np.float64).reshape(-1)
        N = x.shape[-1]
        for f in range(x.shape[0]):
            xo, zo, oo = x[f], z[f], out[f]
            lib.orc_channel_llr(_p(xo, _u8p), _p(zo, _f64p), N, float(s[f]), _p(oo, _f32p))
    return out


# --------------------------------------------------------------------------
# decoders
# --------------------------------------------------------------------------

def bp_frame(llr, frozen, c=0, poly=0, max_iter=100, stop=1, llr_max=20.0, rule=0, W=None,
             save=False, prec="f64"):
    """One frame of (weighted) BP.  Returns dict(u_hat, llr_u, llr_x, iters, ok[, save])."""
    llr = _f32(llr)
    fr = _u8(frozen)
    N = len(fr)
    n = N.bit_length() - 1
    uh = np.zeros(N, np.uint8)
    lu = np.zeros(N, np.float64)
    lx = np.zeros(N, np.float64)
    ok = np.zeros(1, np.uint8)
    sv = np.zeros((max_iter, 2, n, N), np.float64) if save else None
    if W is not None:
        W = _f64(W)
        assert W.size >= max_iter * 2 * n * N
    it = _lib(prec).orc_bp_frame(_p(llr, _f32p), N, _p(fr, _u8p), c, poly, max_iter, stop,
                                 llr_max, rule, _p(W, _f64p), _p(uh, _u8p), _p(lu, _f64p),
                                 _p(lx, _f64p), _p(ok, _u8p), _p(sv, _f64p))
    out = dict(u_hat=uh, llr_u=lu, llr_x=lx, iters=it, ok=int(ok[0]))
    if save:
        out["save"] = sv[:it]
    return out


def bp_batch(llr, frozen, c=0, poly=0, max_iter=100, stop=1, llr_max=20.0, rule=0, W=None,
             prec="f64", soft=False):
    fr = _u8(frozen)
    N = len(fr)
    n = N.bit_length() - 1
    llr = _f32(llr).reshape(-1, N)
    B = llr.shape[0]
    uh = np.zeros((B, N), np.uint8)
    lu = np.zeros((B, N), np.float64) if soft else None
    it = np.zeros(B, np.int32)
    ok = np.zeros(B, np.uint8)
    if W is not None:
        W = _f64(W)
        assert W.size >= max_iter * 2 * n * N
    _lib(prec).orc_bp_batch(_p(llr, _f32p), B, N, _p(fr, _u8p), c, poly, max_iter, stop,
                            llr_max, rule, _p(W, _f64p), _p(uh, _u8p), _p(lu, _f64p),
                            _p(it, _i32p), _p(ok, _u8p))
    out = dict(u_hat=uh, iters=it, ok=ok)
    if soft:
        out["llr_u"] = lu
    return out


def sc_frame(llr, frozen, rule=0, prec="f64") -> np.ndarray:
    llr = _f32(llr)
    fr = _u8(frozen)
    uh = np.zeros(len(fr), np.uint8)
    _lib(prec).orc_sc_frame(_p(llr, _f32p), len(fr), _p(fr, _u8p), rule, _p(uh, _u8p))
    return uh


def scl_frame(llr, frozen, L, c=0, poly=0, rule=0, prec="f64", all_paths=False, da=None):
    """CA-SCL of one frame; `da` (mask [N] or None) marks decision-aided
    positions, where every path takes its hard decision without branching."""
    llr = _f32(llr)
    fr = _u8(frozen)
    da = None if da is None else _u8(da)
    N = len(fr)
    uh = np.zeros(N, np.uint8)
    ok = np.zeros(1, np.uint8)
    pm = np.zeros(1, np.float64)
    au = np.zeros((L, N), np.uint8) if all_paths else None
    ap = np.zeros(L, np.float64) if all_paths else None
    ln = _lib(prec).orc_scl_frame(_p(llr, _f32p), N, _p(fr, _u8p), _p(da, _u8p), c, poly, L, rule,
                                  _p(uh, _u8p), _p(ok, _u8p), _p(pm, _f64p), _p(au, _u8p),
                                  _p(ap, _f64p))
    out = dict(u_hat=uh, crc_ok=int(ok[0]), pm=float(pm[0]), n_paths=ln)
    if all_paths:
        out["all_u"] = au[:ln]
        out["all_pm"] = ap[:ln]
    return out


def scl_batch(llr, frozen, L, c=0, poly=0, rule=0, prec="f64", da=None):
    fr = _u8(frozen)
    da = None if da is None else _u8(da)
    N = len(fr)
    llr = _f32(llr).reshape(-1, N)
    B = llr.shape[0]
    uh = np.zeros((B, N), np.uint8)
    ok = np.zeros(B, np.uint8)
    pm = np.zeros(B, np.float64)
    _lib(prec).orc_scl_batch(_p(llr, _f32p), B, N, _p(fr, _u8p), _p(da, _u8p), c, poly, L, rule,
                             _p(uh, _u8p), _p(ok, _u8p), _p(pm, _f64p))
    return dict(u_hat=uh, crc_ok=ok, pm=pm)


def hybrid_batch(llr, frozen, K, c, poly, max_iter, L, llr_max=20.0, W=None, prec="f64", da=None, rule=0, stop=1):
    """BP (rule 0 min-sum, 1 exact) with the re-encoding stop (stop 1) or the
    CRC stop (stop 2), then CA-SCL (min-sum metric) on the frames whose BP
    verdict is not ok."""
    assert stop in (1, 2)
    fr = _u8(frozen)
    da = None if da is None else _u8(da)
    N = len(fr)
    n = N.bit_length() - 1
    llr = _f32(llr).reshape(-1, N)
    B = llr.shape[0]
    info = np.zeros((B, K), np.uint8)
    used = np.zeros(B, np.uint8)
    it = np.zeros(B, np.int32)
    if W is not None:
        W = _f64(W)
        assert W.size >= max_iter * 2 * n * N
    _lib(prec).orc_hybrid_batch(_p(llr, _f32p), B, N, _p(fr, _u8p), _p(da, _u8p), K, c, poly, max_iter,
                                int(stop), llr_max, int(rule), _p(W, _f64p), L, _p(info, _u8p), _p(used, _u8p),
                                _p(it, _i32p))
    return dict(info=info, used_scl=used, iters=it)


def wbp_grad(llr, frozen, u_true, T, W, llr_max=20.0, scale=None, prec="f64", want_dllr=False, multi=False,
             kind=None, fail_weight=0.0):
    """Loss and gradients of the weighted BP (batch).  Returns (loss, dW[, dllr]).

    kind 0 (default): the BCE of LLR(u) after the last iteration; kind 1
    (or multi=True): the sum of that BCE after every iteration; kind 2: the
    frame-failure surrogate prod_t (1 - exp(-S_t)), S_t the frame's BCE sum
    after iteration t; kind 3: sum_{u<T} P_u + fail_weight * P_T with
    P_u = prod_{t<=u} (1 - exp(-S_t)) (expected iterations beyond the first of
    an early-stopping decoder, plus a price on frames still undecided after
    T).  scale defaults to 1 / (B * k) for kind 0, 1 / (B * k * T) for kind 1
    (means over frames, non-frozen bits and iterations) and 1 / B for kinds 2
    and 3 (the mean over frames)."""
    kind = (1 if multi else 0) if kind is None else int(kind)
    fr = _u8(frozen)
    N = len(fr)
    n = N.bit_length() - 1
    llr = _f32(llr).reshape(-1, N)
    u_true = _u8(u_true).reshape(-1, N)
    B = llr.shape[0]
    k = int((fr == 0).sum())
    if scale is None:
        scale = {0: 1.0 / (B * k), 1: 1.0 / (B * k * T), 2: 1.0 / B, 3: 1.0 / B}[kind]
    W = _f64(W).reshape(T, 2, n, N)
    dW = np.zeros((T, 2, n, N), np.float64)
    dl = np.zeros((B, N), np.float64) if want_dllr else None
    loss = _lib(prec).orc_wbp_grad_batch(_p(llr, _f32p), B, N, _p(fr, _u8p), _p(u_true, _u8p),
                                         T, llr_max, _p(W, _f64p), scale, kind, float(fail_weight), _p(dW, _f64p),
                                         _p(dl, _f64p))
    if want_dllr:
        return loss, dW, dl
    return loss, dW


def wbp_backward(llr, frozen, T, W, dlam, llr_max=20.0, prec="f64"):
    """Adjoint of the weighted BP for a given d loss / d lambda: [B][N] (after
    the last iteration) or [B][T][N] (after every iteration).
    Returns (dW [T][2][n][N] summed over frames in frame order, dllr [B][N])."""
    fr = _u8(frozen)
    N = len(fr)
    n = N.bit_length() - 1
    llr = _f32(llr).reshape(-1, N)
    B = llr.shape[0]
    W = _f64(W).reshape(T, 2, n, N)
    dlam = _f64(dlam)
    nl = T if dlam.size == B * T * N and dlam.size != B * N else 1
    dlam = dlam.reshape(B, nl, N)
    dW = np.zeros((T, 2, n, N), np.float64)
    dl = np.zeros((B, N), np.float64)
    _lib(prec).orc_wbp_backward_batch(_p(llr, _f32p), B, N, _p(fr, _u8p), T, llr_max, _p(W, _f64p),
                                      _p(dlam, _f64p), nl, _p(dW, _f64p), _p(dl, _f64p))
    return dW, dl


def adam_step(w, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (w, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _lib().orc_adam_step(_p(w, _f64p), _p(grad, _f64p), _p(m, _f64p), _p(v, _f64p), w.size, t,
                         lr, beta1, beta2, eps)


def lib_path(prec: str = "f64") -> str:
    return _build.LIBS[prec]


__all__ = [n for n in dir() if not n.startswith("_")]
