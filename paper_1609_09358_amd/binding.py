"""Thin Python binding of libpolarhip (the C ABI in include/polar.h).

Argument marshalling only: every function here checks tensor shapes, dtypes
and devices, takes raw device pointers and the current HIP stream from torch,
and calls the entry point of the same name.  All decoding runs in the HIP
kernels of the library.  There is no fallback: if the library is missing the
import of this module's functions raises.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolarhip.so")

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "NO_MEMORY", 4: "DEVICE", 5: "WORKSPACE"}
DEFAULT_POLY = {0: 0, 8: 0x07, 16: 0x1021, 24: 0x864CFB}


class PolarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class polar_code_desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("crc_bits", C.c_int32), ("crc_poly", C.c_uint32),
                ("design_ebn0_db", C.c_double), ("frozen", C.POINTER(C.c_uint8)), ("da_bits", C.c_int32)]


class bp_params(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("stop", C.c_int32), ("llr_max", C.c_float), ("rule", C.c_int32),
                ("weights", C.c_void_p), ("weight_iters", C.c_int32), ("variant", C.c_int32),
                ("weight_layout", C.c_int32)]


_lib = None


def lib():
    """Load libpolarhip.so (built by build.py); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpolarhip.so not found at {LIB_PATH}: build it with "
                               "python paper_1609_09358_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_size_t
        L.polar_last_error.restype = C.c_char_p
        L.polar_last_error.argtypes = []
        sig = {
            "polar_build_code": [C.POINTER(polar_code_desc), C.POINTER(vp)],
            "polar_construct_frozen": [i32, i32, i32, C.c_double, C.POINTER(C.c_uint8)],
            "polar_code_params": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(u32)],
            "polar_code_frozen": [vp, C.POINTER(C.c_uint8)],
            "polar_code_decision_aided": [vp, C.POINTER(C.c_uint8)],
            "polar_encode": [vp, vp, i64, vp, vp, vp],
            "polar_channel_awgn": [vp, vp, vp, i64, i32, vp, vp],
            "bp_decode_batch": [vp, vp, i64, C.POINTER(bp_params), vp, vp, vp, vp, vp],
            "polar_bp_variants": [i32, C.POINTER(i32), i32, C.POINTER(i32)],
            "scl_decode_batch": [vp, vp, i64, i32, vp, vp, vp, vp, vp, sz, vp],
            "hybrid_decode_batch": [vp, vp, i64, C.POINTER(bp_params), i32, vp, vp, vp, vp, sz, vp],
            "hybrid_decode_batch_static": [vp, vp, i64, C.POINTER(bp_params), i32, vp, vp, vp, vp],
            "polar_workspace_size": [vp, i64, i32, C.POINTER(bp_params), C.POINTER(sz)],
            "wbp_forward": [vp, vp, i64, vp, i32, C.c_float, i32, vp, vp, vp, vp],
            "wbp_bce": [vp, vp, vp, i64, C.c_double, vp, vp, vp],
            "wbp_backward": [vp, vp, i64, vp, i32, C.c_float, i32, vp, vp, i32, vp, vp, vp],
            "wbp_bce_multi": [vp, vp, vp, i64, i32, C.c_double, vp, vp, vp],
            "polar_adam_step": [vp, vp, vp, vp, i64, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp],
            "polar_adam_step_bounded": [vp, vp, vp, vp, i64, i32] + [C.c_float] * 6 + [vp],
            "wbp_frame_loss": [vp, vp, vp, i64, i32, C.c_double, vp, vp, vp],
            "wbp_iteration_loss": [vp, vp, vp, i64, i32, C.c_double, C.c_double, vp, vp, vp],
            "wbp_column_weights": [vp, vp, i32, vp, vp],
            "wbp_column_grad": [vp, vp, i32, vp, vp],
            "polar_set_scl_lds_budget": [i64],
            "polar_set_pipeline_bp_occupancy": [i32],
            "polar_set_pipeline_scl_occupancy": [i32],
            "polar_set_scl_ranking": [i32],
            "hybrid_decode_pipelined": [vp, i64, vp, i64, C.POINTER(bp_params), i32, vp, vp, vp, vp, sz, vp, vp],
            "polar_pipeline_workspace_size": [vp, i64, i32, C.POINTER(bp_params), C.POINTER(sz)],
            "polar_mixed_create": [vp, i32, i64, C.POINTER(bp_params), i32, vp, C.POINTER(vp)],
            "polar_mixed_decode": [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp],
            "polar_mixed_decode_graph": [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.polar_set_hybrid_graphs.argtypes = [i32]
        L.polar_set_hybrid_graphs.restype = C.c_int
        L.polar_get_hybrid_graphs.argtypes = []
        L.polar_get_hybrid_graphs.restype = i32
        L.polar_get_scl_ranking.argtypes = []
        L.polar_get_scl_ranking.restype = i32
        L.polar_get_pipeline_bp_occupancy.argtypes = []
        L.polar_get_pipeline_bp_occupancy.restype = i32
        L.polar_get_pipeline_scl_occupancy.argtypes = []
        L.polar_get_pipeline_scl_occupancy.restype = i32
        L.polar_get_scl_lds_budget.argtypes = []
        L.polar_get_scl_lds_budget.restype = i64
        L.polar_mixed_free.argtypes = [vp]
        L.polar_mixed_free.restype = None
        L.polar_free_code.argtypes = [vp]
        L.polar_free_code.restype = None
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise PolarError(status, lib().polar_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape, name):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


# --------------------------------------------------------------------------- codes

class PolarCode:
    """Owner of a polar_code handle (frozen set and device tables)."""

    def __init__(self, N, K, crc_bits=0, crc_poly=0, design_ebn0_db=2.0, frozen=None, da_bits=0):
        d = polar_code_desc()
        d.N, d.K, d.crc_bits = N, K, crc_bits
        d.da_bits = da_bits
        d.crc_poly = crc_poly
        d.design_ebn0_db = design_ebn0_db
        self._frozen_in = None
        if frozen is not None:
            self._frozen_in = np.ascontiguousarray(frozen, dtype=np.uint8)
            d.frozen = self._frozen_in.ctypes.data_as(C.POINTER(C.c_uint8))
        h = C.c_void_p()
        _check(lib().polar_build_code(C.byref(d), C.byref(h)))
        self.handle = h
        n_, k_, c_, p_ = C.c_int32(), C.c_int32(), C.c_int32(), C.c_uint32()
        _check(lib().polar_code_params(h, C.byref(n_), C.byref(k_), C.byref(c_), C.byref(p_)))
        self.N, self.K, self.crc_bits, self.crc_poly = n_.value, k_.value, c_.value, p_.value
        self.n = self.N.bit_length() - 1
        self.k = self.K + self.crc_bits
        mask = np.zeros(self.N, np.uint8)
        _check(lib().polar_code_frozen(h, mask.ctypes.data_as(C.POINTER(C.c_uint8))))
        self.frozen = mask
        self.info_pos = np.where(mask == 0)[0]
        da = np.zeros(self.N, np.uint8)
        _check(lib().polar_code_decision_aided(h, da.ctypes.data_as(C.POINTER(C.c_uint8))))
        self.decision_aided = da

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.polar_free_code(h)
            self.handle = None


def polar_construct_frozen(N, K, crc_bits=0, design_ebn0_db=2.0):
    """Frozen mask (1 = frozen) of the library's construction, computed on the host."""
    mask = np.zeros(N, np.uint8)
    _check(lib().polar_construct_frozen(N, K, crc_bits, design_ebn0_db, mask.ctypes.data_as(C.POINTER(C.c_uint8))))
    return mask


def polar_build_code(N, K, crc_bits=0, crc_poly=0, design_ebn0_db=2.0, frozen=None) -> PolarCode:
    return PolarCode(N, K, crc_bits, crc_poly, design_ebn0_db, frozen)


def make_bp_params(max_iter=100, stop=1, llr_max=20.0, weights=None, variant=0, rule=0):
    """weights: [T][2][n][N] (one per node) or [T][2][n] (one per stage column)."""
    p = bp_params()
    p.max_iter, p.stop, p.llr_max, p.rule = int(max_iter), int(stop), float(llr_max), int(rule)
    p.weights = None if weights is None else weights.data_ptr()
    p.weight_iters = 0 if weights is None else int(weights.shape[0])
    p.variant = int(variant)
    p.weight_layout = 1 if weights is not None and weights.dim() == 3 else 0
    return p


# --------------------------------------------------------------------------- entry points

def polar_encode(code: PolarCode, info: torch.Tensor, want_u=False):
    B = info.shape[0]
    _dev(info, torch.uint8, (B, code.K), "info")
    x = torch.empty((B, code.N), dtype=torch.uint8, device=info.device)
    u = torch.empty_like(x) if want_u else None
    _check(lib().polar_encode(code.handle, _ptr(info), B, _ptr(u), _ptr(x), _stream()))
    return (u, x) if want_u else x


def polar_channel_awgn(x: torch.Tensor, z: torch.Tensor, sigma2: torch.Tensor) -> torch.Tensor:
    B, N = x.shape
    _dev(x, torch.uint8, (B, N), "x")
    _dev(z, torch.float32, (B, N), "z")
    _dev(sigma2, torch.float32, (B,), "sigma2")
    llr = torch.empty((B, N), dtype=torch.float32, device=x.device)
    _check(lib().polar_channel_awgn(_ptr(x), _ptr(z), _ptr(sigma2), B, N, _ptr(llr), _stream()))
    return llr


def bp_decode_batch(code: PolarCode, llr: torch.Tensor, max_iter=100, stop=1, llr_max=20.0, weights=None,
                    variant=0, soft=False, out=None, rule=0):
    B = llr.shape[0]
    _dev(llr, torch.float32, (B, code.N), "llr")
    if weights is not None:
        _dev(weights, torch.float32, (weights.shape[0], 2, code.n) + ((code.N,) if weights.dim() == 4 else ()),
             "weights")
    dev = llr.device
    if out is None:
        out = dict(u_hat=torch.empty((B, code.N), dtype=torch.uint8, device=dev),
                   iters=torch.empty(B, dtype=torch.int32, device=dev),
                   ok=torch.empty(B, dtype=torch.uint8, device=dev))
        if soft:
            out["llr_u"] = torch.empty((B, code.N), dtype=torch.float32, device=dev)
    p = make_bp_params(max_iter, stop, llr_max, weights, variant, rule)
    _check(lib().bp_decode_batch(code.handle, _ptr(llr), B, C.byref(p), _ptr(out["u_hat"]), _ptr(out.get("llr_u")),
                                 _ptr(out["iters"]), _ptr(out["ok"]), _stream()))
    return out


def polar_bp_variants(N):
    ids = (C.c_int32 * 8)()
    cnt = C.c_int32()
    _check(lib().polar_bp_variants(N, ids, 8, C.byref(cnt)))
    return [ids[i] for i in range(cnt.value)]


def polar_workspace_size(code: PolarCode, B, L, hybrid_params=None):
    s = C.c_size_t()
    p = C.byref(hybrid_params) if hybrid_params is not None else None
    _check(lib().polar_workspace_size(code.handle, B, L, p, C.byref(s)))
    return s.value


def polar_set_scl_lds_budget(nbytes: int):
    """Per-workgroup LDS budget of the list decoder (0 = default); process-wide."""
    _check(lib().polar_set_scl_lds_budget(int(nbytes)))


def polar_get_scl_lds_budget() -> int:
    return int(lib().polar_get_scl_lds_budget())


def polar_set_scl_ranking(mode: int):
    """List decoder survivor selection: 0 automatic, 1 pruned pseudo sort, 2 bitonic network,
    3 threshold selection."""
    _check(lib().polar_set_scl_ranking(int(mode)))


def polar_get_scl_ranking() -> int:
    return int(lib().polar_get_scl_ranking())


def polar_set_hybrid_graphs(mode: int):
    """hybrid_decode_batch: 1 (default) replay a captured graph from the second
    call with the same arguments on, 0 launch the kernels directly."""
    _check(lib().polar_set_hybrid_graphs(int(mode)))


def polar_get_hybrid_graphs() -> int:
    return int(lib().polar_get_hybrid_graphs())


def polar_set_pipeline_bp_occupancy(wgs_per_cu: int):
    """BP workgroups per CU in the pipelined hybrid (0 = no limit); process-wide."""
    _check(lib().polar_set_pipeline_bp_occupancy(int(wgs_per_cu)))


def polar_get_pipeline_bp_occupancy() -> int:
    return int(lib().polar_get_pipeline_bp_occupancy())


def polar_set_pipeline_scl_occupancy(wgs_per_cu: int):
    """List-decoder workgroups per CU in the pipelined hybrid (0 = as many as
    fit); process-wide."""
    _check(lib().polar_set_pipeline_scl_occupancy(int(wgs_per_cu)))


def polar_get_pipeline_scl_occupancy() -> int:
    return int(lib().polar_get_pipeline_scl_occupancy())


def scl_decode_batch(code: PolarCode, llr: torch.Tensor, L, frame_ids=None, out=None, workspace=None):
    rows = llr.shape[0]
    _dev(llr, torch.float32, (rows, code.N), "llr")
    B = rows if frame_ids is None else frame_ids.shape[0]
    if frame_ids is not None:
        _dev(frame_ids, torch.int32, (B,), "frame_ids")
    dev = llr.device
    if out is None:
        out = dict(u_hat=torch.zeros((rows, code.N), dtype=torch.uint8, device=dev),
                   crc_ok=torch.zeros(rows, dtype=torch.uint8, device=dev),
                   pm=torch.zeros(rows, dtype=torch.float32, device=dev))
    need = polar_workspace_size(code, B, L)
    if workspace is None and need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().scl_decode_batch(code.handle, _ptr(llr), B, L, _ptr(frame_ids), _ptr(out["u_hat"]),
                                  _ptr(out["crc_ok"]), _ptr(out["pm"]), _ptr(workspace),
                                  0 if workspace is None else workspace.numel(), _stream()))
    return out


class HybridDecoder:
    """hybrid_decode_batch with its workspace kept between calls."""

    def __init__(self, code: PolarCode, max_iter=200, L=8, stop=1, llr_max=20.0, weights=None, variant=0, rule=0):
        self.code, self.L = code, L
        self.weights = weights
        self.params = make_bp_params(max_iter, stop, llr_max, weights, variant, rule)
        self.workspace = None

    def __call__(self, llr: torch.Tensor, out=None, stats=None):
        return hybrid_decode_batch(self.code, llr, self.params, self.L, out=out, stats=stats, decoder=self)


def hybrid_decode_batch(code: PolarCode, llr: torch.Tensor, params: bp_params, L: int, out=None, stats=None,
                        workspace=None, decoder=None):
    B = llr.shape[0]
    _dev(llr, torch.float32, (B, code.N), "llr")
    dev = llr.device
    if out is None:
        out = dict(info=torch.empty((B, code.K), dtype=torch.uint8, device=dev),
                   used_scl=torch.empty(B, dtype=torch.uint8, device=dev))
    if stats is not None:
        _dev(stats, torch.int64, (8,), "stats")
    need = polar_workspace_size(code, B, L, params)
    if workspace is None and decoder is not None:
        if decoder.workspace is None or decoder.workspace.numel() < need:
            decoder.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        workspace = decoder.workspace
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().hybrid_decode_batch(code.handle, _ptr(llr), B, C.byref(params), L, _ptr(out["info"]),
                                     _ptr(out["used_scl"]), _ptr(stats), _ptr(workspace), workspace.numel(),
                                     _stream()))
    return out


def hybrid_decode_batch_static(code: PolarCode, llr: torch.Tensor, params: bp_params, L: int, out=None,
                               stats=None):
    """hybrid_decode_batch without a workspace: the library's fixed device
    scratch is used (no allocation inside the call; calls on one device must
    not overlap)."""
    B = llr.shape[0]
    _dev(llr, torch.float32, (B, code.N), "llr")
    dev = llr.device
    if out is None:
        out = dict(info=torch.empty((B, code.K), dtype=torch.uint8, device=dev),
                   used_scl=torch.empty(B, dtype=torch.uint8, device=dev))
    _dev(out["info"], torch.uint8, (B, code.K), "info")
    _dev(out.get("used_scl"), torch.uint8, (B,), "used_scl")
    if stats is not None:
        _dev(stats, torch.int64, (8,), "stats")
    _check(lib().hybrid_decode_batch_static(code.handle, _ptr(llr), B, C.byref(params), L, _ptr(out["info"]),
                                            _ptr(out.get("used_scl")), _ptr(stats), _stream()))
    return out


def polar_pipeline_workspace_size(code: PolarCode, B, L, params: bp_params) -> int:
    s = C.c_size_t()
    _check(lib().polar_pipeline_workspace_size(code.handle, B, L, C.byref(params), C.byref(s)))
    return s.value


class HybridPipeline:
    """hybrid_decode_pipelined (BP on the current stream, CA-SCL and merge on a
    second stream of default priority) with its workspace kept between calls."""

    def __init__(self, code: PolarCode, max_iter=200, L=8, stop=1, llr_max=20.0, weights=None, variant=0):
        self.code, self.L = code, L
        self.weights = weights
        self.params = make_bp_params(max_iter, stop, llr_max, weights, variant)
        self.workspace = None
        self.scl_stream = torch.cuda.Stream()

    def __call__(self, llrs, outs=None, stats=None, want_used=False):
        """Decode the batches `llrs` (a list of [B][N] tensors of one shape, which
        may repeat); returns one dict(info[, used_scl]) per batch."""
        code = self.code
        nb = len(llrs)
        if nb == 0:
            return []
        B = llrs[0].shape[0]
        for t in llrs:
            _dev(t, torch.float32, (B, code.N), "llr")
        dev = llrs[0].device
        if outs is None:
            outs = []
            for _ in range(nb):
                o = dict(info=torch.empty((B, code.K), dtype=torch.uint8, device=dev))
                if want_used:
                    o["used_scl"] = torch.empty(B, dtype=torch.uint8, device=dev)
                outs.append(o)
        if stats is not None:
            _dev(stats, torch.int64, (8,), "stats")
        need = polar_pipeline_workspace_size(code, B, self.L, self.params)
        if self.workspace is None or self.workspace.numel() < need:
            self.workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        arr = C.c_void_p * nb
        llr_a = arr(*[t.data_ptr() for t in llrs])
        info_a = arr(*[o["info"].data_ptr() for o in outs])
        used_a = arr(*[o["used_scl"].data_ptr() for o in outs]) if all("used_scl" in o for o in outs) else None
        _check(lib().hybrid_decode_pipelined(code.handle, nb, llr_a, B, C.byref(self.params), self.L, info_a, used_a,
                                             _ptr(stats), _ptr(self.workspace), self.workspace.numel(), _stream(),
                                             C.c_void_p(self.scl_stream.cuda_stream)))
        return outs


class MixedPlan:
    """polar_mixed plan: hybrid decoding of ragged batches mixing several codes."""

    def __init__(self, codes, max_frames, max_iter=200, L=8, stop=1, llr_max=20.0, variants=None):
        self.codes = list(codes)
        self.max_frames = int(max_frames)
        self.params = make_bp_params(max_iter, stop, llr_max)
        n = len(self.codes)
        arr = (C.c_void_p * n)(*[c.handle.value for c in self.codes])
        var = None if variants is None else (C.c_int32 * n)(*[int(v) for v in variants])
        h = C.c_void_p()
        _check(lib().polar_mixed_create(arr, n, self.max_frames, C.byref(self.params), int(L), var, C.byref(h)))
        self.handle = h

    def layout(self, code_of_frame):
        """Row offsets of a ragged batch laid out densely in frame order:
        (llr_off, out_off, total LLR elements, total information bits)."""
        cf = np.asarray(code_of_frame)
        Ns = np.array([c.N for c in self.codes], np.int64)[cf]
        Ks = np.array([c.K for c in self.codes], np.int64)[cf]
        llr_off = np.concatenate([[0], np.cumsum(Ns)[:-1]]).astype(np.int64)
        out_off = np.concatenate([[0], np.cumsum(Ks)[:-1]]).astype(np.int64)
        return llr_off, out_off, int(Ns.sum()), int(Ks.sum())

    def __call__(self, llr, code_of_frame, llr_off, out_off, info_hat, used_scl=None, stats=None, graph=False):
        B = int(code_of_frame.shape[0])
        for t, dt, nm in ((code_of_frame, torch.int32, "code_of_frame"), (llr_off, torch.int64, "llr_off"),
                          (out_off, torch.int64, "out_off")):
            _dev(t, dt, (B,), nm)
        _dev(llr, torch.float32, None, "llr")
        _dev(info_hat, torch.uint8, None, "info_hat")
        if used_scl is not None:
            _dev(used_scl, torch.uint8, (B,), "used_scl")
        if stats is not None:
            _dev(stats, torch.int64, (8,), "stats")
        fn = lib().polar_mixed_decode_graph if graph else lib().polar_mixed_decode
        _check(fn(self.handle, B, _ptr(llr), _ptr(code_of_frame), _ptr(llr_off), _ptr(out_off), _ptr(info_hat),
                  _ptr(used_scl), _ptr(stats), _stream()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.polar_mixed_free(h)
            self.handle = None


# --------------------------------------------------------------------------- weighted (learned) BP

def wbp_forward(code: PolarCode, llr, W, llr_max=20.0, variant=0, save=False, out=None):
    """T = W.shape[0] weighted iterations, no early stop.  Returns dict(llr_u, u_hat[, saved])."""
    B = llr.shape[0]
    T = W.shape[0]
    _dev(llr, torch.float32, (B, code.N), "llr")
    _dev(W, torch.float32, (T, 2, code.n, code.N), "W")
    dev = llr.device
    if out is None:
        out = dict(llr_u=torch.empty((B, code.N), dtype=torch.float32, device=dev),
                   u_hat=torch.empty((B, code.N), dtype=torch.uint8, device=dev))
        if save:
            out["saved"] = torch.empty((B, T, 2, code.n, code.N), dtype=torch.float32, device=dev)
    _check(lib().wbp_forward(code.handle, _ptr(llr), B, _ptr(W), T, llr_max, variant, _ptr(out["llr_u"]),
                             _ptr(out["u_hat"]), _ptr(out.get("saved")), _stream()))
    return out


def wbp_bce(code: PolarCode, llr_u, u_true, scale=None, want_loss=True):
    """Per-frame BCE loss (times scale) and d loss / d llr_u; scale defaults to 1/(B k)."""
    B = llr_u.shape[0]
    _dev(llr_u, torch.float32, (B, code.N), "llr_u")
    _dev(u_true, torch.uint8, (B, code.N), "u_true")
    if scale is None:
        scale = 1.0 / (B * code.k)
    dlam = torch.empty_like(llr_u)
    loss = torch.empty(B, dtype=torch.float32, device=llr_u.device) if want_loss else None
    _check(lib().wbp_bce(code.handle, _ptr(llr_u), _ptr(u_true), B, float(scale), _ptr(loss), _ptr(dlam), _stream()))
    return loss, dlam


def wbp_bce_multi(code: PolarCode, saved, u_true, T, scale=None, want_loss=True):
    """Per-frame loss summed over all T iterations (times scale) and
    d loss / d LLR(u) after every iteration, [B][T][N]; scale defaults to
    1/(B k T).  Call before wbp_backward, which consumes `saved`."""
    B = saved.shape[0]
    _dev(saved, torch.float32, (B, T, 2, code.n, code.N), "saved")
    _dev(u_true, torch.uint8, (B, code.N), "u_true")
    if scale is None:
        scale = 1.0 / (B * code.k * T)
    dlam = torch.empty((B, T, code.N), dtype=torch.float32, device=saved.device)
    loss = torch.empty(B, dtype=torch.float32, device=saved.device) if want_loss else None
    _check(lib().wbp_bce_multi(code.handle, _ptr(saved), _ptr(u_true), B, T, float(scale), _ptr(loss), _ptr(dlam),
                               _stream()))
    return loss, dlam


def wbp_frame_loss(code: PolarCode, saved, u_true, T, scale=None, want_loss=True):
    """Frame-failure surrogate prod_t (1 - exp(-S_t)) per frame (times scale)
    and d loss / d LLR(u) after every iteration, [B][T][N]; scale defaults to
    1/B.  Call before wbp_backward, which consumes `saved`."""
    B = saved.shape[0]
    _dev(saved, torch.float32, (B, T, 2, code.n, code.N), "saved")
    _dev(u_true, torch.uint8, (B, code.N), "u_true")
    if scale is None:
        scale = 1.0 / B
    dlam = torch.empty((B, T, code.N), dtype=torch.float32, device=saved.device)
    loss = torch.empty(B, dtype=torch.float32, device=saved.device) if want_loss else None
    _check(lib().wbp_frame_loss(code.handle, _ptr(saved), _ptr(u_true), B, T, float(scale), _ptr(loss), _ptr(dlam),
                                _stream()))
    return loss, dlam


def wbp_iteration_loss(code: PolarCode, saved, u_true, T, fail_weight, scale=None, want_loss=True):
    """Expected-iterations loss sum_{u<T} P_u + fail_weight * P_T per frame
    (times scale) and d loss / d LLR(u) after every iteration, [B][T][N];
    scale defaults to 1/B.  Call before wbp_backward, which consumes `saved`."""
    B = saved.shape[0]
    _dev(saved, torch.float32, (B, T, 2, code.n, code.N), "saved")
    _dev(u_true, torch.uint8, (B, code.N), "u_true")
    if scale is None:
        scale = 1.0 / B
    dlam = torch.empty((B, T, code.N), dtype=torch.float32, device=saved.device)
    loss = torch.empty(B, dtype=torch.float32, device=saved.device) if want_loss else None
    _check(lib().wbp_iteration_loss(code.handle, _ptr(saved), _ptr(u_true), B, T, float(fail_weight), float(scale),
                                    _ptr(loss), _ptr(dlam), _stream()))
    return loss, dlam


def wbp_column_weights(code: PolarCode, Wc, out=None):
    """[T][2][n] column weights -> [T][2][n][N] per-node weights."""
    T = Wc.shape[0]
    _dev(Wc, torch.float32, (T, 2, code.n), "Wc")
    if out is None:
        out = torch.empty((T, 2, code.n, code.N), dtype=torch.float32, device=Wc.device)
    _dev(out, torch.float32, (T, 2, code.n, code.N), "W")
    _check(lib().wbp_column_weights(code.handle, _ptr(Wc), T, _ptr(out), _stream()))
    return out


def wbp_column_grad(code: PolarCode, dW, out=None):
    """[T][2][n][N] per-node gradient -> [T][2][n] column sums."""
    T = dW.shape[0]
    _dev(dW, torch.float32, (T, 2, code.n, code.N), "dW")
    if out is None:
        out = torch.empty((T, 2, code.n), dtype=torch.float32, device=dW.device)
    _dev(out, torch.float32, (T, 2, code.n), "dWc")
    _check(lib().wbp_column_grad(code.handle, _ptr(dW), T, _ptr(out), _stream()))
    return out


def wbp_backward(code: PolarCode, llr, W, saved, dlam, llr_max=20.0, variant=0, want_dllr=False):
    """Weight gradient (summed over frames) and optionally d/d llr; `saved` is
    consumed.  dlam: [B][N] (loss after the last iteration) or [B][T][N]."""
    B = llr.shape[0]
    T = W.shape[0]
    _dev(llr, torch.float32, (B, code.N), "llr")
    _dev(W, torch.float32, (T, 2, code.n, code.N), "W")
    _dev(saved, torch.float32, (B, T, 2, code.n, code.N), "saved")
    dlam_iters = T if dlam.dim() == 3 else 1
    _dev(dlam, torch.float32, (B, T, code.N) if dlam.dim() == 3 else (B, code.N), "dlam")
    dW = torch.empty_like(W)
    dllr = torch.empty_like(llr) if want_dllr else None
    _check(lib().wbp_backward(code.handle, _ptr(llr), B, _ptr(W), T, llr_max, variant, _ptr(saved), _ptr(dlam),
                              dlam_iters, _ptr(dW), _ptr(dllr), _stream()))
    return dW, dllr


def polar_adam_step(w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    for name, t in (("w", w), ("g", g), ("m", m), ("v", v)):
        _dev(t, torch.float32, tuple(w.shape), name)
    _check(lib().polar_adam_step(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), int(step), lr, beta1, beta2, eps,
                                 _stream()))


def polar_adam_step_bounded(w, g, m, v, step, lr=1e-3, lo=0.0, hi=1.0, beta1=0.9, beta2=0.999, eps=1e-8):
    for name, t in (("w", w), ("g", g), ("m", m), ("v", v)):
        _dev(t, torch.float32, tuple(w.shape), name)
    _check(lib().polar_adam_step_bounded(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), int(step), lr, beta1, beta2,
                                         eps, lo, hi, _stream()))


class WeightedBPLoss(torch.autograd.Function):
    """loss = mean BCE of the weighted BP's soft outputs on the non-frozen bits.

    forward(llr, W, u_true, code) runs wbp_forward (saving messages) and wbp_bce
    in the library; backward runs wbp_backward.  Gradients flow to W (and to the
    channel LLRs when they require grad)."""

    @staticmethod
    def forward(ctx, llr, W, u_true, code):
        fw = wbp_forward(code, llr.detach().contiguous(), W.detach().contiguous(), save=True)
        loss_f, dlam = wbp_bce(code, fw["llr_u"], u_true)
        ctx.code = code
        ctx.save_for_backward(llr.detach(), W.detach(), fw["saved"], dlam)
        return loss_f.sum()

    @staticmethod
    def backward(ctx, grad_out):
        llr, W, saved, dlam = ctx.saved_tensors
        dlam = dlam * grad_out if grad_out.numel() == 1 and float(grad_out) != 1.0 else dlam
        dW, dllr = wbp_backward(ctx.code, llr, W, saved, dlam.contiguous(), want_dllr=ctx.needs_input_grad[0])
        return dllr, dW, None, None


EXPORTED = ["polar_last_error", "polar_build_code", "polar_construct_frozen", "polar_free_code", "polar_code_params", "polar_code_frozen",
            "polar_code_decision_aided",
            "polar_encode", "polar_channel_awgn", "bp_decode_batch", "polar_bp_variants", "scl_decode_batch",
            "hybrid_decode_batch", "hybrid_decode_batch_static", "polar_set_hybrid_graphs",
            "polar_get_hybrid_graphs", "polar_workspace_size", "wbp_forward", "wbp_bce",
            "wbp_backward", "wbp_bce_multi", "wbp_frame_loss", "wbp_iteration_loss", "wbp_column_weights", "wbp_column_grad",
            "polar_adam_step", "polar_adam_step_bounded", "polar_set_scl_lds_budget", "polar_get_scl_lds_budget",
            "hybrid_decode_pipelined", "polar_pipeline_workspace_size", "polar_set_pipeline_bp_occupancy",
            "polar_get_pipeline_bp_occupancy", "polar_set_pipeline_scl_occupancy",
            "polar_get_pipeline_scl_occupancy", "polar_set_scl_ranking", "polar_get_scl_ranking", "polar_mixed_create", "polar_mixed_decode",
            "polar_mixed_decode_graph", "polar_mixed_free"]
