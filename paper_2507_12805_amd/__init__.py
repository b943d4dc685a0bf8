"""Python binding of libpmklc (the MI355X PMKLC hot path).

Argument marshalling only: every step of compression and decompression
runs in the HIP kernels of ``libpmklc.so`` behind the C ABI declared in
``include/pmklc.h``. PyTorch provides device memory and the current stream.
If the library is missing, every entry point raises; there is no fallback.

Configurations are plain dicts with the keys of ``synth.workloads``
(s, k, t, bs, E, hidden, optimizer, lr, beta1, beta2, eps, selector,
smp_ppm, seed, n_blocks / block_len, file_blocks, ms_threshold, arch, heads,
static_arch, static_E, gru_h, gru_layers, dense) plus ``precision``
("fp32" | "bf16") and ``schedule`` ("batched" | "plain").
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmklc.so")
_lib = None

STATUS = {0: "ok", -1: "invalid argument", -2: "invalid base", -3: "buffer too small", -4: "corrupt container",
          -5: "model mismatch", -6: "device error", -7: "unsupported configuration",
          -8: "input exceeds the no-allocation scratch buffer"}


class PmklcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({code})")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("s", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("t", ctypes.c_uint32), ("bs", ctypes.c_uint32), ("embed", ctypes.c_uint32),
                ("n_hidden", ctypes.c_uint32), ("hidden", ctypes.c_uint32 * 4), ("optimizer", ctypes.c_uint32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("precision", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("selector", ctypes.c_uint32), ("smp_ppm", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("n_blocks", ctypes.c_uint32), ("block_len_host", ctypes.POINTER(ctypes.c_uint64)),
                ("n_files", ctypes.c_uint32), ("file_blocks_host", ctypes.POINTER(ctypes.c_uint64)),
                ("static_host", ctypes.POINTER(ctypes.c_float)), ("static_len", ctypes.c_uint64),
                ("ms_threshold", ctypes.c_uint64), ("arch", ctypes.c_uint32), ("heads", ctypes.c_uint32),
                ("static_arch", ctypes.c_uint32), ("static_embed", ctypes.c_uint32), ("gru_hidden", ctypes.c_uint32),
                ("gru_layers", ctypes.c_uint32), ("dense", ctypes.c_uint32)]


class Timing(ctypes.Structure):
    _fields_ = [("step_ms", ctypes.c_float), ("call_ms", ctypes.c_float), ("model_rows", ctypes.c_uint64),
                ("coded_tokens", ctypes.c_uint64), ("max_steps", ctypes.c_uint64), ("launches", ctypes.c_uint32),
                ("threads", ctypes.c_uint32), ("wall_khz", ctypes.c_uint32), ("phase_ticks", ctypes.c_uint64 * 12),
                ("f1_units", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_u64p = ctypes.POINTER(ctypes.c_uint64)


def load():
    """Load libpmklc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_2507_12805_amd/build.py (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    cp = ctypes.POINTER(_Config)
    L.pmklc_encode_skmer.argtypes = [_vp, _u64, _u32, _u32, _vp, _u64, _u64p, _vp]
    L.pmklc_compress_bound.argtypes = [cp, _u64, _u64p, _u64p]
    L.pmklc_compress.argtypes = [cp, _vp, _u64, _vp, _u64, _vp, _u64, _u64p, _vp]
    L.pmklc_compress_noalloc.argtypes = [cp, _vp, _u64, _vp, _u64, _u64p, _vp]
    L.pmklc_decompress_info.argtypes = [_vp, _u64, _u64p, _u64p]
    L.pmklc_decompress.argtypes = [_vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _u64p, _vp]
    L.pmklc_status_string.argtypes = [ctypes.c_int]
    L.pmklc_status_string.restype = ctypes.c_char_p
    L.pmklc_quantise.argtypes = [_vp, _u32, _u32, _vp, _vp]
    L.pmklc_wnc_encode.argtypes = [_vp, _vp, _u64, _vp, _u64, _u64p, _vp]
    L.pmklc_wnc_decode.argtypes = [_vp, _u64, _vp, _u32, _u64, _vp, _vp]
    L.pmklc_model_trace.argtypes = [cp, _vp, _u64, _vp, _vp, _u64, _u64p, _u32, _vp, _vp, _vp, _u64, _u64p, _vp]
    L.pmklc_dm_workspace.argtypes = [cp, _u32, _u64p]
    L.pmklc_dm_forward.argtypes = [cp, _vp, _vp, _u32, _vp, _vp, _u64, _vp]
    L.pmklc_dm_backward.argtypes = [cp, _vp, _vp, _u32, _vp, _vp, _vp, _u64, _vp]
    for f in ["pmklc_dm_workspace", "pmklc_dm_forward", "pmklc_dm_backward"]:
        getattr(L, f).restype = ctypes.c_int
    L.pmklc_last_timing.argtypes = [ctypes.POINTER(Timing)]
    L.pmklc_last_timing.restype = ctypes.c_int
    L.pmklc_param_count.argtypes = [cp]
    L.pmklc_param_count.restype = _u64
    for f in ["pmklc_encode_skmer", "pmklc_compress_bound", "pmklc_compress", "pmklc_compress_noalloc",
              "pmklc_decompress_info",
              "pmklc_decompress", "pmklc_quantise", "pmklc_wnc_encode", "pmklc_wnc_decode", "pmklc_model_trace"]:
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        raise PmklcError(rc, what)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(x, dtype):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)
    return t.contiguous()


SELECTORS = {"uniform": 0, "dm": 4, "spum_dm": 5, "sprm_dm": 6, "spum_sprm_dm": 7, "auto": 8}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp32_valu": 2}
ARCHS = {"mlp": 0, "transformer": 1}


def make_config(cfg: dict, static=None):
    """dict -> (ctypes config, keep-alive list)."""
    c = _Config()
    c.struct_size = ctypes.sizeof(_Config)
    c.s, c.k, c.t, c.bs, c.embed = cfg["s"], cfg["k"], cfg["t"], cfg["bs"], cfg["E"]
    h = list(cfg["hidden"])
    c.n_hidden = len(h)
    for i, v in enumerate(h):
        c.hidden[i] = v
    c.optimizer = 1 if cfg.get("optimizer", "sgd") == "adam" else 0
    c.lr, c.beta1, c.beta2, c.eps = cfg.get("lr", 1e-3), cfg.get("beta1", 0.9), cfg.get("beta2", 0.999), \
        cfg.get("eps", 1e-8)
    c.precision = PRECISIONS[cfg.get("precision", "fp32")]
    c.schedule = 1 if cfg.get("schedule", "batched") == "plain" else 0
    c.selector = SELECTORS[cfg.get("selector", "dm")]
    c.ms_threshold = int(cfg.get("ms_threshold", 0))
    c.arch = ARCHS[cfg.get("arch", "mlp")]
    c.heads = int(cfg.get("heads", 0)) if c.arch == 1 else 0
    if cfg.get("static_arch", "mlp") == "bigru":
        c.static_arch = 1
        c.static_embed, c.gru_hidden = int(cfg.get("static_E", 16)), int(cfg.get("gru_h", 32))
        c.gru_layers, c.dense = int(cfg.get("gru_layers", 2)), int(cfg.get("dense", 128))
    c.smp_ppm = int(cfg.get("smp_ppm", 0))
    c.seed = int(cfg["seed"])
    keep = []
    bl = cfg.get("block_len")
    if bl is not None:
        a = np.ascontiguousarray(bl, dtype=np.uint64)
        keep.append(a)
        c.n_blocks = len(a)
        c.block_len_host = a.ctypes.data_as(_u64p)
    else:
        c.n_blocks = int(cfg.get("n_blocks", 1))
    fb = cfg.get("file_blocks")
    if fb is not None:
        a = np.ascontiguousarray(fb, dtype=np.uint64)
        keep.append(a)
        c.n_files = len(a)
        c.file_blocks_host = a.ctypes.data_as(_u64p)
    else:
        c.n_files = 1
    if static is not None:
        s = np.ascontiguousarray(static, dtype=np.float32)
        keep.append(s)
        c.static_host = s.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        c.static_len = s.size
    return c, keep


def last_timing() -> dict:
    """HIP-event timing of the step kernel in the last compress/decompress
    call on this thread, and the work it did."""
    t = Timing()
    _check(load().pmklc_last_timing(ctypes.byref(t)), "pmklc_last_timing")
    out = {f: getattr(t, f) for f, _ in Timing._fields_}
    out["phase_ticks"] = list(t.phase_ticks)
    return out


def param_count(cfg: dict) -> int:
    c, _ = make_config(cfg)
    return int(load().pmklc_param_count(ctypes.byref(c)))


def encode_skmer(bases, s: int, k: int):
    """Sec. 4.1 GskE on the GPU: ASCII ACGT (device uint8 tensor) -> tokens."""
    torch = _torch()
    L = load()
    x = _dev_tensor(bases, torch.uint8)
    n = x.numel()
    l = (n - k) // s + 1 if n >= k else 0
    out = torch.empty(max(l, 1), dtype=torch.uint8, device="cuda")
    nt = ctypes.c_uint64(0)
    _check(L.pmklc_encode_skmer(_dptr(x) if n else None, n, s, k, _dptr(out), l, ctypes.byref(nt), _stream()),
           "pmklc_encode_skmer")
    return out[:nt.value]


class Workspace:
    """Device workspace reused across calls (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        return self.buf


_ws = Workspace()


def compress_bound(cfg: dict, n: int, static=None):
    c, keep = make_config(cfg, static)
    mo, ws = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().pmklc_compress_bound(ctypes.byref(c), n, ctypes.byref(mo), ctypes.byref(ws)),
           "pmklc_compress_bound")
    return mo.value, ws.value


def compress(cfg: dict, data, static=None, workspace: Workspace | None = None, out: np.ndarray | None = None) -> bytes:
    """Compress device-resident ASCII DNA (uint8 tensor) into a container."""
    torch = _torch()
    L = load()
    x = _dev_tensor(data, torch.uint8)
    n = x.numel()
    c, keep = make_config(cfg, static)
    mo, wsb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(L.pmklc_compress_bound(ctypes.byref(c), n, ctypes.byref(mo), ctypes.byref(wsb)), "pmklc_compress_bound")
    ws = (workspace or _ws).get(wsb.value)
    if out is None or out.size < mo.value:
        out = np.empty(mo.value, dtype=np.uint8)
    olen = ctypes.c_uint64(0)
    _check(L.pmklc_compress(ctypes.byref(c), _dptr(x) if n else None, n, _dptr(ws), ws.numel(),
                            out.ctypes.data_as(ctypes.c_void_p), out.size, ctypes.byref(olen), _stream()),
           "pmklc_compress")
    return out[:olen.value].tobytes()


def compress_noalloc(cfg: dict, data, static=None, out: np.ndarray | None = None) -> bytes:
    """pmklc_compress_noalloc: the same container as compress(), with the
    workspace taken from the library's fixed device buffer (no device
    allocation by the call)."""
    torch = _torch()
    L = load()
    x = _dev_tensor(data, torch.uint8)
    n = x.numel()
    c, keep = make_config(cfg, static)
    mo = ctypes.c_uint64(0)
    _check(L.pmklc_compress_bound(ctypes.byref(c), n, ctypes.byref(mo), None), "pmklc_compress_bound")
    if out is None or out.size < mo.value:
        out = np.empty(mo.value, dtype=np.uint8)
    olen = ctypes.c_uint64(0)
    _check(L.pmklc_compress_noalloc(ctypes.byref(c), _dptr(x) if n else None, n,
                                    out.ctypes.data_as(ctypes.c_void_p), out.size, ctypes.byref(olen), _stream()),
           "pmklc_compress_noalloc")
    return out[:olen.value].tobytes()


def decompress_info(blob: bytes):
    b = np.frombuffer(blob, dtype=np.uint8)
    nb, ws = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().pmklc_decompress_info(b.ctypes.data_as(ctypes.c_void_p), b.size, ctypes.byref(nb),
                                        ctypes.byref(ws)), "pmklc_decompress_info")
    return nb.value, ws.value


def decompress(blob: bytes, static=None, workspace: Workspace | None = None, out=None):
    """Container -> device uint8 tensor of ASCII DNA."""
    torch = _torch()
    L = load()
    b = np.frombuffer(blob, dtype=np.uint8)
    nb, wsb = decompress_info(blob)
    ws = (workspace or _ws).get(wsb)
    if out is None or out.numel() < nb:
        out = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    s = None if static is None else np.ascontiguousarray(static, dtype=np.float32)
    olen = ctypes.c_uint64(0)
    _check(L.pmklc_decompress(b.ctypes.data_as(ctypes.c_void_p), b.size,
                              s.ctypes.data_as(ctypes.c_void_p) if s is not None else None,
                              0 if s is None else s.size, _dptr(ws), ws.numel(), _dptr(out), out.numel(),
                              ctypes.byref(olen), _stream()), "pmklc_decompress")
    return out[:olen.value]


# ---------------------------------------------------------------- test exports
def quantise(P):
    """[rows, V] FP32 probabilities (device) -> [rows, V+1] integer CDF."""
    torch = _torch()
    P = _dev_tensor(P, torch.float32)
    rows, V = P.shape
    out = torch.zeros((rows, V + 1), dtype=torch.int32, device="cuda")
    _check(load().pmklc_quantise(_dptr(P), rows, V, _dptr(out), _stream()), "pmklc_quantise")
    return out


def wnc_encode(cum_lo, cum_hi):
    torch = _torch()
    lo = _dev_tensor(np.asarray(cum_lo, dtype=np.int64).astype(np.int32), torch.int32)
    hi = _dev_tensor(np.asarray(cum_hi, dtype=np.int64).astype(np.int32), torch.int32)
    m = lo.numel()
    cap = 4 * ((17 * m + 2 + 31) // 32 + 1)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    nbits = ctypes.c_uint64(0)
    _check(load().pmklc_wnc_encode(_dptr(lo), _dptr(hi), m, _dptr(out), cap, ctypes.byref(nbits), _stream()),
           "pmklc_wnc_encode")
    nb = (nbits.value + 7) // 8
    return out[:nb].cpu().numpy().tobytes(), nbits.value


def wnc_decode(data: bytes, cdfs):
    torch = _torch()
    c = _dev_tensor(np.asarray(cdfs, dtype=np.int64).astype(np.int32), torch.int32)
    m, V1 = c.shape
    padded = data + b"\0" * ((-len(data)) % 4)
    buf = torch.tensor(list(padded) or [0, 0, 0, 0], dtype=torch.uint8, device="cuda")
    out = torch.zeros(max(m, 1), dtype=torch.int32, device="cuda")
    _check(load().pmklc_wnc_decode(_dptr(buf), len(padded), _dptr(c), V1 - 1, m, _dptr(out), _stream()),
           "pmklc_wnc_decode")
    return out[:m]


def model_trace(cfg: dict, tokens, steps=(), static=None, init=None, stop: int = 0, streams: bool = False):
    """Run one block's learning loop over ``tokens`` on the GPU; returns
    (P[len(steps), bs, V] float32, params[n+1] float32) as device tensors,
    plus the block's concatenated segment streams (bytes) if ``streams``."""
    torch = _torch()
    L = load()
    tok = _dev_tensor(tokens, torch.uint8)
    c, keep = make_config(cfg)
    n = int(L.pmklc_param_count(ctypes.byref(c)))
    V = 4 ** cfg["k"]
    st = np.ascontiguousarray(sorted(steps), dtype=np.uint64)
    P = torch.zeros((max(len(st), 1), cfg["bs"], V), dtype=torch.float32, device="cuda")
    params = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    sd = None if static is None else _dev_tensor(static, torch.float32)
    ini = None if init is None else _dev_tensor(init, torch.float32)
    buf = np.empty(4 * ((17 * (tok.numel() // cfg["bs"]) + 2 + 31) // 32 + 1) * cfg["bs"] + 16, dtype=np.uint8)
    slen = ctypes.c_uint64(0)
    _check(L.pmklc_model_trace(ctypes.byref(c), _dptr(tok), tok.numel(), _dptr(sd), _dptr(ini), stop,
                               st.ctypes.data_as(_u64p) if len(st) else None, len(st), _dptr(P), _dptr(params),
                               buf.ctypes.data_as(ctypes.c_void_p) if streams else None, buf.size if streams else 0,
                               ctypes.byref(slen) if streams else None, _stream()), "pmklc_model_trace")
    if streams:
        return P[:len(st)], params, buf[:slen.value].tobytes()
    return P[:len(st)], params


# ------------------------------------------------- differentiable DM op
def dm_forward(cfg: dict, params, ctx):
    """Logits [rows, V] of the dynamic model for contexts ctx [rows, t]."""
    torch = _torch()
    L = load()
    c, _ = make_config(cfg)
    p = _dev_tensor(params, torch.float32)
    x = _dev_tensor(ctx, torch.uint8)
    rows = x.shape[0]
    ws_b = ctypes.c_uint64(0)
    _check(L.pmklc_dm_workspace(ctypes.byref(c), rows, ctypes.byref(ws_b)), "pmklc_dm_workspace")
    ws = torch.empty(ws_b.value, dtype=torch.uint8, device="cuda")
    out = torch.empty((rows, 4 ** cfg["k"]), dtype=torch.float32, device="cuda")
    _check(L.pmklc_dm_forward(ctypes.byref(c), _dptr(p), _dptr(x), rows, _dptr(out), _dptr(ws), ws.numel(),
                              _stream()), "pmklc_dm_forward")
    return out


def dm_backward(cfg: dict, params, ctx, dlogits):
    """Gradient of sum(dlogits * logits) with respect to the flat parameters
    (activations recomputed by the kernel)."""
    torch = _torch()
    L = load()
    c, _ = make_config(cfg)
    p = _dev_tensor(params, torch.float32)
    x = _dev_tensor(ctx, torch.uint8)
    g = _dev_tensor(dlogits, torch.float32)
    rows = x.shape[0]
    ws_b = ctypes.c_uint64(0)
    _check(L.pmklc_dm_workspace(ctypes.byref(c), rows, ctypes.byref(ws_b)), "pmklc_dm_workspace")
    ws = torch.empty(ws_b.value, dtype=torch.uint8, device="cuda")
    grad = torch.zeros_like(p)
    _check(L.pmklc_dm_backward(ctypes.byref(c), _dptr(p), _dptr(x), rows, _dptr(g), _dptr(grad), _dptr(ws),
                               ws.numel(), _stream()), "pmklc_dm_backward")
    return grad
