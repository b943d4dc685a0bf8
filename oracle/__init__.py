"""PMKLC CPU oracle (FP64) — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-checkable C implementation of what the hot path
computes (``pmklc_oracle.c``), loaded with ctypes. Only ``tests/``, the
smoke check and the bench's CPU-baseline leg may import this package; the
GPU library neither links nor calls it.

Parity status per function (see the tests under ``tests/test_oracle_*``):
  encode_skmer  pinned: paper's worked example (Sec. 4.1) + brute force
  quantise      pinned: sum/positivity/monotonicity invariants, KL bound
  wnc_*         pinned: uniform-model closed form, code-length bounds,
                round trip, hand-computed bit strings
  step          pinned: torch FP64 autograd on the same graph + central FD
  opt_step      pinned: SGD / Adam closed forms
  compress      pinned: uniform closed form (2 bits/base at s = k), round
                trip, edge cases; the learned-model ratio on synthetic data
                is parity unpinned (the paper's datasets are unavailable)
  transformer   pinned: torch FP64 autograd with torch's own attention
                routine, finite differences, t = 1 and zero-key closed
                forms, learning-loop replay (SGD, Adam)
  BiGRU static  pinned: torch.nn.GRU (bidirectional, 1-2 layers, FP64) with
                the oracle's weights, zero-recurrence closed form, Eq. (1)
                mixing at the first learned step
  private model pinned: training block gathered from its definition and run
                through the pinned trace; coding pass equal to the public-
                model container with the stored weights; the selector's
                size rule at its boundary
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmklc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "invalid base", -3: "buffer too small", -4: "corrupt",
          -5: "model mismatch", -8: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"oracle {what}: {ERRORS.get(code, code)} ({code})")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP across blocks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)


class _Cfg(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("k", ctypes.c_int32), ("t", ctypes.c_int32), ("bs", ctypes.c_int32),
                ("E", ctypes.c_int32), ("nh", ctypes.c_int32), ("hidden", ctypes.c_int32 * 4),
                ("optimizer", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("selector", ctypes.c_int32),
                ("smp_ppm", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("n_blocks", ctypes.c_int32),
                ("block_len", _u64p), ("n_files", ctypes.c_int32), ("file_blocks", _u64p),
                ("init_override", _dp), ("ms_threshold", ctypes.c_uint64), ("arch", ctypes.c_int32),
                ("heads", ctypes.c_int32), ("static_arch", ctypes.c_int32), ("static_E", ctypes.c_int32),
                ("gru_h", ctypes.c_int32), ("gru_layers", ctypes.c_int32), ("dense", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = ctypes.CDLL(_LIB)
    L.or_skmer_count.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
    L.or_skmer_count.restype = ctypes.c_uint64
    L.or_encode_skmer.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _u8p, ctypes.c_uint64, _u64p]
    L.or_quantise.argtypes = [_dp, ctypes.c_int, _u32p]
    L.or_quantise.restype = None
    L.or_wnc_encode.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.POINTER(_u8p), _u64p]
    L.or_wnc_decode.argtypes = [_u8p, ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_uint64, _u32p]
    L.or_crc32.argtypes = [_u8p, ctypes.c_uint64]
    L.or_crc32.restype = ctypes.c_uint32
    L.or_param_count.argtypes = [ctypes.c_int] * 4 + [_i32p, ctypes.c_int, ctypes.c_int]
    L.or_param_count.restype = ctypes.c_uint64
    L.or_init_params.argtypes = [ctypes.c_int] * 4 + [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _dp]
    L.or_step.argtypes = [ctypes.c_int] * 4 + [_i32p, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double, _u8p,
                                                _u8p, ctypes.c_int, _dp, _dp, _dp, _dp]
    L.or_opt_step.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              _dp, _dp, _dp, _dp, ctypes.c_uint64, ctypes.c_uint64]
    L.or_opt_step.restype = None
    L.or_compress.argtypes = [ctypes.POINTER(_Cfg), _u8p, ctypes.c_uint64, _fp, ctypes.c_uint64,
                              ctypes.POINTER(_u8p), _u64p]
    L.or_decompress.argtypes = [_u8p, ctypes.c_uint64, _fp, ctypes.c_uint64, ctypes.POINTER(_u8p), _u64p]
    L.or_trace_block.argtypes = [ctypes.POINTER(_Cfg), _u8p, ctypes.c_uint64, _fp, _dp, ctypes.c_uint64, _u64p,
                                 ctypes.c_uint64, _dp, _dp, _dp]
    L.or_static_param_count.argtypes = [ctypes.POINTER(_Cfg)]
    L.or_static_param_count.restype = ctypes.c_uint64
    L.or_static_init.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_uint64, _dp]
    L.or_static_forward.argtypes = [ctypes.POINTER(_Cfg), _dp, _u8p, ctypes.c_int, _dp]
    L.or_static_step.argtypes = [ctypes.POINTER(_Cfg), _dp, _u8p, _u8p, ctypes.c_int, _dp, _dp,
                                 ctypes.POINTER(ctypes.c_double)]
    L.or_free.argtypes = [ctypes.c_void_p]
    L.or_free.restype = None
    L.or_num_threads.restype = ctypes.c_int
    _lib = L
    return L


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def num_threads() -> int:
    return _load().or_num_threads()


# --------------------------------------------------------------------- GskE
def skmer_count(n: int, s: int, k: int) -> int:
    return int(_load().or_skmer_count(n, s, k))


def encode_skmer(ascii_bases, s: int, k: int) -> np.ndarray:
    if isinstance(ascii_bases, str):
        ascii_bases = ascii_bases.encode()
    if isinstance(ascii_bases, (bytes, bytearray)):
        a = np.frombuffer(bytes(ascii_bases), dtype=np.uint8).copy()
    else:
        a = np.ascontiguousarray(ascii_bases, dtype=np.uint8)
    if a.size == 0:
        a = np.zeros(0, dtype=np.uint8)
    cap = max(1, skmer_count(len(a), s, k))
    out = np.zeros(cap, dtype=np.uint8)
    nt = ctypes.c_uint64(0)
    src = a if a.size else np.zeros(1, dtype=np.uint8)
    _check(_load().or_encode_skmer(_ptr(src, _u8p), len(a), s, k, _ptr(out, _u8p), cap, ctypes.byref(nt)),
           "encode_skmer")
    return out[:nt.value]


# ---------------------------------------------------------------- quantiser
def quantise(P) -> np.ndarray:
    """P: [rows, V] probabilities (float64 or float32, taken exactly) ->
    integer CDF [rows, V+1] with total 2^16."""
    P = np.ascontiguousarray(np.atleast_2d(P), dtype=np.float64)
    rows, V = P.shape
    out = np.zeros((rows, V + 1), dtype=np.uint32)
    L = _load()
    for r in range(rows):
        L.or_quantise(_ptr(P[r], _dp), V, _ptr(out[r], _u32p))
    return out


# -------------------------------------------------------------------- coder
def wnc_encode(cum_lo, cum_hi) -> tuple[bytes, int]:
    lo = np.ascontiguousarray(cum_lo, dtype=np.uint32)
    hi = np.ascontiguousarray(cum_hi, dtype=np.uint32)
    out = _u8p()
    nbits = ctypes.c_uint64(0)
    L = _load()
    _check(L.or_wnc_encode(_ptr(lo, _u32p), _ptr(hi, _u32p), len(lo), ctypes.byref(out), ctypes.byref(nbits)),
           "wnc_encode")
    nb = (nbits.value + 7) // 8
    data = ctypes.string_at(out, nb) if nb else b""
    L.or_free(out)
    return data, int(nbits.value)


def wnc_decode(data: bytes, cdfs) -> np.ndarray:
    c = np.ascontiguousarray(np.atleast_2d(cdfs), dtype=np.uint32)
    m, V1 = c.shape
    buf = np.frombuffer(data, dtype=np.uint8).copy() if data else np.zeros(1, dtype=np.uint8)
    out = np.zeros(m, dtype=np.uint32)
    _check(_load().or_wnc_decode(_ptr(buf, _u8p), len(data), _ptr(c, _u32p), V1 - 1, m, _ptr(out, _u32p)),
           "wnc_decode")
    return out


def crc32(data) -> int:
    a = np.frombuffer(bytes(data), dtype=np.uint8).copy() if not isinstance(data, np.ndarray) else \
        np.ascontiguousarray(data).view(np.uint8).reshape(-1)
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint8)
        return int(_load().or_crc32(_ptr(a, _u8p), 0))
    return int(_load().or_crc32(_ptr(a, _u8p), a.size))


# -------------------------------------------------------------------- model
def _hidden(cfg):
    h = list(cfg["hidden"])
    arr = np.zeros(4, dtype=np.int32)
    arr[:len(h)] = h
    return arr, len(h)


ARCHS = {"mlp": 0, "transformer": 1}


def _arch(cfg):
    """(arch code, heads) of a configuration: "mlp" (default) or
    "transformer" (hidden = [A, F], heads)."""
    a = ARCHS[cfg.get("arch", "mlp")]
    return a, int(cfg.get("heads", 0)) if a == 1 else 0


def param_count(cfg) -> int:
    h, nh = _hidden(cfg)
    return int(_load().or_param_count(cfg["k"], cfg["t"], cfg["E"], nh, _ptr(h, _i32p), *_arch(cfg)))


def init_params(cfg, seed=None) -> np.ndarray:
    h, nh = _hidden(cfg)
    n = param_count(cfg)
    w = np.zeros(n, dtype=np.float64)
    _check(_load().or_init_params(cfg["k"], cfg["t"], cfg["E"], nh, _ptr(h, _i32p), *_arch(cfg),
                                  cfg["seed"] if seed is None else seed, _ptr(w, _dp)), "init_params")
    return w


def param_slices(cfg) -> dict:
    """Offsets of each tensor in the flat parameter vector."""
    V = 4 ** cfg["k"]
    if _arch(cfg)[0] == 1:
        E, t, (A, F) = cfg["E"], cfg["t"], cfg["hidden"]
        out, off = {}, 0
        for name, shp in [("emb", (V, E)), ("pos", (t, E)), ("Wqkv", (E, 3 * A)), ("bqkv", (3 * A,)),
                          ("Wo", (A, A)), ("bo", (A,)), ("W1", (A, F)), ("b1", (F,)), ("W2", (F, A)),
                          ("b2", (A,)), ("Wh", (A, V)), ("bh", (V,))]:
            out[name] = (off, shp)
            off += int(np.prod(shp))
        return out
    dims = [cfg["t"] * cfg["E"]] + list(cfg["hidden"]) + [V]
    off = 0
    out = {"emb": (off, (V, cfg["E"]))}
    off += V * cfg["E"]
    for l in range(len(dims) - 1):
        out[f"W{l}"] = (off, (dims[l], dims[l + 1]))
        off += dims[l] * dims[l + 1]
        out[f"b{l}"] = (off, (dims[l + 1],))
        off += dims[l + 1]
    return out


def step(cfg, w, ctx, tgt, ws=None, a_alpha=0.0, grad=True):
    """One learning step over bs rows. Returns (P, grad, g_alpha, loss)."""
    h, nh = _hidden(cfg)
    V = 4 ** cfg["k"]
    ctx = np.ascontiguousarray(ctx, dtype=np.uint8)
    tgt = np.ascontiguousarray(tgt, dtype=np.uint8)
    bs = ctx.shape[0]
    w = np.ascontiguousarray(w, dtype=np.float64)
    ws = None if ws is None else np.ascontiguousarray(ws, dtype=np.float64)
    P = np.zeros((bs, V), dtype=np.float64)
    g = np.zeros_like(w) if grad else None
    ga = ctypes.c_double(0)
    loss = ctypes.c_double(0)
    _check(_load().or_step(cfg["k"], cfg["t"], cfg["E"], nh, _ptr(h, _i32p), *_arch(cfg), _ptr(w, _dp), _ptr(ws, _dp),
                           float(a_alpha), _ptr(ctx, _u8p), _ptr(tgt, _u8p), bs, _ptr(P, _dp), _ptr(g, _dp),
                           ctypes.byref(ga), ctypes.byref(loss)), "step")
    return P, g, ga.value, loss.value


def opt_step(kind, lr, b1, b2, eps, w, g, m, v, tau):
    for a in (w, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().or_opt_step(kind, lr, b1, b2, eps, _ptr(w, _dp), _ptr(g, _dp), _ptr(m, _dp), _ptr(v, _dp), len(w), tau)


# ----------------------------------------------------------------- pipeline
def _mkcfg(cfg, n):
    h, nh = _hidden(cfg)
    c = _Cfg()
    c.s, c.k, c.t, c.bs, c.E, c.nh = cfg["s"], cfg["k"], cfg["t"], cfg["bs"], cfg["E"], nh
    for i in range(4):
        c.hidden[i] = int(h[i])
    c.optimizer = 1 if cfg.get("optimizer", "sgd") == "adam" else 0
    c.lr, c.beta1, c.beta2, c.eps = cfg.get("lr", 1e-3), cfg.get("beta1", 0.9), cfg.get("beta2", 0.999), \
        cfg.get("eps", 1e-8)
    sel = cfg.get("selector", "dm")
    c.selector = {"uniform": 0, "dm": 4, "spum_dm": 5, "sprm_dm": 6, "spum_sprm_dm": 7, "auto": 8}[sel]
    c.ms_threshold = int(cfg.get("ms_threshold", 0))
    c.arch, c.heads = _arch(cfg)
    if cfg.get("static_arch", "mlp") == "bigru":
        c.static_arch = 1
        c.static_E, c.gru_h = int(cfg.get("static_E", 16)), int(cfg.get("gru_h", 32))
        c.gru_layers, c.dense = int(cfg.get("gru_layers", 2)), int(cfg.get("dense", 128))
    c.smp_ppm = int(cfg.get("smp_ppm", 0))
    c.seed = int(cfg["seed"])
    keep = []
    bl = cfg.get("block_len")
    if bl is not None:
        arr = np.ascontiguousarray(bl, dtype=np.uint64)
        keep.append(arr)
        c.n_blocks = len(arr)
        c.block_len = _ptr(arr, _u64p)
    else:
        c.n_blocks = int(cfg.get("n_blocks", 1))
    fb = cfg.get("file_blocks")
    if fb is not None:
        arr = np.ascontiguousarray(fb, dtype=np.uint64)
        keep.append(arr)
        c.n_files = len(arr)
        c.file_blocks = _ptr(arr, _u64p)
    else:
        c.n_files = 1
    ini = cfg.get("init_override")
    if ini is not None:
        arr = np.ascontiguousarray(ini, dtype=np.float64)
        keep.append(arr)
        c.init_override = _ptr(arr, _dp)
    return c, keep


def static_param_count(cfg) -> int:
    """Parameters of the static public model (the DM's MLP shape, or the
    BiGRU of static_arch "bigru")."""
    c, keep = _mkcfg(cfg, 0)
    return int(_load().or_static_param_count(ctypes.byref(c)))


def static_init(cfg, seed) -> np.ndarray:
    c, keep = _mkcfg(cfg, 0)
    w = np.zeros(static_param_count(cfg), dtype=np.float64)
    _check(_load().or_static_init(ctypes.byref(c), seed, _ptr(w, _dp)), "static_init")
    return w


def static_forward(cfg, ws, ctx) -> np.ndarray:
    """Logits L^u [rows, V] of the static public model for contexts [rows, t]."""
    c, keep = _mkcfg(cfg, 0)
    ctx = np.ascontiguousarray(ctx, dtype=np.uint8)
    ws = np.ascontiguousarray(ws, dtype=np.float64)
    out = np.zeros((ctx.shape[0], 4 ** cfg["k"]), dtype=np.float64)
    _check(_load().or_static_forward(ctypes.byref(c), _ptr(ws, _dp), _ptr(ctx, _u8p), ctx.shape[0], _ptr(out, _dp)),
           "static_forward")
    return out


def static_step(cfg, ws, ctx, tgt):
    """(P [rows, V], gradient, loss) of one learning step of the static
    model alone (its private-model training step)."""
    c, keep = _mkcfg(cfg, 0)
    ctx = np.ascontiguousarray(ctx, dtype=np.uint8)
    tgt = np.ascontiguousarray(tgt, dtype=np.uint8)
    ws = np.ascontiguousarray(ws, dtype=np.float64)
    rows, V = ctx.shape[0], 4 ** cfg["k"]
    P = np.zeros((rows, V), dtype=np.float64)
    g = np.zeros(ws.size, dtype=np.float64)
    loss = ctypes.c_double(0.0)
    _check(_load().or_static_step(ctypes.byref(c), _ptr(ws, _dp), _ptr(ctx, _u8p), _ptr(tgt, _u8p), rows,
                                  _ptr(P, _dp), _ptr(g, _dp), ctypes.byref(loss)), "static_step")
    return P, g, loss.value


def _static_arg(static):
    if static is None:
        return None, 0
    s = np.ascontiguousarray(static, dtype=np.float32)
    return s, s.size


def compress(cfg, data, static=None) -> bytes:
    a = np.ascontiguousarray(data, dtype=np.uint8)
    c, keep = _mkcfg(cfg, len(a))
    s, sl = _static_arg(static)
    out = _u8p()
    olen = ctypes.c_uint64(0)
    buf = a if a.size else np.zeros(1, dtype=np.uint8)
    L = _load()
    _check(L.or_compress(ctypes.byref(c), _ptr(buf, _u8p), a.size, _ptr(s, _fp), sl, ctypes.byref(out),
                         ctypes.byref(olen)), "compress")
    res = ctypes.string_at(out, olen.value)
    L.or_free(out)
    return res


def decompress(blob: bytes, static=None) -> np.ndarray:
    b = np.frombuffer(blob, dtype=np.uint8).copy()
    s, sl = _static_arg(static)
    out = _u8p()
    olen = ctypes.c_uint64(0)
    L = _load()
    _check(L.or_decompress(_ptr(b, _u8p), b.size, _ptr(s, _fp), sl, ctypes.byref(out), ctypes.byref(olen)),
           "decompress")
    res = np.frombuffer(ctypes.string_at(out, olen.value), dtype=np.uint8).copy() if olen.value else \
        np.zeros(0, dtype=np.uint8)
    L.or_free(out)
    return res


def trace_block(cfg, tokens, steps=(), static=None, init=None, stop=0):
    """Run the compression loop of one block of ``tokens`` (all L steps, or
    the first ``stop``); returns (P[len(steps), bs, V], loss[L],
    w[n+1] after the last step run)."""
    tok = np.ascontiguousarray(tokens, dtype=np.uint8)
    c, keep = _mkcfg(cfg, len(tok))
    s, sl = _static_arg(static)
    V = 4 ** cfg["k"]
    bs = cfg["bs"]
    L_steps = len(tok) // bs
    st = np.ascontiguousarray(sorted(steps), dtype=np.uint64)
    P = np.zeros((max(1, len(st)), bs, V), dtype=np.float64)
    loss = np.zeros(max(1, L_steps), dtype=np.float64)
    n = param_count(cfg)
    wf = np.zeros(n + 1, dtype=np.float64)
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.float64)
    _check(_load().or_trace_block(ctypes.byref(c), _ptr(tok, _u8p), len(tok), _ptr(s, _fp), _ptr(ini, _dp),
                                  int(stop), _ptr(st, _u64p) if len(st) else None, len(st), _ptr(P, _dp), _ptr(loss, _dp),
                                  _ptr(wf, _dp)), "trace_block")
    return P[:len(st)], loss[:L_steps], wf
