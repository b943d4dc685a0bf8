"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bit-exact: (s,k)-mer tokens, integer CDFs given identical FP32
probabilities, coded bytes given identical CDF streams, the whole container
under the uniform model, GPU-alone round trips, determinism across launch
schedules. Tolerances: per-symbol probabilities within 1e-4 of the FP64
oracle for the FP32 path (teacher-forced at identical weights, and along a
whole block's trajectory); compression ratio within 0.5% of the oracle's.
"""
import math
import os

import numpy as np
import pytest

import synth
from synth.workloads import model_small
from tests import cbf

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAIRS = [(s, k) for k in range(1, 5) for s in range(1, k + 1)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_12805_amd as P
    P.load()
    return P


def _dna(n, seed=0, order=3, n_rate=0.0, rho=0.0):
    return synth.generate(synth.Recipe(n=n, order=order, seed=seed, n_rate=n_rate, n_max=30, rho=rho))


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------------------------------ GskE
@pytest.mark.parametrize("s,k", PAIRS)
def test_skmer_matches_oracle(gpu, orc, s, k):
    for n in [0, 1, 3, 4, 5, 17, 1023, 4097, 100003]:
        a = _dna(n, seed=n + 7 * k + s)
        got = gpu.encode_skmer(_cuda(a), s, k).cpu().numpy()
        assert np.array_equal(got, orc.encode_skmer(a, s, k)), (s, k, n)


def test_skmer_unaligned_input_and_errors(gpu, orc):
    a = _dna(20000, seed=3)
    x = _cuda(a)
    for off in [1, 2, 3]:
        got = gpu.encode_skmer(x[off:], 3, 3).cpu().numpy()
        assert np.array_equal(got, orc.encode_skmer(a[off:], 3, 3))
    bad = a.copy()
    bad[12345] = ord("N")
    with pytest.raises(gpu.PmklcError) as e:
        gpu.encode_skmer(_cuda(bad), 3, 3)
    assert e.value.code == -2
    bad[12345] = ord("a")
    with pytest.raises(gpu.PmklcError):
        gpu.encode_skmer(_cuda(bad), 1, 1)
    with pytest.raises(gpu.PmklcError) as e:
        gpu.encode_skmer(x, 4, 3)
    assert e.value.code == -1


def test_skmer_table8_size_sampled(gpu, orc):
    """The (s,k) sweep input size of the paper's Table 8 (554,197,554 bases):
    every (s,k) pair on the full sequence, checked on sampled windows."""
    n = 554_197_554
    a = synth.generate(synth.recipe_cfg1(seed=8, n=n))
    x = _cuda(a)
    rng = np.random.default_rng(0)
    for s, k in PAIRS:
        tok = gpu.encode_skmer(x, s, k)
        l = (n - k) // s + 1
        assert tok.numel() == l
        idx = np.sort(rng.integers(0, l, size=2000))
        idx[-1] = l - 1
        got = tok[_cuda(idx.astype(np.int64))].cpu().numpy()
        want = np.array([orc.encode_skmer(a[j * s:j * s + k], s, k)[0] for j in idx])
        assert np.array_equal(got, want), (s, k)
        del tok


# ----------------------------------------------------- quantiser, coder
@pytest.mark.parametrize("V", [4, 16, 64, 256])
def test_quantiser_bit_exact(gpu, orc, V):
    rng = np.random.default_rng(V)
    P = rng.dirichlet([0.1] * V, size=3000).astype(np.float32)
    P[0] = 0.0
    P[0, 5 % V] = 1.0
    P[1] = np.float32(1.0 / V)
    # products p * (2^16 - V) at and next to integers: the FP32 floor's
    # residual test decides these (row sums stay <= 1, so the residual is >= 0)
    c = 65536 - V
    n = rng.integers(0, c // V, size=(200, V))
    near = (n / c).astype(np.float32)
    P[2:202] = near
    P[202:402] = np.nextafter(near, np.float32(0))
    P[402:602] = np.nextafter(near, np.float32(1))
    P[602:702] = np.float32(0.9 / V)                    # all ties: lowest index takes the residual
    got = gpu.quantise(_cuda(P)).cpu().numpy().astype(np.uint32)
    want = orc.quantise(P.astype(np.float64))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("V,skew", [(4, 0.5), (64, 0.05), (256, 0.2)])
def test_coder_bytes_bit_exact(gpu, orc, V, skew):
    rng = np.random.default_rng(11 * V)
    m = 5000
    P = rng.dirichlet([skew] * V, size=m)
    cdf = orc.quantise(P)
    sym = np.array([rng.choice(V, p=P[i]) for i in range(m)])
    lo, hi = cdf[np.arange(m), sym], cdf[np.arange(m), sym + 1]
    data_g, nb_g = gpu.wnc_encode(lo, hi)
    data_o, nb_o = orc.wnc_encode(lo, hi)
    assert nb_g == nb_o and data_g == data_o
    dec = gpu.wnc_decode(data_g, cdf).cpu().numpy()
    assert np.array_equal(dec, sym)


# --------------------------------------------------------- containers
def _tiny(**kw):
    c = model_small(t=4, E=4, hidden=[8], bs=8)
    c.update(kw)
    return c


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_uniform_container_bit_exact_with_oracle(gpu, orc, k):
    a = _dna(50003, seed=k, n_rate=0.001)
    cfg = _tiny(s=k, k=k, selector="uniform", n_blocks=5)
    blob_g = gpu.compress(cfg, _cuda(a))
    blob_o = orc.compress(cfg, a)
    assert blob_g == blob_o
    assert np.array_equal(gpu.decompress(blob_g).cpu().numpy(), a)


@pytest.mark.parametrize("s,k", [(s, k) for (s, k) in PAIRS if s < k])
def test_uniform_container_bit_exact_overlapping_kmers(gpu, orc, s, k):
    """Overlapping (s,k)-mers (s < k) through pmklc_compress's own scan and
    tokeniser: under the uniform model the container equals the oracle's
    byte for byte (N runs, tails, remainder tokens and every stream)."""
    a = _dna(40009 + s, seed=10 * k + s, n_rate=0.001)
    cfg = _tiny(s=s, k=k, selector="uniform", n_blocks=3)
    blob_g = gpu.compress(cfg, _cuda(a))
    assert blob_g == orc.compress(cfg, a)
    assert np.array_equal(gpu.decompress(blob_g).cpu().numpy(), a)


ROUNDTRIP = {
    "cfg1": (dict(), 1 << 18, 1, 0.0),
    "tiny_multi_N": (dict(t=4, E=4, hidden=[8], bs=8, n_blocks=3), 30011, 1, 0.003),
    "s1k3_static": (dict(s=1, k=3, t=8, E=4, hidden=[16], bs=16, selector="spum_dm", n_blocks=2), 20000, 2, 0.001),
    "two_hidden_adam": (dict(t=6, E=8, hidden=[16, 12], bs=8, optimizer="adam", n_blocks=2), 24000, 3, 0.0),
    "s2k3": (dict(s=2, k=3, t=5, E=4, hidden=[8], bs=12), 9001, 4, 0.0),
    "k4": (dict(s=4, k=4, t=3, E=4, hidden=[8], bs=4), 8000, 5, 0.0),
}


@pytest.mark.parametrize("name", list(ROUNDTRIP))
def test_gpu_roundtrip_and_ratio(gpu, orc, name):
    kw, n, seed, nrate = ROUNDTRIP[name]
    cfg = model_small(**kw)
    a = _dna(n, seed=seed, n_rate=nrate, rho=0.05)
    static = None
    if cfg["selector"] == "spum_dm":
        static = orc.init_params(cfg, seed=123).astype(np.float32)
    blob = gpu.compress(cfg, _cuda(a), static=static)
    back = gpu.decompress(blob, static=static).cpu().numpy()
    assert np.array_equal(back, a)
    assert gpu.compress(cfg, _cuda(a), static=static) == blob          # deterministic
    blob_o = orc.compress(cfg, a, static=static)
    assert len(blob) == pytest.approx(len(blob_o), rel=0.005, abs=2)
    pg, po = cbf.parse(blob), cbf.parse(blob_o)
    assert pg["header"]["path"] in (1, 3) and po["header"]["path"] == 0
    for bg, bo in zip(pg["blocks"], po["blocks"]):     # identical metadata
        assert (bg["raw_len"], bg["runs"], bg["extras"]) == (bo["raw_len"], bo["runs"], bo["extras"])


def test_plain_and_batched_schedules_give_identical_bytes(gpu):
    a = _dna(40000, seed=9)
    cfg = _tiny(n_blocks=4)
    b1 = gpu.compress(dict(cfg, schedule="batched"), _cuda(a))
    b2 = gpu.compress(dict(cfg, schedule="plain"), _cuda(a))
    assert b1 == b2


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp32_valu"])
@pytest.mark.parametrize("hidden", [32, 64])
def test_autotuner_choices_give_identical_bytes(gpu, precision, hidden, monkeypatch):
    """Every launch shape the autotuner may pick yields the same container:
    both workgroup widths, and for the global-weight matrix-core kernel at
    a hidden width of 64 both F1 units (four or two hidden tiles per unit);
    the on-chip kernel has one shape."""
    monkeypatch.setenv("PMKLC_NO_CHIP", "1")
    a = _dna(60000, seed=21, n_rate=0.001)
    cfg = model_small(n_blocks=3, precision=precision, hidden=[hidden])
    mfma = precision != "fp32_valu"
    f1s = ["4", "2"] if mfma and hidden % 64 == 0 else [None]
    blobs = []
    for nt in ["256", "512"]:
        for f1 in f1s:
            monkeypatch.setenv("PMKLC_NT", nt)
            if f1:
                monkeypatch.setenv("PMKLC_F1", f1)
            blobs.append(gpu.compress(cfg, _cuda(a)))
            tm = gpu.last_timing()
            assert tm["threads"] == int(nt)
            assert tm["f1_units"] == (int(f1) if f1 else (2 if mfma else 0))
    monkeypatch.delenv("PMKLC_NT")
    monkeypatch.delenv("PMKLC_F1", raising=False)
    blobs.append(gpu.compress(cfg, _cuda(a)))          # the autotuner's own choice
    print(f"{precision} hidden {hidden}: chose {gpu.last_timing()['threads']} threads, "
          f"F1 units of {gpu.last_timing()['f1_units']}")
    assert all(b == blobs[0] for b in blobs)
    assert np.array_equal(gpu.decompress(blobs[0]).cpu().numpy(), a)


def test_smp_chain_roundtrip_and_snapshot(gpu, orc):
    a = _dna(30000, seed=10, n_rate=0.001)
    cfg = _tiny(block_len=[5000, 7000, 3000, 9000, 6000], file_blocks=[3, 2], smp_ppm=50000)
    blob = gpu.compress(cfg, _cuda(a))
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    blob_o = orc.compress(cfg, a)
    assert len(blob) == pytest.approx(len(blob_o), rel=0.005)
    assert blob != gpu.compress(dict(cfg, smp_ppm=0), _cuda(a))


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp32_valu", "bf16_global"])
def test_smp_snapshot_bit_exact(gpu, orc, precision, monkeypatch):
    """Model passing (Sec. 4.3): the second block of a file starts from the
    first block's parameters after ceil(5% of its steps) steps. Its segment
    streams in the chained container equal, byte for byte, those of a
    single-block run over its tokens started from the parameters the first
    block's own run reaches at that step, and differ from a start one step
    later; the first block's streams equal its seeded single-block run.
    (BF16 on the on-chip kernel, which writes its parameters back for the
    snapshot, and on the global-weight kernel.)"""
    if precision == "bf16_global":
        monkeypatch.setenv("PMKLC_NO_CHIP", "1")
        precision = "bf16"
    cfg = model_small(precision=precision)
    bs, t = cfg["bs"], cfg["t"]
    L0, L1 = 800, 300
    n0, n1 = 3 * bs * L0, 3 * bs * L1 + 5        # (3,3)-mers: l = (n - 3) // 3 + 1 tokens
    a = _dna(n0 + n1, seed=12, rho=0.05)
    chain = dict(cfg, block_len=[n0, n1], file_blocks=[2], smp_ppm=50000)
    blob = gpu.compress(chain, _cuda(a))
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    p = cbf.parse(blob)
    assert [b["L"] for b in p["blocks"]] == [L0, L1]
    S = -(-50000 * L0 // 1000000)                 # ceil(5% of the first block's steps)
    assert S > t                                  # the snapshot carries learned weights
    tok0 = orc.encode_skmer(a[:n0], 3, 3)
    tok1 = orc.encode_skmer(a[n0:], 3, 3)
    _, _, s0 = gpu.model_trace(cfg, tok0, streams=True)
    assert s0 == b"".join(p["blocks"][0]["streams"])
    _, wS = gpu.model_trace(cfg, tok0, stop=S)
    _, _, s1 = gpu.model_trace(cfg, tok1, init=wS, streams=True)
    assert s1 == b"".join(p["blocks"][1]["streams"])
    _, wS1 = gpu.model_trace(cfg, tok0, stop=S + 1)
    _, _, s1b = gpu.model_trace(cfg, tok1, init=wS1, streams=True)
    assert s1b != s1


@pytest.mark.parametrize("raw", ["", "A", "AC", "ACG", "N" * 40, "ANNNNNC", "ACGT" * 9, "NACGTN" * 30])
def test_edge_cases(gpu, orc, raw):
    a = np.frombuffer(raw.encode(), dtype=np.uint8).copy()
    for nblk in [1, 3]:
        cfg = _tiny(n_blocks=nblk)
        blob = gpu.compress(cfg, _cuda(a) if len(a) else np.zeros(0, np.uint8))
        assert np.array_equal(gpu.decompress(blob).cpu().numpy()[:len(a)], a)
        pg, po = cbf.parse(blob), cbf.parse(orc.compress(cfg, a))
        for bg, bo in zip(pg["blocks"], po["blocks"]):
            assert (bg["raw_len"], bg["runs"], bg["extras"], bg["L"]) == (bo["raw_len"], bo["runs"], bo["extras"],
                                                                          bo["L"])
            if bg["L"] <= cfg["t"]:      # only uniform steps: identical streams
                assert bg["streams"] == bo["streams"]


def test_errors(gpu):
    cfg = _tiny()
    with pytest.raises(gpu.PmklcError) as e:
        gpu.compress(cfg, _cuda(np.frombuffer(b"ACGTACGTXACGT", dtype=np.uint8).copy()))
    assert e.value.code == -2
    a = _dna(5000, seed=1)
    blob = gpu.compress(cfg, _cuda(a))
    for bad in [blob[:50], blob[:-2], b"QQQQ" + blob[4:]]:
        with pytest.raises(gpu.PmklcError) as e:
            gpu.decompress(bad)
        assert e.value.code in (-4, -5)
    cs = _tiny(selector="spum_dm")
    st = np.random.default_rng(0).normal(0, 0.1, gpu.param_count(cs)).astype(np.float32)
    b2 = gpu.compress(cs, _cuda(a), static=st)
    wrong = st.copy()
    wrong[3] += 1
    with pytest.raises(gpu.PmklcError) as e:
        gpu.decompress(b2, static=wrong)
    assert e.value.code == -5


# ------------------------------------------------- probability parity
@pytest.mark.parametrize("precision", ["fp32", "fp32_valu"])
def test_teacher_forced_probabilities_and_gradient(gpu, orc, precision):
    """At identical weights the GPU's FP32 step (matrix-core and per-thread
    FMA kernels) gives P within 1e-4 of the FP64 oracle, and its SGD update
    matches w - lr * grad_oracle."""
    rec, cfg = synth.recipe_cfg1(), model_small(precision=precision)
    a = synth.generate(rec)
    tok = orc.encode_skmer(a, 3, 3)
    L = len(tok) // cfg["bs"]
    for i in [cfg["t"], cfg["t"] + 1, L // 2, L - 1]:
        _, w_i = gpu.model_trace(cfg, tok, stop=i)
        P_i, w_i1 = gpu.model_trace(cfg, tok, steps=[i], stop=i + 1)
        w64 = w_i.cpu().numpy().astype(np.float64)
        n = len(w64) - 1
        rows = np.arange(cfg["bs"]) * L + i
        ctx = np.stack([tok[r - cfg["t"]:r] for r in rows])
        Po, g, _, _ = orc.step(cfg, w64[:n], ctx, tok[rows])
        assert np.max(np.abs(P_i[0].cpu().numpy() - Po)) <= 1e-4
        expect = w64[:n] - cfg["lr"] * g
        assert np.max(np.abs(w_i1.cpu().numpy()[:n] - expect)) <= 1e-6


@pytest.mark.parametrize("precision", ["fp32", "fp32_valu"])
def test_trajectory_probabilities_cfg1(gpu, orc, precision):
    """Whole-block trajectory of the first workload (256 KiB, one block):
    sampled steps' P within 1e-4 of the FP64 oracle, code ratio within 0.5%."""
    rec, cfg = synth.recipe_cfg1(), model_small(precision=precision)
    a = synth.generate(rec)
    tok = orc.encode_skmer(a, 3, 3)
    L = len(tok) // cfg["bs"]
    steps = [0, cfg["t"], cfg["t"] + 5, 100, L // 2, L - 2, L - 1]
    Pg, wg = gpu.model_trace(cfg, tok, steps=steps)
    Po, _, wo = orc.trace_block(cfg, tok, steps=steps)
    d = np.abs(Pg.cpu().numpy() - Po)
    assert d.max() <= 1e-4, d.max()
    assert np.max(np.abs(wg.cpu().numpy() - wo)) <= 1e-4
    blob_g = gpu.compress(cfg, _cuda(a))
    blob_o = orc.compress(cfg, a)
    assert abs(len(blob_g) - len(blob_o)) <= 0.005 * len(blob_o)


@pytest.mark.parametrize("precision,path,path2,nochip", [("fp32", 3, 3, "0"), ("fp32_valu", 1, 1, "0"),
                                                          ("bf16", 4, 2, "0"), ("bf16", 2, 2, "1")])
def test_numeric_paths_roundtrip_and_ratio(gpu, orc, precision, path, path2, nochip, monkeypatch):
    """Every numeric path: bit-exact GPU round trip, identical bytes from
    both launch schedules, ratio within 0.5% of the FP64 oracle on the first
    workload (path) and on a 1 MiB sample of the static + dynamic workload
    (path2). BF16 runs the on-chip kernel (path 4) where it has the shape,
    or, with PMKLC_NO_CHIP=1, the global-weight kernel (path 2). BF16
    probabilities are reported (|dp| statistics), not held to 1e-4."""
    from synth.workloads import cfg2
    monkeypatch.setenv("PMKLC_NO_CHIP", nochip)
    static = np.fromfile(os.path.join(GOLD, "static_cfg2.f32"), dtype=np.float32)
    rec2, c2 = cfg2(n=1 << 20, n_blocks=16)
    cases = [(synth.generate(synth.recipe_cfg1()), model_small(), None, path),
             (synth.generate(rec2), c2, static, path2)]
    for a, cfg, st, pid in cases:
        cfg = dict(cfg, precision=precision)
        blob = gpu.compress(cfg, _cuda(a), static=st)
        assert blob[5] == pid
        assert np.array_equal(gpu.decompress(blob, static=st).cpu().numpy(), a)
        assert gpu.compress(dict(cfg, schedule="plain"), _cuda(a), static=st) == blob
        blob_o = orc.compress(cfg, a, static=st)
        rel = len(blob) / len(blob_o) - 1
        print(f"{precision}: {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
        assert abs(rel) <= 0.005
    rec, cfg = synth.recipe_cfg1(), model_small(precision=precision)
    tok = orc.encode_skmer(synth.generate(rec), 3, 3)
    L = len(tok) // cfg["bs"]
    steps = [cfg["t"], 200, L - 1]
    Pg, _ = gpu.model_trace(cfg, tok, steps=steps)
    Po, _, _ = orc.trace_block(cfg, tok, steps=steps)
    dp = np.abs(Pg.cpu().numpy() - Po)
    print(f"{precision}: |dp| max {dp.max():.3g} mean {dp.mean():.3g}")
    assert dp.max() <= (1e-4 if precision != "bf16" else 0.05)


# matrix-core shapes beyond the two workloads: 256 symbols with E 8 and 32 rows
# (B2 takes more symbol tiles than row tiles; a 16-wide tile of inputs spans two
# context positions), E 24 with 96 rows and H 96 (partial 4-tile F1 units and
# hidden chunks), 128 rows with Adam
MFMA_SHAPES = {
    "k4_E8_bs32_H64": dict(s=2, k=4, t=32, E=8, hidden=[64], bs=32),
    "E24_bs96_H96_t16": dict(s=3, k=3, t=16, E=24, hidden=[96], bs=96),
    "bs128_adam": dict(s=3, k=3, t=32, E=16, hidden=[32], bs=128, optimizer="adam", lr=3e-3),
}


@pytest.mark.parametrize("precision,path", [("bf16", 2), ("fp32", 3)])
@pytest.mark.parametrize("name", sorted(MFMA_SHAPES))
def test_mfma_shapes_roundtrip_ratio_probabilities(gpu, orc, name, precision, path):
    """Bit-exact round trip on the matrix-core path (container path id) and
    ratio within 0.5% of the FP64 oracle.  On the FP32 matrix-core path:
    with SGD, probabilities within 1e-4 of the oracle along the whole
    trajectory; with Adam, whose update lr m/(sqrt(v)+eps) turns a rounding-
    level gradient into a full lr step, the trajectory is compared over its
    first steps, probabilities at the GPU's own late weights against the
    oracle's at the same weights, and the first Adam update against the
    oracle's optimiser step wherever the gradient is not rounding-level."""
    cfg = model_small(**MFMA_SHAPES[name], precision=precision)
    rec = synth.recipe_cfg1(seed=31, n=1 << 16)
    a = synth.generate(rec)
    blob = gpu.compress(cfg, _cuda(a))
    assert blob[5] == path
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    blob_o = orc.compress(cfg, a)
    rel = len(blob) / len(blob_o) - 1
    print(f"{name} {precision}: {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
    assert abs(rel) <= 0.005
    if precision != "fp32":
        return
    tok = orc.encode_skmer(a, cfg["s"], cfg["k"])
    L, t, bs = len(tok) // cfg["bs"], cfg["t"], cfg["bs"]
    adam = cfg.get("optimizer") == "adam"
    steps = [t, t + 3] if adam else [t, (t + L) // 2, L - 1]
    Pg, _ = gpu.model_trace(cfg, tok, steps=steps)
    Po, _, _ = orc.trace_block(cfg, tok, steps=steps)
    print(f"trajectory |dp| max {np.abs(Pg.cpu().numpy() - Po).max():.3g}")
    assert np.abs(Pg.cpu().numpy() - Po).max() <= 1e-4
    if not adam:
        return

    def oracle_at(i, w64):
        rows = np.arange(bs) * L + i
        ctx = np.stack([tok[r - t:r] for r in rows])
        return orc.step(cfg, w64, ctx, tok[rows])

    n = orc.param_count(cfg)
    for i in [(t + L) // 2, L - 1]:                    # teacher-forced, late
        _, w_i = gpu.model_trace(cfg, tok, stop=i)
        P_i, _ = gpu.model_trace(cfg, tok, steps=[i], stop=i + 1)
        Po_i = oracle_at(i, w_i.cpu().numpy().astype(np.float64)[:n])[0]
        assert np.abs(P_i[0].cpu().numpy() - Po_i).max() <= 1e-4
    _, w0 = gpu.model_trace(cfg, tok, stop=t)         # first Adam update from zero moments
    _, w1 = gpu.model_trace(cfg, tok, stop=t + 1)
    w0 = w0.cpu().numpy().astype(np.float64)[:n]
    _, g, _, _ = oracle_at(t, w0)
    want = w0.copy()
    orc.opt_step(1, cfg["lr"], cfg["beta1"], cfg["beta2"], cfg["eps"], want, g, np.zeros(n), np.zeros(n), 1)
    big = np.abs(g) > 1e-4 * np.abs(g).max()
    err = np.abs(w1.cpu().numpy()[:n] - want)
    print(f"first Adam step: {big.sum()} of {n} coordinates compared, max err {err[big].max():.3g}")
    assert big.sum() > n // 4 and err[big].max() <= 1e-6


def test_static_mixer_probabilities(gpu, orc):
    """Eq. 1 with the frozen static model (the second workload's model
    shape) on a short sequence: P within 1e-4 along the trajectory."""
    cfg = model_small(s=1, k=3, hidden=[128], selector="spum_dm")
    static = np.fromfile(os.path.join(GOLD, "static_cfg2.f32"), dtype=np.float32)
    a = synth.generate(synth.recipe_cfg2(seed=22, n=64 * 400 + 2))
    a = a[a != ord("N")]
    tok = orc.encode_skmer(a, 1, 3)
    L = len(tok) // cfg["bs"]
    steps = [cfg["t"], 100, L - 1]
    Pg, wg = gpu.model_trace(cfg, tok, steps=steps, static=static)
    Po, _, wo = orc.trace_block(cfg, tok, steps=steps, static=static)
    assert np.abs(Pg.cpu().numpy() - Po).max() <= 1e-4
    assert abs(float(wg[-1]) - wo[-1]) <= 1e-4      # learned mixing weight


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_uneven_blocks_workload_scaled(gpu, orc, precision):
    """The third workload's structure at 1/256 scale: 256 blocks of lognormal
    length in one persistent launch; round trip and ratio within 0.5%."""
    from synth.workloads import cfg3
    rec, cfg = cfg3(n=1 << 22)
    cfg = dict(cfg, precision=precision)
    a = synth.generate(rec)
    assert len(cfg["block_len"]) == 256 and sum(cfg["block_len"]) == len(a)
    blob = gpu.compress(cfg, _cuda(a))
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    assert abs(len(blob) / len(orc.compress(cfg, a)) - 1) <= 0.005


def test_archive_with_model_passing_scaled(gpu, orc):
    """The fifth workload's structure at 1/1024 scale (64 files, log-uniform
    sizes, per-file sources, N runs, 8 KiB blocks, model passing at 5%
    within each file); every file round-trips bit-exactly."""
    from synth.workloads import cfg5
    recs, cfg = cfg5(scale=1 / 1024, block=8192)
    files = [synth.generate(r) for r in recs]
    a = np.concatenate(files)
    blob = gpu.compress(cfg, _cuda(a))
    back = gpu.decompress(blob).cpu().numpy()
    off = 0
    for f in files:
        assert np.array_equal(back[off:off + len(f)], f)
        off += len(f)
    assert abs(len(blob) / len(orc.compress(cfg, a)) - 1) <= 0.005


def test_large_model_adam_global_activations(gpu, orc):
    """The fourth workload's model (context 64, embed 64, hidden [256, 256],
    bs 128, Adam): activations exceed the LDS and live in a per-workgroup
    global slab. Round trip, ratio within 0.5%, P along the trajectory."""
    from synth.workloads import cfg4
    rec, cfg = cfg4(n=3 * 128 * 80 + 2, n_blocks=1)
    a = synth.generate(rec)
    blob = gpu.compress(cfg, _cuda(a))
    assert blob[5] == 1
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    blob_o = orc.compress(cfg, a)
    assert abs(len(blob) / len(blob_o) - 1) <= 0.005
    tok = orc.encode_skmer(a, 3, 3)
    L = len(tok) // cfg["bs"]
    steps = [cfg["t"], cfg["t"] + 3, L - 1]
    Pg, wg = gpu.model_trace(cfg, tok, steps=steps)
    Po, _, wo = orc.trace_block(cfg, tok, steps=steps)
    d = np.abs(Pg.cpu().numpy() - Po)
    print(f"adam large model |dp| max {d.max():.3g}")
    assert d.max() <= 1e-4


# ---------------------------------------------------- full-size workload
def _oracle_golden(name, a):
    """Container size of the FP64 oracle on the whole workload input
    (tests/golden/<name>_oracle.txt, written by the oracle alone), checked
    against the input's SHA-256; None if that file is absent."""
    import hashlib
    path = os.path.join(GOLD, f"{name}_oracle.txt")
    if not os.path.exists(path):
        return None
    kv = dict(line.split(None, 1) for line in open(path) if line.strip() and not line.startswith("#"))
    assert kv["input_sha256"].strip() == hashlib.sha256(memoryview(a)).hexdigest(), "golden input differs"
    return int(kv["container_bytes"])


def _check_golden(name, a, blob):
    gold = _oracle_golden(name, a)
    if gold is None:
        pytest.skip(f"no full-size oracle result for {name} (tests/golden/make_oracle_goldens.py)")
    rel = len(blob) / gold - 1
    print(f"{name}: GPU {len(blob)} bytes, oracle {gold}, rel {rel:+.6f}")
    assert abs(rel) <= 0.005


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_size_static_workload_roundtrip(gpu, orc, precision):
    """The 64 MiB, 16-block static + dynamic workload at full size, on the
    FP32 and BF16 matrix-core paths: bit-exact GPU round trip, metadata equal
    to the oracle's, teacher-forced P at sampled steps of block 0 (FP32),
    and the container within 0.5% of the oracle's on the whole input."""
    from synth.workloads import cfg2
    rec, cfg = cfg2()
    cfg = dict(cfg, precision=precision)
    static = np.fromfile(os.path.join(GOLD, "static_cfg2.f32"), dtype=np.float32)
    a = synth.generate(rec)
    x = _cuda(a)
    blob = gpu.compress(cfg, x, static=static)
    back = gpu.decompress(blob, static=static)
    assert bool((back == x).all())
    del back
    p = cbf.parse(blob)
    assert p["header"]["n_blocks"] == 16
    # block metadata (N runs) against the oracle's scan of the same bytes
    blk_len = len(a) // 16
    for b in [0, 7, 15]:
        seg = a[b * blk_len:(b + 1) * blk_len]
        isn = np.r_[False, seg == ord("N"), False]
        starts = np.flatnonzero(~isn[:-1] & isn[1:])
        ends = np.flatnonzero(isn[:-1] & ~isn[1:])
        assert p["blocks"][b]["runs"] == list(zip(starts.tolist(), (ends - starts).tolist()))
    # teacher-forced probabilities at sampled steps of block 0
    seg = a[:blk_len]
    tok = orc.encode_skmer(seg[seg != ord("N")], 1, 3)
    L = len(tok) // cfg["bs"]
    for i in [cfg["t"], 1000]:
        _, w_i = gpu.model_trace(cfg, tok, static=static, stop=i)
        P_i, _ = gpu.model_trace(cfg, tok, static=static, steps=[i], stop=i + 1)
        w64 = w_i.cpu().numpy().astype(np.float64)
        n = len(w64) - 1
        rows = np.arange(cfg["bs"]) * L + i
        ctx = np.stack([tok[r - cfg["t"]:r] for r in rows])
        Po, _, _, _ = orc.step(cfg, w64[:n], ctx, tok[rows], ws=static.astype(np.float64), a_alpha=w64[n])
        assert np.max(np.abs(P_i[0].cpu().numpy() - Po)) <= (1e-4 if precision == "fp32" else 0.05)
    _check_golden("static64", a, blob)


def test_full_size_uneven_workload_vs_oracle(gpu):
    """The 1 GiB, 256-block lognormal workload at full size on the BF16
    matrix-core path, one persistent launch: bit-exact round trip and the
    container within 0.5% of the FP64 oracle's on the whole input."""
    from synth.workloads import cfg3
    rec, cfg = cfg3()
    cfg = dict(cfg, precision="bf16")
    a = synth.generate(rec)
    x = _cuda(a)
    blob = gpu.compress(cfg, x)
    assert bool((gpu.decompress(blob) == x).all())
    _check_golden("uneven1g", a, blob)


def test_full_size_archive_vs_oracle(gpu):
    """The 64-file archive at full size (4 MiB blocks, model passing at 5%
    within each file), BF16 matrix cores: bit-exact round trip and the
    container within 0.5% of the FP64 oracle's."""
    from synth.workloads import cfg5
    recs, cfg = cfg5()
    cfg = dict(cfg, precision="bf16")
    a = np.concatenate([synth.generate(r) for r in recs])
    x = _cuda(a)
    blob = gpu.compress(cfg, x)
    assert bool((gpu.decompress(blob) == x).all())
    _check_golden("archive", a, blob)
