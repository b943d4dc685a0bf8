"""Benchmark of the PMKLC hot path on one MI355X.

One step = compress + decompress of the whole workload through the C ABI
(GskE tokens -> per-block online-learned probabilities -> arithmetic
coder, and back), input already resident in HBM. Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload uneven1g]
                    [--precision fp32|bf16] [--schedule batched|plain]

The default workload is 1 GiB of synthetic DNA in 256 blocks of lognormal
length (median 2 MiB, sigma 1), (3,3)-mers, context 32, embedding 16, one
hidden layer of 32, SGD 1e-3, all blocks in one persistent launch with the
model GEMMs in BF16 on the matrix cores. ``value`` is Eq. 4's throughput,
input bases / (CT + DT), in MB/s with MB = 10^6 bases.  Beside it: the
plain per-block FP32 form (one launch per block) on a stated sample of
blocks, the container size against the FP64 oracle's on the whole input
(tests/golden), ``roofline`` for the step kernel (the learning + coding
loop, >99% of the time) from HIP-event timings, and ``cpu_baseline``, the
FP64 oracle on a bounded sample of the same workload on the host cores.

Other workloads (``--workload``): static64 (64 MiB, frozen static model
mixed by Eq. 1), archive (the 64-file archive with model passing), tf32m
(the paper's Transformer dynamic model on 32 MiB), fourth4g (4 GiB, 1024
blocks, the 1.1 M-parameter Adam model on the launch-sequence loop),
bigru64 (the static64 input with the paper's one-layer BiGRU as the
private static model, trained on the input), small256k; ``--encoder``
times the standalone GskE encoder instead.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK = {"fp32_alu_tflops": 157.3, "bf16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0}

# Sources that define the step kernel; a stored HBM-traffic measurement is
# reported only while their hash matches the one it was taken with.
KERNEL_SOURCES = ["paper_2507_12805_amd/csrc/step_mfma.h", "paper_2507_12805_amd/csrc/step_mfma_inst.hip",
                  "paper_2507_12805_amd/csrc/step_chip.hip",
                  "paper_2507_12805_amd/csrc/step_common.h", "paper_2507_12805_amd/csrc/pmklc_internal.h"]
# the kernel that computed a container, by its numeric-path byte
PATH_KERNEL = {1: "step_kernel (FP32 per-thread FMA)", 2: "step_mfma_kernel (BF16 matrix cores, weights in global memory)",
               3: "step_mfma_kernel (FP32 matrix cores)", 4: "step_chip_kernel (BF16 matrix cores, network on chip)",
               5: "Transformer loop (gemm_kernel BF16 MFMA + attention + coder launches)",
               6: "Transformer loop (gemm_kernel FP32 MFMA + attention + coder launches)",
               7: "MLP launch-sequence loop (gemm_kernel BF16 MFMA + coder launches)",
               8: "MLP launch-sequence loop (gemm_kernel FP32 MFMA + coder launches)"}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(name: str):
    """HBM bytes per step-kernel launch from the counter runs summarised in
    profiles/<name>.json (FETCH_SIZE and WRITE_SIZE, each scaled by the
    factor a copy of known size gives), or None when absent or stale."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return int(t["hbm_bytes_per_launch"])


def flops_per_row(cfg: dict) -> int:
    """Algorithmic FLOPs of one model row (one token of one segment): dynamic
    model forward, its backward (weight and input gradients of every layer),
    and the static model's forward when mixed in."""
    V = 4 ** cfg["k"]
    if cfg.get("arch") == "transformer":
        # K/V for the t positions, q at the last, scores and weighted sum,
        # Wo, the FFN, the head; backward twice the forward
        t, E, (A, F) = cfg["t"], cfg["E"], cfg["hidden"]
        fwd = 2 * (t * E * 2 * A + E * A + 2 * t * A + A * A + 2 * A * F + A * V)
        return 3 * fwd
    dims = [cfg["t"] * cfg["E"]] + list(cfg["hidden"]) + [V]
    fwd = sum(2 * dims[i] * dims[i + 1] for i in range(len(dims) - 1))
    f = 3 * fwd
    if cfg.get("selector") in ("spum_dm", "sprm_dm"):
        if cfg.get("static_arch") == "bigru":
            # both directions' gates over the t positions per layer, Dense, head
            E, h, gd, L = cfg["static_E"], cfg["gru_h"], cfg["dense"], cfg["gru_layers"]
            f += sum(2 * cfg["t"] * 3 * h * ((E if l == 0 else 2 * h) + h) * 2 for l in range(L))
            f += 2 * (2 * h * gd + gd * V)
        else:
            f += fwd
    return f


def oracle_golden(name: str, data: np.ndarray):
    """The FP64 oracle's container size for the whole workload input
    (tests/golden/<name>_oracle.txt, written by the oracle alone), when the
    input's SHA-256 matches."""
    import hashlib
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, val = line.split(None, 1)
                kv[key] = val.strip()
    if kv.get("input_sha256") != hashlib.sha256(memoryview(data)).hexdigest():
        return None
    return int(kv["container_bytes"]), float(kv["bits_per_base"])


def workload(name: str, scale: float = 1.0):
    import synth
    from synth import workloads as W
    if name == "uneven1g":
        n = int((1 << 30) * scale)
        rec, cfg = W.cfg3(n=n)
        desc = (f"uneven1g: {n} bases of order-3 synthetic DNA (5% repeats), 256 blocks of lognormal length "
                "(median 2 MiB x scale, sigma 1), (3,3)-mers, t=32, E=16, hidden [32], bs=64, SGD 1e-3")
        return synth.generate(rec), cfg, None, desc
    if name == "archive":
        recs, cfg = W.cfg5(scale=scale)
        data = np.concatenate([synth.generate(r) for r in recs])
        desc = (f"archive: 64 synthetic files, log-uniform 1 KiB-512 MiB x {scale}, per-file order 2-8, GC 0.3-0.7, "
                "repeats 0-30%, N runs; 4 MiB blocks, model passing at 5% of each block's steps within a file; "
                "(3,3)-mers, t=32, E=16, hidden [32], bs=64, SGD 1e-3")
        return data, cfg, None, desc
    if name == "static64":
        rec, cfg = W.cfg2()
        static = np.fromfile(os.path.join(ROOT, "tests", "golden", "static_cfg2.f32"), dtype=np.float32)
        desc = ("static64: 64 MiB synthetic DNA (order-5 Markov, GC 0.35-0.65 per MiB, 10% repeats half "
                "reverse-complement, 0.01% N runs), 16 equal blocks, (1,3)-mers, t=32, E=16, hidden [128], "
                "bs=64, SGD 0.1, frozen static model + dynamic model mixed by Eq. 1")
    elif name == "tf32m":
        rec, cfg = W.tf_paper()
        static = None
        desc = ("tf32m: 32 MiB order-3 synthetic DNA, 16 equal blocks, (3,3)-mers, t=32, bs=320, the paper's "
                "Transformer DM (embed 64, 8 heads of width 256, FFN 4096), Adam 1e-3")
    elif name == "bigru64":
        rec, cfg = W.bigru_private()
        static = None
        desc = ("bigru64: the static64 input and dynamic model ((1,3)-mers, t=32, E=16, hidden [128], bs=64, "
                "SGD 0.1) with the paper's one-layer BiGRU (embedding 16, 32 units per direction, Dense 128) as "
                "the static private model, trained on the input (8192 steps) and mixed by Eq. 1")
    elif name == "fourth4g":
        n = int((1 << 32) * scale) // 1024 * 1024
        rec, cfg = W.cfg4(n=n)
        static = None
        size = "4 GiB" if n == 1 << 32 else f"{n} bases of"
        desc = (f"fourth4g: {size} order-3 synthetic DNA (5% repeats), 1024 equal blocks, (3,3)-mers, t=64, E=64, "
                "hidden [256, 256], bs=128, Adam 1e-3")
    elif name == "small256k":
        rec, cfg = W.cfg1()
        static = None
        desc = "small256k: 256 KiB order-3 synthetic DNA, one block, (3,3)-mers, t=32, E=16, hidden [32], bs=64"
    else:
        raise SystemExit(f"unknown workload {name}")
    return synth.generate(rec), cfg, static, desc


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(cfg, static, data, sample_bytes):
    """The oracle as it stands, on the first ``sample_bytes`` of the input
    split into as many equal blocks as the workload has."""
    import oracle
    nblk = cfg.get("n_blocks", 1)
    sample = np.ascontiguousarray(data[:sample_bytes])
    c = dict(cfg, n_blocks=nblk)
    t0 = time.perf_counter()
    blob = oracle.compress(c, sample, static=static)
    t1 = time.perf_counter()
    back = oracle.decompress(blob, static=static)
    t2 = time.perf_counter()
    assert np.array_equal(back, sample)
    cores = min(oracle.num_threads(), nblk)
    return {"value": round(len(sample) / (t2 - t0) / 1e6, 6), "unit": "MB/s", "cores": cores, "kind": "oracle",
            "sample": f"first {len(sample)} bases of the workload as {nblk} equal blocks, compress+decompress "
                      f"({t1 - t0:.1f}s + {t2 - t1:.1f}s), FP64",
            "ratio_bits_per_base": 8.0 * len(blob) / len(sample)}, blob, sample


SKMER_PAIRS = [(s, k) for k in range(1, 5) for s in range(1, k + 1)]
TABLE8_BASES = 554_197_554   # the size of the sequence of the paper's (s,k) sweep (Table 8)


def run_encoder(a, P, torch):
    """GskE alone (Sec. 4.1) on a Table-8-sized synthetic sequence, every (s,k)
    with s <= k <= 4: HBM bytes moved (ASCII read + tokens written) per second
    of device time (HIP events around each call, best of a.reps), against the
    HBM peak; the oracle's tokeniser timed on a sample beside it."""
    import synth
    log(f"generating {TABLE8_BASES} bases")
    data = synth.generate(synth.recipe_cfg1(seed=8, n=TABLE8_BASES))
    n = len(data)
    x = torch.from_numpy(data).cuda()
    pairs = {}
    best_gbs, best_ms = 0.0, 0.0
    for s, k in SKMER_PAIRS:
        P.encode_skmer(x, s, k)   # warm-up
        times = []
        for _ in range(a.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            tok = P.encode_skmer(x, s, k)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = min(times)
        l = tok.numel()
        gbs = (n + l) / (ms * 1e-3) / 1e9
        pairs[f"({s},{k})"] = {"tokens": l, "ms": round(ms, 4), "GB_per_s": round(gbs, 1),
                               "Mbases_per_s": round(n / (ms * 1e-3) / 1e6, 1)}
        log(f"(s,k)=({s},{k}): {l} tokens, {ms:.3f} ms, {gbs:.0f} GB/s")
        if gbs > best_gbs:
            best_gbs, best_ms = gbs, ms
        del tok
    mean_gbs = sum(v["GB_per_s"] for v in pairs.values()) / len(pairs)
    res = {
        "metric": "GskE tokenisation GB/s (ASCII read + tokens written), Table-8-sized sequence",
        "value": round(mean_gbs, 1), "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "u8", "data": "synthetic (seeded order-3 Markov DNA stand-in for the paper's genome)",
        "config": {"workload": f"skmer: {n} bases, all (s,k) with 1 <= s <= k <= 4, standalone encoder",
                   "bases": n, "reps": a.reps},
        "per_pair": pairs,
        "roofline": {"bound": "hbm", "achieved": round(best_gbs, 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                     "frac": round(best_gbs / PEAK["hbm_gbs"], 4), "traffic": None, "kernel": "skmer_direct_kernel",
                     "bytes_per_launch": "n + tokens (1 B per input base read, 1 B per token written)"},
    }
    if not a.no_cpu_baseline:
        import oracle
        m = min(n, 16 << 20)
        sample = np.ascontiguousarray(data[:m])
        t0 = time.perf_counter()
        want = oracle.encode_skmer(sample, 3, 3)
        t1 = time.perf_counter()
        got = P.encode_skmer(torch.from_numpy(sample).cuda(), 3, 3).cpu().numpy()
        res["cpu_baseline"] = {"value": round((m + len(want)) / (t1 - t0) / 1e9, 4), "unit": "GB/s", "cores": 1,
                               "kind": "oracle", "sample": f"first {m} bases, (s,k)=(3,3), plain C",
                               "tokens_equal_gpu": bool(np.array_equal(got, want))}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven1g", choices=["static64", "small256k", "uneven1g", "archive", "tf32m",
                                                                "fourth4g", "bigru64"])
    ap.add_argument("--scale", type=float, default=1.0, help="size scale for uneven1g / archive / fourth4g")
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp32_valu"])
    ap.add_argument("--no-fp32-compare", action="store_true",
                    help="skip the batched FP32 compress+decompress measured beside the main precision")
    ap.add_argument("--schedule", default="batched", choices=["batched", "plain"])
    ap.add_argument("--cpu-sample-bytes", type=int, default=1 << 22)
    ap.add_argument("--cpu-sample-blocks", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-blocks", type=int, default=4,
                    help="blocks compressed with one launch per block for the plain-FP32 comparison (0 = skip)")
    ap.add_argument("--encoder", action="store_true",
                    help="measure the standalone GskE encoder on a Table-8-sized sequence instead")
    ap.add_argument("--reps", type=int, default=5, help="timed calls per (s,k) in --encoder mode")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the hot path shards by independent blocks, "
              "see the design notes", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2507_12805_amd as P
    P.load()
    torch.cuda.set_device(0)
    if a.copy_probe_mib:
        src = torch.empty(a.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if a.encoder:
        run_encoder(a, P, torch)
        return
    log(f"generating workload {a.workload}")
    data, cfg, static, desc = workload(a.workload, a.scale)
    cfg = dict(cfg, precision=a.precision, schedule=a.schedule)
    n = len(data)
    x = torch.from_numpy(data).cuda()
    ws = P.Workspace()
    wsd = P.Workspace()
    out = None
    ct, dt, ks_c, ks_d = [], [], [], []
    ok = True
    blob = b""
    tim_c = tim_d = None
    for it in range(a.warmup + a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        blob = P.compress(cfg, x, static=static, workspace=ws)
        t1 = time.perf_counter()
        tim_c = P.last_timing()
        out = P.decompress(blob, static=static, workspace=wsd, out=out)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tim_d = P.last_timing()
        if it == 0 or it == a.warmup + a.steps - 1:
            ok = ok and bool((out[:n] == x).all())
        log(f"step {it} ({'warmup' if it < a.warmup else 'timed'}): compress {t1 - t0:.3f}s "
            f"(kernel {tim_c['step_ms']:.1f} ms), decompress {t2 - t1:.3f}s (kernel {tim_d['step_ms']:.1f} ms), "
            f"{len(blob)} bytes")
        if it >= a.warmup:
            ct.append(t1 - t0)
            dt.append(t2 - t1)
            ks_c.append(tim_c["step_ms"])
            ks_d.append(tim_d["step_ms"])
    CT, DT = float(np.mean(ct)), float(np.mean(dt))
    value = n / (CT + DT) / 1e6
    fpr = flops_per_row(cfg)
    launch_ms = float(np.mean(ks_c + ks_d))
    flops_launch = tim_c["model_rows"] * fpr
    achieved = flops_launch / (launch_ms * 1e-3) / 1e12
    bound, peak = ("mfma", PEAK["bf16_mfma_tflops"]) if a.precision == "bf16" else ("alu", PEAK["fp32_alu_tflops"])
    res = {
        "metric": "compress/decompress MB/s at ratio within 0.5% of oracle, batched BF16 vs plain FP32",
        "value": round(value, 4), "unit": "MB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round((CT + DT) * 1e3, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if a.precision == "fp32" else "bf16",
        "data": "synthetic (seeded Markov DNA stand-in for the paper's genomes)",
        "config": {"workload": desc, "bases": n, "blocks": len(cfg["block_len"]) if "block_len" in cfg else cfg.get("n_blocks", 1), "precision": a.precision,
                   "schedule": a.schedule},
        "compress_MBps": round(n / CT / 1e6, 4), "decompress_MBps": round(n / DT / 1e6, 4),
        "ratio_bits_per_base": round(8.0 * len(blob) / n, 5), "roundtrip_bit_exact": ok,
        "step_kernel_ms": {"compress": round(float(np.mean(ks_c)), 3), "decompress": round(float(np.mean(ks_d)), 3)},
        "roofline": {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 6),
                     "traffic": stored_traffic(f"traffic_step_kernel_{a.workload}_{a.precision}")
                     if a.schedule == "batched" and a.scale == 1.0 else None,
                     "kernel": PATH_KERNEL.get(blob[5] if blob else 0, "step kernel"),
                     "flops_per_launch": int(flops_launch), "flops_per_row": fpr,
                     "rows_per_launch": int(tim_c["model_rows"]), "max_steps": int(tim_c["max_steps"])},
    }
    res["threads_per_workgroup"] = int(tim_c["threads"])
    gold = oracle_golden(a.workload, data) if a.scale == 1.0 else None
    if gold:
        res["oracle_full"] = {"container_bytes": gold[0], "bits_per_base": gold[1],
                              "gpu_container_bytes": len(blob), "ratio_rel_diff": round(len(blob) / gold[0] - 1.0, 6),
                              "source": f"tests/golden/{a.workload}_oracle.txt (FP64 oracle on the whole input)"}
    # the sample of blocks for the per-block comparisons: the first few blocks
    if "block_len" in cfg:
        lens = [int(v) for v in cfg["block_len"]]
    else:
        nb = cfg.get("n_blocks", 1)
        lens = [n // nb] * (nb - 1) + [n - (n // nb) * (nb - 1)]
    kb = min(a.plain_blocks, len(lens))
    sub_n = sum(lens[:kb])
    sub = x[:sub_n]
    sub_cfg = {q: v for q, v in cfg.items() if q not in ("block_len", "file_blocks", "smp_ppm")}
    sub_cfg.update(block_len=lens[:kb], n_blocks=kb)
    sample_desc = f"blocks 0-{kb - 1} of {len(lens)} ({sub_n} bases), model passing off"
    # the launch-sequence loop (paths 5-8) runs every block's step in one
    # sequence of launches: it has no per-block launch form
    tf = cfg.get("arch") == "transformer" or (blob[5] in (5, 6, 7, 8) if blob else False)
    if kb and a.schedule == "batched" and not tf:
        cp = dict(sub_cfg, precision="fp32", schedule="plain")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bp = P.compress(cp, sub, static=static, workspace=ws)
        t1 = time.perf_counter()
        op = P.decompress(bp, static=static, workspace=wsd)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res["plain_fp32"] = {"compress_MBps": round(sub_n / (t1 - t0) / 1e6, 4),
                             "decompress_MBps": round(sub_n / (t2 - t1) / 1e6, 4),
                             "value": round(sub_n / (t2 - t0) / 1e6, 4),
                             "roundtrip_bit_exact": bool((op[:sub_n] == sub).all()),
                             "sample": sample_desc + ", one FP32 launch per block"}
        log(f"plain fp32, {kb} blocks: compress {t1 - t0:.3f}s decompress {t2 - t1:.3f}s")
        if not a.no_fp32_compare and a.precision != "fp32":
            cf = dict(sub_cfg, precision="fp32")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b32 = P.compress(cf, sub, static=static, workspace=ws)
            t1 = time.perf_counter()
            o32 = P.decompress(b32, static=static, workspace=wsd)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            bb = P.compress(dict(sub_cfg), sub, static=static, workspace=ws)
            res["fp32_batched"] = {"compress_MBps": round(sub_n / (t1 - t0) / 1e6, 4),
                                   "decompress_MBps": round(sub_n / (t2 - t1) / 1e6, 4),
                                   "value": round(sub_n / (t2 - t0) / 1e6, 4),
                                   "roundtrip_bit_exact": bool((o32[:sub_n] == sub).all()),
                                   "bf16_ratio_cost_rel": round(len(bb) / len(b32) - 1.0, 6),
                                   "sample": sample_desc + ", one batched FP32 launch"}
            log(f"fp32 batched, {kb} blocks: compress {t1 - t0:.3f}s decompress {t2 - t1:.3f}s")
    if not a.no_cpu_baseline:
        log("oracle on the CPU sample")
        ccfg = {k: v for k, v in cfg.items() if k not in ("block_len", "file_blocks", "smp_ppm")}
        ccfg["n_blocks"] = a.cpu_sample_blocks if not tf else 2
        # the Transformer's FP64 oracle costs ~20 MFLOP a row: two blocks of
        # 40 steps (8 learned) keep it to about a minute
        cb, oblob, sample = cpu_baseline(ccfg, static, data, a.cpu_sample_bytes if not tf else 2 * 3 * 320 * 40)
        gcfg = ccfg
        gblob = P.compress(dict(gcfg, schedule="batched"), torch.from_numpy(sample).cuda(), static=static)
        cb["gpu_ratio_bits_per_base_same_sample"] = round(8.0 * len(gblob) / len(sample), 5)
        cb["ratio_rel_diff"] = round(len(gblob) / len(oblob) - 1.0, 6)
        res["cpu_baseline"] = cb
    res["paper_context"] = ("PMKLC-S 20.987 KB/s and PMKLC-M 60.897 KB/s average Eq. 4 throughput (Table 5) on "
                            "1x / multiple RTX 4090 with a Transformer+BiGRU model on real genomes; not like-for-like")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
