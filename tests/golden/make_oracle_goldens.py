"""Write the full-size oracle results of the benchmark workloads.

For each workload this runs the FP64 oracle's compressor over the whole
seeded synthetic input (for the fourth workload: its first 16 blocks, each
at full length) and records the input's SHA-256, the container length and
SHA-256, and the compression ratio (Eq. 3: container bits per input base).
The GPU tests and the bench compare their own container sizes with these
numbers (ratio within 0.5%).

Only ``oracle/`` and ``synth/`` are called: no stored value comes from the
GPU path.

    python tests/golden/make_oracle_goldens.py WORKLOAD [--threads N]

WORKLOAD is one of static64, uneven1g, archive, fourth16. The result goes
to tests/golden/<WORKLOAD>_oracle.txt. Runs take from tens of minutes to a
few hours on 8 host cores (the oracle runs blocks in parallel, each block
on one core).
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def workload(name: str):
    """(input bytes, model configuration, static weights or None, description)."""
    import synth
    from synth import workloads as W
    if name == "static64":
        rec, cfg = W.cfg2()
        static = np.fromfile(os.path.join(HERE, "static_cfg2.f32"), dtype=np.float32)
        return synth.generate(rec), cfg, static, "64 MiB, 16 equal blocks, (1,3)-mers, static + dynamic model"
    if name == "uneven1g":
        rec, cfg = W.cfg3()
        return synth.generate(rec), cfg, None, "1 GiB, 256 lognormal blocks, (3,3)-mers, t 32, E 16, H [32]"
    if name == "archive":
        recs, cfg = W.cfg5()
        data = np.concatenate([synth.generate(r) for r in recs])
        return data, cfg, None, "64 files (1 KiB-512 MiB), 4 MiB blocks, model passing at 5%"
    if name == "fourth16":
        rec, cfg = W.cfg4()
        data = synth.generate(rec)
        per = len(data) // cfg["n_blocks"]
        sample = np.ascontiguousarray(data[:16 * per])
        del data
        return sample, dict(cfg, n_blocks=16), None, \
            "blocks 0-15 (4 MiB each) of the 4 GiB, 1024-block input; t 64, E 64, H [256, 256], bs 128, Adam"
    raise SystemExit(f"unknown workload {name}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["static64", "uneven1g", "archive", "fourth16"])
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import oracle
    t0 = time.time()
    data, cfg, static, desc = workload(a.workload)
    tg = time.time() - t0
    isha = hashlib.sha256(memoryview(data)).hexdigest()
    print(f"[golden] {a.workload}: {len(data)} bases generated in {tg:.1f}s, sha256 {isha}", flush=True)
    t1 = time.time()
    blob = oracle.compress(cfg, data, static=static)
    tc = time.time() - t1
    csha = hashlib.sha256(blob).hexdigest()
    bpb = 8.0 * len(blob) / len(data)
    out = a.out or os.path.join(HERE, f"{a.workload}_oracle.txt")
    with open(out, "w") as f:
        f.write(f"# FP64 oracle compression of the {a.workload} workload: {desc}\n")
        f.write(f"# written by: python tests/golden/make_oracle_goldens.py {a.workload}\n")
        f.write(f"# oracle compress time {tc:.0f} s on {oracle.num_threads()} host threads\n")
        f.write(f"input_bases {len(data)}\n")
        f.write(f"input_sha256 {isha}\n")
        f.write(f"container_bytes {len(blob)}\n")
        f.write(f"container_sha256 {csha}\n")
        f.write(f"bits_per_base {bpb:.6f}\n")
    print(f"[golden] {a.workload}: {len(blob)} bytes, {bpb:.5f} bits/base, {tc:.0f}s -> {out}", flush=True)


if __name__ == "__main__":
    main()
