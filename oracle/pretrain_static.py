"""Write the frozen static model used by the static + dynamic workload.

The paper pre-trains its static public model on a multi-species corpus
(Sec. 4, stage (a); Sec. 5.1.4) that is not available here. Stand-in: the
oracle's own online method (dynamic model only, the same MLP shape) is run
once over a separate seeded synthetic sequence from the same source recipe,
and its final weights are frozen and stored as little-endian FP32.

Only the oracle is called, so no input of the oracle's comparisons comes
from the GPU path.

    python -m oracle.pretrain_static [--n BASES] [--out PATH]
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth.workloads import cfg2_static_pretrain  # noqa: E402

DEFAULT_OUT = os.path.join(ROOT, "tests", "golden", "static_cfg2.f32")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args(argv)
    rec, cfg = cfg2_static_pretrain(n=a.n)
    seq = synth.generate(rec)
    seq = seq[seq != ord("N")]
    tok = oracle.encode_skmer(seq, cfg["s"], cfg["k"])
    t0 = time.time()
    _, loss, w = oracle.trace_block(cfg, tok)
    n = oracle.param_count(cfg)
    ws = w[:n].astype(np.float32)
    ws.tofile(a.out)
    digest = hashlib.sha256(ws.tobytes()).hexdigest()
    with open(a.out + ".txt", "w") as f:
        f.write(f"# frozen static model for the static + dynamic workload (FP32 little-endian, {n} values)\n")
        f.write(f"# written by: python -m oracle.pretrain_static --n {a.n}\n")
        f.write(f"# training sequence: synth recipe_cfg2_static(seed={rec.seed}, n={rec.n}), N removed\n")
        f.write(f"# mean loss first/last 1000 steps (nats): {loss[cfg['t']:cfg['t'] + 1000].mean():.5f} "
                f"{loss[-1000:].mean():.5f}\n")
        f.write(f"sha256 {digest}\n")
    print(f"wrote {a.out} ({n} params) in {time.time() - t0:.1f}s sha256={digest}")


if __name__ == "__main__":
    main()
