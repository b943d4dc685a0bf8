"""Workload descriptions: a synthetic data recipe plus the method's knobs.

Plain dictionaries that the oracle wrapper and the GPU binding each turn
into their own configuration structs. No arithmetic of the method here.

Keys: s, k (GskE step and window), t (context tokens), bs (segments per
block = rows per step), E (embedding width), hidden (MLP widths),
optimizer ("sgd" | "adam"), lr, beta1, beta2, eps, selector ("uniform" |
"dm" | "spum_dm"), smp_ppm (step-wise model passing point in parts per
million of a block's steps; 0 = off), seed (model initialisation),
n_blocks / block_len (raw bytes per block) and file_blocks (blocks per
file; model passing never crosses a file).
"""
from __future__ import annotations

from . import MiB, Recipe, archive_files, lognormal_blocks, recipe_cfg1, recipe_cfg2


def model_small(**kw) -> dict:
    """Embed 16, one hidden layer of 32, context 32, (3,3)-mers, bs 64, SGD 1e-3."""
    c = dict(s=3, k=3, t=32, bs=64, E=16, hidden=[32], optimizer="sgd", lr=1e-3, beta1=0.9, beta2=0.999,
             eps=1e-8, selector="dm", smp_ppm=0, seed=0x5EED, n_blocks=1)
    c.update(kw)
    return c


def cfg1() -> tuple[Recipe, dict]:
    """256 KiB, one block, DM only."""
    return recipe_cfg1(), model_small()


CFG2_LR = 0.1   # the workload names no rate; SGD at 1e-3 leaves (1,3)-mers near 6 bits/base


def cfg2(n: int = 1 << 26, n_blocks: int = 16) -> tuple[Recipe, dict]:
    """64 MiB, 16 equal blocks, (1,3)-mers, static model mixed with the DM
    (Eq. 1), hidden 128, FP32, SGD 0.1."""
    return recipe_cfg2(n=n), model_small(s=1, k=3, hidden=[128], selector="spum_dm", n_blocks=n_blocks, lr=CFG2_LR)


def bigru_private(n: int = 1 << 26, n_blocks: int = 16) -> tuple[Recipe, dict]:
    """The 64 MiB input and dynamic model of cfg2 with the paper's BiGRU as
    the static private model (Sec. 4.2.2 widths, one layer: 16-d embedding,
    32 units per direction, Dense 128), trained on the input before coding
    and mixed by Eq. 1."""
    return recipe_cfg2(n=n), model_small(s=1, k=3, hidden=[128], selector="sprm_dm", n_blocks=n_blocks, lr=CFG2_LR,
                                         static_arch="bigru", static_E=16, gru_h=32, gru_layers=1, dense=128)


def cfg2_static_pretrain(n: int = 1 << 20) -> tuple[Recipe, dict]:
    """The sequence and DM-only run whose final weights become the frozen
    static model of cfg2 (same shape as cfg2's DM)."""
    from . import recipe_cfg2_static
    return recipe_cfg2_static(n=n), model_small(s=1, k=3, hidden=[128], selector="dm", n_blocks=1, seed=0x57A7,
                                                lr=CFG2_LR)


def cfg3(n: int = 1 << 30, n_blocks: int = 256) -> tuple[Recipe, dict]:
    """1 GiB, 256 lognormal blocks (median 2 MiB, sigma 1), cfg1 model."""
    r = recipe_cfg1(seed=3, n=n)
    bl = lognormal_blocks(n, n_blocks, median=max(1, (2 * MiB * n) >> 30), sigma=1.0, seed=3)
    return r, model_small(block_len=bl)


def cfg4(n: int = 1 << 32, n_blocks: int = 1024) -> tuple[Recipe, dict]:
    """4 GiB, 1024 blocks, context 64, embed 64, hidden [256, 256], bs 128, Adam."""
    r = recipe_cfg1(seed=4, n=n)
    return r, model_small(t=64, E=64, hidden=[256, 256], bs=128, optimizer="adam", n_blocks=n_blocks)


def tf_paper(n: int = 32 * MiB, n_blocks: int = 16) -> tuple[Recipe, dict]:
    """The paper's dynamic model (Sec. 4.2.4): Transformer with a 64-d
    embedding, 8-head attention of width 256 and a 4096-wide FFN, at the
    paper's defaults (3,3)-mers, t 32, bs 320 (Sec. 5.1.4); Adam 1e-3 (the
    paper names no optimiser); 32 MiB of the order-3 source in 16 equal
    blocks."""
    r = recipe_cfg1(seed=7, n=n)
    return r, model_small(t=32, E=64, hidden=[256, 4096], bs=320, arch="transformer", heads=8, optimizer="adam",
                          lr=1e-3, n_blocks=n_blocks)


def cfg5(scale: float = 1.0, block: int = 4 * MiB) -> tuple[list[Recipe], dict]:
    """Mixed archive of 64 files; 4 MiB blocks per file; model passing at 5%
    of each block's steps between consecutive blocks of a file."""
    files = archive_files(scale=scale)
    bl, fb = [], []
    for r in files:
        nb = max(1, (r.n + block - 1) // block)
        fb.append(nb)
        for q in range(nb):
            bl.append(min(block, r.n - q * block))
    return files, model_small(block_len=bl, file_blocks=fb, smp_ppm=50000)
