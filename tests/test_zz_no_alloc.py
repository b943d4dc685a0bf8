"""GPU check of pmklc_compress_noalloc (the compress entry point that takes
its workspace from the library's fixed device buffer instead of a caller's
allocation): its containers equal pmklc_compress's byte for byte on two
calls in a row, the second with a smaller input (the buffer keeps the first
call's contents), they decode back to the input, and an input whose
workspace exceeds the buffer is rejected before any device work."""
import numpy as np
import pytest

import synth
from synth.workloads import model_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_12805_amd as P
    P.load()
    return P


def _dna(n, seed):
    return synth.generate(synth.Recipe(n=n, order=3, seed=seed, rho=0.05, n_rate=0.001, n_max=20))


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [
    # matrix-core BF16 path, the default small model, 3 uneven blocks
    (dict(model_small(precision="bf16"), block_len=[150000, 90000, 60000]), 300000,
     dict(model_small(precision="bf16"), block_len=[70000, 50000]), 120000),
    # per-thread FMA path, two hidden layers, Adam, model passing in one file
    (model_small(t=8, E=8, hidden=[24, 16], bs=16, n_blocks=3, optimizer="adam", lr=3e-3, smp_ppm=50000,
                 precision="fp32_valu"), 90000,
     model_small(t=8, E=8, hidden=[24, 16], bs=16, n_blocks=2, optimizer="adam", lr=3e-3, smp_ppm=50000,
                 precision="fp32_valu"), 30001),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_compress_twice(gpu, case):
    cfg1, n1, cfg2, n2 = CASES[case]
    for cfg, n, seed in [(cfg1, n1, 500 + case), (cfg2, n2, 600 + case)]:
        a = _dna(n, seed)
        x = _cuda(a)
        want = gpu.compress(cfg, x)
        got = gpu.compress_noalloc(cfg, x)
        assert got == want, (case, n, len(got), len(want))
        assert np.array_equal(gpu.decompress(got).cpu().numpy(), a)


def test_noalloc_uniform_and_empty(gpu):
    cfg = model_small(selector="uniform", n_blocks=2)
    a = _dna(10001, 7)
    assert gpu.compress_noalloc(cfg, _cuda(a)) == gpu.compress(cfg, _cuda(a))
    e = np.zeros(0, dtype=np.uint8)
    assert gpu.compress_noalloc(cfg, _cuda(e)) == gpu.compress(cfg, _cuda(e))


def test_noalloc_rejects_inputs_beyond_its_buffer(gpu):
    import torch
    cfg = model_small()
    n = 8 << 20
    _, ws = gpu.compress_bound(cfg, n)
    assert ws > 64 << 20
    x = torch.full((n,), ord("A"), dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu.PmklcError) as e:
        gpu.compress_noalloc(cfg, x)
    assert e.value.code == -8
    # the entry point still works afterwards
    a = _dna(5000, 9)
    assert gpu.compress_noalloc(cfg, _cuda(a)) == gpu.compress(cfg, _cuda(a))
