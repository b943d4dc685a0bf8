"""GPU checks of the boundary's robustness: unaligned encoder inputs for
every (s,k), model-passing chains whose total wait far exceeds the wait
bound (the bound applies to a running predecessor that makes no step), the
give-up path of that wait forced from the host, and the differentiable op's
rejection of out-of-vocabulary context tokens without writing outside its
workspace."""
import ctypes

import numpy as np
import pytest

import synth
from synth.workloads import model_small

pytestmark = pytest.mark.gpu

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


@pytest.mark.parametrize("s,k", PAIRS)
def test_skmer_unaligned_every_pair(gpu, orc, s, k):
    """Input pointers 1, 2 and 3 bytes past a 4-byte boundary, with token
    counts around the 4096-token workgroup tile and a ragged last tile."""
    a = _dna(5 * 4096 * s + 64, seed=40 + 4 * k + s)
    x = _cuda(a)
    for off in [1, 2, 3]:
        for l in [1, 4095, 4096, 4097, 2 * 4096 + 13, 5 * 4096 - 1]:
            n = (l - 1) * s + k + (s - 1)          # ragged tail of s - 1 bases
            got = gpu.encode_skmer(x[off:off + n], s, k).cpu().numpy()
            want = orc.encode_skmer(a[off:off + n], s, k)
            assert len(want) == l
            assert np.array_equal(got, want), (s, k, off, l)


def _chain_case():
    # one file of 48 blocks, each passing its model to the next at 5% of its
    # steps, on the per-thread FMA kernel with a two-hidden-layer model
    cfg = model_small(t=8, E=8, hidden=[64, 64], bs=16, precision="fp32_valu", smp_ppm=50000)
    lens = [3000 + 37 * (b % 5) for b in range(48)]
    a = _dna(sum(lens), seed=77, rho=0.05)
    return dict(cfg, block_len=lens, file_blocks=[len(lens)]), a


def test_long_passing_chain_with_small_wait_bound(gpu, monkeypatch):
    """The last block of a 48-block chain waits for 47 predecessors in turn,
    far longer in total than a wait bound of 2^14 sleeps (a few ms), yet
    every predecessor steps within it: the call must succeed and round-trip."""
    cfg, a = _chain_case()
    ref = gpu.compress(cfg, _cuda(a))
    monkeypatch.setenv("PMKLC_SPIN_LIMIT", str(1 << 14))
    blob = gpu.compress(cfg, _cuda(a))
    assert blob == ref
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)


def test_passing_wait_give_up_path(gpu, monkeypatch):
    """With a zero wait bound a waiting block gives up as soon as its running
    predecessor takes longer than one poll for a step: the call reports a
    device error, every kernel still ends, and the next call is unaffected."""
    cfg, a = _chain_case()
    monkeypatch.setenv("PMKLC_SPIN_LIMIT", "0")
    with pytest.raises(gpu.PmklcError) as e:
        gpu.compress(cfg, _cuda(a))
    assert e.value.code == -6
    monkeypatch.delenv("PMKLC_SPIN_LIMIT")
    blob = gpu.compress(cfg, _cuda(a))
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)


def test_dm_backward_rejects_out_of_vocabulary_tokens(gpu):
    """A context token >= 4^k gives PMKLC_ERR_INVALID_ARG from the backward,
    and nothing past the workspace it was given is written."""
    import torch
    cfg = model_small(t=64, E=64, hidden=[256, 256], bs=128)
    L = gpu.load()
    c, _ = gpu.make_config(cfg)
    rows = 128
    ws_b = ctypes.c_uint64(0)
    assert L.pmklc_dm_workspace(ctypes.byref(c), rows, ctypes.byref(ws_b)) == 0
    guard = 1 << 18
    buf = torch.full((ws_b.value + guard,), 0xA5, dtype=torch.uint8, device="cuda")
    n = gpu.param_count(cfg)
    params = torch.randn(n, dtype=torch.float32, device="cuda") * 0.05
    ctx = torch.randint(0, 64, (rows, 64), dtype=torch.uint8, device="cuda")
    ctx[5, 7] = 255
    ctx[100, 0] = 200
    dl = torch.randn(rows, 64, dtype=torch.float32, device="cuda")
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.pmklc_dm_backward(ctypes.byref(c), ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(ctx.data_ptr()),
                             rows, ctypes.c_void_p(dl.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                             ctypes.c_void_p(buf.data_ptr()), ws_b.value, st)
    torch.cuda.synchronize()
    assert rc == -1
    assert bool((buf[ws_b.value:] == 0xA5).all())
