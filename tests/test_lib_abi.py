"""CPU checks of the C-ABI library: it loads, exports every function that
include/pmklc.h declares, and the Python binding's config struct has the
C layout (no GPU compute is called here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmklc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pmklc_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_2507_12805_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2507_12805_amd import build
        build.build()
    return P


def test_library_exports_every_declared_symbol(lib):
    L = lib.load()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def test_config_struct_layout_matches_c(lib, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "pmklc.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(pmklc_config), '
                   'offsetof(pmklc_config, seed), offsetof(pmklc_config, block_len_host), '
                   'offsetof(pmklc_config, static_len));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    C = lib._Config
    assert got == [ctypes.sizeof(C), C.seed.offset, C.block_len_host.offset, C.static_len.offset]


def test_status_strings_and_param_count(lib):
    L = lib.load()
    assert L.pmklc_status_string(0) == b"ok"
    assert L.pmklc_status_string(-7) == b"unsupported configuration"
    from synth.workloads import model_small
    assert lib.param_count(model_small()) == 19552
    assert lib.param_count(model_small(s=1, hidden=[128])) == 74944
    assert lib.param_count(model_small(t=64, E=64, hidden=[256, 256], bs=128)) == 1135168


def test_bounds_and_config_errors_without_gpu(lib):
    from synth.workloads import model_small
    mo, ws = lib.compress_bound(model_small(), 1 << 18)
    assert mo > (1 << 18) // 4 and ws > (1 << 18)
    with pytest.raises(lib.PmklcError) as e:
        lib.compress_bound(model_small(s=4, k=3), 100)
    assert e.value.code == -1
    with pytest.raises(lib.PmklcError) as e:
        lib.compress_bound(model_small(E=3), 100)
    assert e.value.code == -7
