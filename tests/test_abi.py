"""The C-ABI library loads, exports every symbol include/camelot.h declares, and the
Python binding's struct layouts match the C compiler's (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2005_02088_amd import camelot as cm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "camelot.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(camelot_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = ctypes.CDLL(cm.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared but not exported"
    assert names == cm.EXPORTS


def test_struct_layouts_match_c(tmp_path):
    fields = {name: [f[0] for f in st._fields_] for name, st in cm.STRUCTS.items()}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for name, fl in fields.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in fl:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for name, st in cm.STRUCTS.items():
        assert int(got[name]) == ctypes.sizeof(st), name
        for f in fields[name]:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, f"{name}.{f}"


def test_stage_row_bytes_and_validation():
    relu = cm.stage_desc(cm.STAGE_GEMM_RELU, dims=(512, 512), weights=(1,))
    assert cm.camelot_stage_row_bytes_in(relu) == 2048
    assert cm.camelot_stage_row_bytes_out(relu) == 2048
    topk = cm.stage_desc(cm.STAGE_TOPK, dims=(4096,), k=10, n_layers=0)
    assert cm.camelot_stage_row_bytes_out(topk) == 80
    mel = cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0)
    assert (cm.camelot_stage_row_bytes_in(mel), cm.camelot_stage_row_bytes_out(mel)) == (8000, 1760)
    mlp = cm.stage_desc(cm.STAGE_MLP_BF16, dims=(440, 2048, 2048, 2048, 4096), weights=(1, 1, 1, 1))
    assert cm.camelot_stage_row_bytes_out(mlp) == 4 * 4096
    with pytest.raises(cm.CamelotError) as e:
        cm.camelot_stage_row_bytes_in(cm.stage_desc(cm.STAGE_TOPK, dims=(4096,), k=0, n_layers=0))
    assert e.value.code == cm.EINVAL
    with pytest.raises(cm.CamelotError):
        cm.camelot_stage_row_bytes_in(cm.stage_desc(cm.STAGE_MLP_BF16, dims=(440, 2050), weights=(1,)))
    with pytest.raises(cm.CamelotError):
        cm.camelot_stage_row_bytes_in(cm.stage_desc(99))


def _brute_handoff(slot_bytes, n_slots):
    import numpy as np
    w = np.arange(slot_bytes // 4, dtype=np.uint64)
    s = 0
    x = 0
    for sl in range(n_slots):
        c = np.uint64((sl * 0x9E3779B1) & 0xFFFFFFFF)
        v = (w ^ c) & np.uint64(0xFFFFFFFF)
        s = (s + int(v.sum())) % (1 << 64)
        x ^= int(np.bitwise_xor.reduce(v))
    return s, x


@pytest.mark.parametrize("slot_bytes,n_slots", [(16, 1), (48, 3), (4096, 7), (65536 + 16, 5)])
def test_handoff_expected_checksum(slot_bytes, n_slots):
    assert cm.camelot_handoff_expected(slot_bytes, n_slots) == _brute_handoff(slot_bytes, n_slots)


def test_noalloc_run_refuses_what_its_array_cannot_hold():
    """The allocation-free stage run checks every argument on the host first: a stage
    whose scratch exceeds the static array, or a bad share, is refused before any
    device call (so this runs without a GPU)."""
    cap = cm.NOALLOC_SCRATCH_BYTES
    # conv scratch = 128 rows x 64 channels x 4 bytes per 64-pixel tile: 256 tiles fit
    assert 32768 * 256 == cap
    big_map = cm.stage_desc(cm.STAGE_CONV_POOL, dims=(129, 128, 64, 64), weights=(1,), n_layers=0)
    with pytest.raises(cm.CamelotError) as e:                 # 258 tiles
        cm.camelot_stage_run_noalloc(big_map, 1, 1, 1, 8)
    assert e.value.code == cm.EINVAL and "scratch" in str(e.value)
    relu = cm.stage_desc(cm.STAGE_GEMM_RELU, dims=(512, 512), weights=(1,))
    for n_cus in (0, 12, 264):
        with pytest.raises(cm.CamelotError) as e:
            cm.camelot_stage_run_noalloc(relu, 1, 1, 1, n_cus)
        assert e.value.code == cm.EINVAL
    with pytest.raises(cm.CamelotError) as e:
        cm.camelot_stage_run_noalloc(relu, 1, 1, cm.MAX_BATCH + 1, 8)
    assert e.value.code == cm.EINVAL


def test_ipc_region_refuses_bad_geometry_before_any_device_call():
    """A cross-process handoff region is checked on the host first: slot sizes that are
    not multiples of 16, no channels, and regions of 2 GiB or more (an opened
    allocation must stay under 2 GiB) are refused without touching a GPU."""
    for slot, depth, ch in ((8, 4, 8), (24, 4, 8), (1 << 20, 0, 8), (1 << 20, 4, 0), (1 << 20, 4, 257)):
        with pytest.raises(cm.CamelotError) as e:
            cm.camelot_ipc_region_create(slot, depth, ch)
        assert e.value.code == cm.EINVAL
    with pytest.raises(cm.CamelotError) as e:
        cm.camelot_ipc_region_create(1 << 29, 4, 128)          # 2 GiB of slots
    assert e.value.code == cm.EINVAL and "2 GiB" in str(e.value)
