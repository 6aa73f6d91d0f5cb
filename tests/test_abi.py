"""Host-side checks of the C-ABI that need no GPU: the library loads, every
function declared in include/mrx.h is exported, and argument validation
rejects bad plans before any device work."""
import ctypes
import os
import re

import pytest

from paper_2202_14005_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "mrx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(mrx_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_loads_and_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"


def test_version_string():
    assert _lib.lib().mrx_version().decode().startswith("mrx")


@pytest.mark.parametrize("n,ok", [(128, 1), (320, 1), (384, 1), (192, 1), (256, 1), (16, 1), (8, 1), (10, 1),
                                  (240, 1), (288, 1), (640, 1), (1024, 1), (54, 1),
                                  (14, 0), (7, 0), (1026, 0), (1152, 0), (330, 0), (6, 0), (450, 0), (972, 0)])
def test_supported_lengths(n, ok):
    assert _lib.lib().mrx_supported_length(n) == ok


def _create(B, H, W, C):
    L = _lib.lib()
    arr = lambda v: (ctypes.c_int32 * len(v))(*v)
    h = ctypes.c_void_p()
    code = L.mrx_plan_create(ctypes.byref(h), B, arr(H), arr(W), arr(C), 0)
    return code, h, L.mrx_last_error().decode()


def test_plan_rejects_odd_size():
    code, h, msg = _create(1, [127], [128], [8])
    assert code == -1 and "even" in msg and not h.value


def test_plan_rejects_unsupported_length():
    code, h, msg = _create(2, [128, 14], [128, 14], [8, 8])
    assert code == -2 and "slice 1" in msg


def test_plan_rejects_bad_coil_count():
    code, _, msg = _create(1, [128], [128], [0])
    assert code == -1 and "coil" in msg
    code, _, msg = _create(1, [128], [128], [65])
    assert code == -1


def test_plan_rejects_bad_batch_and_null():
    L = _lib.lib()
    code, _, _ = _create(0, [128], [128], [8])
    assert code == -1
    assert L.mrx_plan_create(None, 1, None, None, None, 0) == -1


def test_operators_reject_null_plan():
    L = _lib.lib()
    assert L.mrx_sense_normal(None, None, None, None, None, None, None) == -1
    assert "null plan" in L.mrx_last_error().decode()
    assert L.mrx_cg_dc(None, None, None, None, None, None, 10, None, None, None) == -1
    assert L.mrx_plan_workspace_bytes(None) == 0


def test_tune_cache_file_roundtrip_and_errors(tmp_path):
    from paper_2202_14005_amd import ops
    from paper_2202_14005_amd._lib import MrxError
    name = ops.schedules(320)[0]
    good = tmp_path / "good.txt"
    good.write_text(f"# comment\n320 320 15 8 {name}\n")
    assert ops.tune_cache_load(str(good)) == 1
    out = tmp_path / "saved.txt"
    ops.tune_cache_save(str(out))
    assert f"320 320 15 8 {name}" in out.read_text().splitlines()
    bad = tmp_path / "bad.txt"
    bad.write_text(f"320 320 15 8 {name}\n320 320 15 8 no_such_schedule\n")
    with pytest.raises(MrxError, match="line 2"):
        ops.tune_cache_load(str(bad))
    with pytest.raises(MrxError):
        ops.tune_cache_load(str(tmp_path / "missing.txt"))
