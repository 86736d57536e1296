"""The C-ABI library loads without a GPU and exports every function that
include/pabd.h declares (no compute calls are made here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pabd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pabd_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2609_02675_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2609_02675_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.SYMBOLS)


def test_device_count_and_scene_bytes_work_without_a_gpu():
    import paper_2609_02675_amd as P
    from paper_2609_02675_amd import scenes as S
    assert P.device_count() >= 0
    b32 = P.scene_bytes(S.chain8(precision=S.PREC_FP32))
    b64 = P.scene_bytes(S.chain8(precision=S.PREC_FP64))
    assert 0 < b32 < b64
    bad = S.chain8().copy(h=-1.0)
    assert P.scene_bytes(bad) == 0
