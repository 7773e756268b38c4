"""The C ABI library loads and exports every entry point of include/pp.h
(no compute calls, so this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pp.h")
LIB = os.path.join(ROOT, "paper_2512_12094_amd", "libpp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pp_create", "pp_apply_layer", "pp_merge_canonicalize", "pp_truncate",
                     "pp_expectation", "pp_num_terms", "pp_export_terms", "pp_destroy",
                     "pp_last_error", "pp_batch_run"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpp.so not built")
def test_binding_names_match_the_header():
    from paper_2512_12094_amd import _lib
    for n in declared_functions():
        if n in ("pp_last_error",):
            continue
        assert hasattr(_lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpp.so not built")
def test_argument_errors_need_no_gpu():
    """Validation happens on the host before any device call."""
    from paper_2512_12094_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.pp_create(ctypes.byref(h), 0, 0, 0, None, None, None, 0, None, None) == -1
    assert b"unsupported" in L.pp_last_error()
    assert L.pp_create(ctypes.byref(h), 65, 1, 0, None, None, None, 0, None, None) == -1
    assert L.pp_create(ctypes.byref(h), 8, 1, 7, None, None, None, 0, None, None) == -1
    assert L.pp_set_tuning(3, 0, 0, 0, 0) == -1
    assert L.pp_set_tuning(0, 16, 0, 0, 0) == -1
    assert L.pp_set_tuning(0, 0, 0, 0, 65) == -1
    for bad in ((4, 0), (-1, 0), (3, 2)):
        assert L.pp_set_gate_fusion(*bad) == -1
    assert L.pp_set_gate_fusion(3, 0) == 0
    assert L.pp_program_info(None, None) == -1


def test_explicit_group_list_is_validated_on_the_host():
    """pp_create_group rejects lists that are not a group before any device
    work (no GPU needed)."""
    import numpy as np
    from paper_2512_12094_amd import _lib as L
    one = dict(obs_x=np.array([[1]], dtype=np.uint64), obs_z=np.array([[0]], dtype=np.uint64),
               obs_coef=np.array([1.0]))
    bad = {
        "not a permutation": [[0, 1, 2], [0, 0, 2]],
        "no identity": [[1, 2, 0], [2, 0, 1]],
        "not closed": [[0, 1, 2], [1, 2, 0]],
        "repeated": [[0, 1, 2], [0, 1, 2]],
    }
    for why, perms in bad.items():
        with pytest.raises(L.PPError) as e:
            L.pp_create_group(3, perms, **one)
        assert e.value.code == -1, why


def test_autotune_knobs_round_trip():
    """The autotuner's knob families reach their setters and read back
    (host-side calls only)."""
    from paper_2512_12094_amd import autotune as A
    before = A.get_knobs()
    try:
        A.set_knobs(dict(layer_shift=6, layer_block=256, part_shift=13, part_agg_blocks=512,
                         gate_items=2))
        now = A.get_knobs()
        assert now["layer_shift"] == 6 and now["layer_block"] == 256
        assert now["part_shift"] == 13 and now["part_agg_blocks"] == 512
        assert now["gate_items"] == 2 and now["max_blocks"] == before["max_blocks"]
    finally:
        A.set_knobs(before)
    assert A.get_knobs() == before
