"""The C-ABI library loads and exports every function include/nlome.h
declares (no compute call: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nlome.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nlo_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2503_07439_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert "nlo_me2" in names and "nlo_create" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps every declared function under the same name
    assert set(names) <= set(_lib.SIGNATURES)


def test_abi_version_and_process_table():
    import paper_2503_07439_amd as nl
    assert nl.nlo_abi_version() == 2
    assert nl.nlo_num_processes() == len(nl.PROCESSES)


def test_process_info_without_device():
    import paper_2503_07439_amd as nl
    want = {"ee_mumu": (1, 1, 4), "ee_uug": (2, 1, 8), "gg_tt": (3, 2, 16), "uu_tt": (1, 2, 8),
            "gg_ttg": (16, 6, 32), "uu_ttg": (5, 4, 16), "ug_ttu": (5, 4, 16), "gg_ttgg": (123, 24, 64)}
    for name, (nd, nc, ng) in want.items():
        info = nl.nlo_process_info(None, nl.proc_id(name))
        assert info.name.decode() == name
        assert (info.ndiagrams, info.ncolour, info.ngood_hel) == (nd, nc, ng)
    info = nl.nlo_process_info(None, nl.proc_id("gg_ttgg"))
    assert info.ident_factor == 0.5 and info.avg_factor == 1.0 / 256


def test_argument_errors_without_device():
    import paper_2503_07439_amd as nl
    import pytest
    with pytest.raises(nl.NloError) as e:
        nl.nlo_process_info(None, 42)
    assert e.value.status == 2
    assert "unknown process" in nl.nlo_last_error()
    with pytest.raises(nl.NloError) as e:
        nl.nlo_me2(None, 0, 1, 1, 0, 0, 0, 0)
    assert e.value.status == 1
