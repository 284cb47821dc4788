"""The C-ABI library loads and exports every entry point of include/ftn.h."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "ftn.h")).read()
    return sorted(set(re.findall(r"\b(ftn_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = header_symbols()
    for name in ["ftn_tensor_create", "ftn_ftranspose", "ftn_ftensordot", "ftn_compress_bond",
                 "ftn_contract_network", "ftn_net_create", "ftn_fuse", "ftn_flip_dual"]:
        assert name in syms


def test_library_exports_every_header_symbol():
    import ctypes
    path = os.path.join(ROOT, "paper_2410_02215_amd", "libftn.so")
    if not os.path.exists(path):
        pytest.fail("libftn.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2410_02215_amd import ftn
    declared = {n for n, _, _ in ftn.SIGNATURES}
    assert set(header_symbols()) == declared
    lib = ftn.load_library()
    assert lib.ftn_version().startswith(b"ftn")


def test_autotune_table_host_logic(tmp_path):
    # mode checks and the JSON table round trip need no device
    from paper_2410_02215_amd import ftn
    ftn.load_library()
    with pytest.raises(ftn.FtnError):
        ftn.autotune(3)
    p = os.path.join(str(tmp_path), "t.json")
    with open(p, "w") as f:
        f.write('{\n "version": 1,\n "entries": {\n  "k0-m9-n9-k9-g1-s0-x1": [1, 1, 12.5],\n'
                '  "k1-m4-n8-k12-g2-s0-x0": [4, 3, 7.25]\n }\n}\n')
    before = ftn.autotune_stats()["entries"]
    ftn.autotune_load(p)
    q = os.path.join(str(tmp_path), "u.json")
    ftn.autotune_save(q)
    import json
    ent = json.load(open(q))["entries"]
    assert ent["k0-m9-n9-k9-g1-s0-x1"] == [1, 1, 12.5] and ent["k1-m4-n8-k12-g2-s0-x0"] == [4, 3, 7.25]
    assert ftn.autotune_stats()["entries"] >= max(before, 2)
    with open(p, "w") as f:
        f.write('{"entries": {\n  "bad": [9, 1, 1.0]\n}}\n')
    with pytest.raises(ftn.FtnError):
        ftn.autotune_load(p)
    ftn.autotune(0)
