"""The C-ABI library loads without a GPU and exports every function that
include/lg.h declares; the Python binding covers exactly those names."""

import ctypes
import os
import re

from paper_2010_15879_amd import lg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lg_\w+)\s*\(", text, flags=re.M))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lg_encode", "lg_decode_neighbors", "lg_bfs", "lg_pagerank", "lg_free"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lg.LIB_PATH)
    for name in sorted(declared_functions()):
        assert hasattr(L, name), name


def test_binding_matches_header():
    assert set(lg.FUNCTIONS) == declared_functions()
    lg.lib()


def test_struct_layouts():
    # lg_encode_opts: 8 uint32; lg_graph_info: fields in header order
    assert ctypes.sizeof(lg.EncodeOpts) == 32
    assert ctypes.sizeof(lg.GraphInfo) == 2 * 8 + 8 * 4 + 8 * 8 + 4 * 4 + 3 * 8 + 2 * 4 + 8


def test_oracle_is_not_reachable_from_the_product():
    pkg = os.path.join(ROOT, "paper_2010_15879_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("Oracle", "").lower() or f == "graphgen.py", f


def test_weights_length_checked_before_the_library():
    import pytest
    import torch
    off = torch.tensor([0, 1, 2], dtype=torch.int64)
    col = torch.tensor([1, 0], dtype=torch.int32)
    with pytest.raises(ValueError):
        lg.encode(off, col, 2, weights=torch.ones(3, dtype=torch.int32))
