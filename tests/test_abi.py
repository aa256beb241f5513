"""The C ABI library loads and exports every symbol include/hyperim.h declares
(no compute calls: this runs without a GPU), and the binding refuses to work
without it."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperim.h")
LIB = os.path.join(ROOT, "paper_2406_01911_amd", "libhyperim.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hyperim_[a-z_]+)\s*\(", text)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2406_01911_amd import build as b  # noqa: F401
        import importlib
        importlib.import_module("paper_2406_01911_amd.build").build()


def test_header_declares_the_four_hot_path_calls():
    names = _declared()
    for n in ["hyperim_build_graph", "hyperim_stratify", "hyperim_generate_rr", "hyperim_select_seeds"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], stdout=subprocess.PIPE, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (hyperim_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches_exports():
    _ensure_built()
    import torch  # noqa: F401  (binds the HIP runtime first)
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n)
    import paper_2406_01911_amd as hy
    assert sorted(hy.EXPORTS) == _declared()
    lib.hyperim_strerror.restype = ctypes.c_char_p
    assert lib.hyperim_strerror(-3).decode().startswith("pool capacity")


def test_binding_raises_without_library(tmp_path):
    import paper_2406_01911_amd as hy
    saved = hy._lib
    hy._lib = None
    try:
        with pytest.raises(ImportError):
            hy.load_library(str(tmp_path / "missing.so"))
    finally:
        hy._lib = saved


def test_invalid_arguments_rejected_before_any_device_work():
    _ensure_built()
    import paper_2406_01911_amd as hy
    import numpy as np
    hy.load_library()
    with pytest.raises(hy.HyperIMError) as e:
        hy.build_graph(0, np.array([0], np.uint32), np.zeros(0, np.uint32), hy.MODEL_CONST, 0.1)
    assert e.value.status == hy.EINVAL
    with pytest.raises(hy.HyperIMError) as e:
        hy.build_graph(3, np.array([0, 2], np.uint32), np.array([0, 1], np.uint32), hy.MODEL_CONST, float("nan"))
    assert e.value.status == hy.EINVAL
    with pytest.raises(hy.HyperIMError) as e:
        hy.build_graph(3, np.array([0, 2], np.uint32), np.array([0, 1], np.uint32), 7, 0.1)
    assert e.value.status == hy.EINVAL
    for model in (hy.MODEL_LT_CONST, hy.MODEL_GAPS_CONST):
        with pytest.raises(hy.HyperIMError) as e:
            hy.build_graph(3, np.array([0, 2], np.uint32), np.array([0, 1], np.uint32), model, -0.25)
        assert e.value.status == hy.EINVAL


def test_model_constants_match_the_header():
    """The binding's and the input generator's model numbers are the header's."""
    import hypergen
    import paper_2406_01911_amd as hy
    text = open(HEADER).read()
    header = {k: int(v) for k, v in re.findall(r"#define HYPERIM_(MODEL_\w+) (\d+)u", text)}
    assert sorted(header.values()) == list(range(7))
    for name, value in header.items():
        assert getattr(hy, name) == value, name
        assert getattr(hypergen, name) == value, name
