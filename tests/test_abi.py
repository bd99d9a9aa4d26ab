"""The C-ABI library loads and exports every symbol include/lfem.h declares
(no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lfem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lfem_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("lfem_mesh_create", "lfem_pattern_build", "lfem_assemble_mass",
                     "lfem_assemble_stiffness", "lfem_assemble_weighted", "lfem_assemble_batch",
                     "lfem_batch_create", "lfem_shape_grad", "lfem_energy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2605_14035_amd import _lib
    L = _lib.load()
    names = declared_symbols()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(_lib.EXPORTS)


def test_version_string_without_gpu():
    import paper_2605_14035_amd as lf
    assert "gfx950" in lf.lfem_version()
    assert lf.lfem_last_error() == ""


def test_host_only_calls_without_gpu():
    """The calls that touch no device: the tuning cache reset and the debug
    switch (its round trip returns the previous setting)."""
    import paper_2605_14035_amd as lf
    lf.lfem_tune_cache_clear()
    prev = lf.lfem_set_debug(True)
    assert lf.lfem_set_debug(False) is True
    lf.lfem_set_debug(prev)


def test_no_oracle_in_product_path():
    """The package never imports the oracle (they share no code)."""
    pkg = os.path.join(ROOT, "paper_2605_14035_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "lfem_oracle" not in src, f
