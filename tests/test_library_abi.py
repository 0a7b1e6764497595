"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tapt.h")
LIB = os.path.join(ROOT, "paper_2509_23043_amd", "libtapt.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["pt_create", "pt_sweep", "pt_propose", "pt_energies", "pt_state", "pt_destroy",
              "pt_batch_create", "pt_batch_sweep", "pt_last_error"]:
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtapt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtapt.so not built")
def test_binding_loads_and_matches_header():
    from paper_2509_23043_amd import binding
    L = binding.lib()
    assert set(binding.EXPORTS) <= set(declared_symbols())
    for s in binding.EXPORTS:
        assert hasattr(L, s)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2509_23043_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.lib()


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2509_23043_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.c" not in text and "liboracle" not in text, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtapt.so not built")
def test_overlong_acceptance_table_is_refused_not_truncated():
    """A swap table longer than the library's cap (a ladder spaced by 1e-6,
    whose Eq. 1 table runs to about 2.2e7 entries) makes pt_create fail with
    PT_EUNSUPPORTED. The tables are built on the host before any device call,
    so this runs without a GPU."""
    import numpy as np

    from paper_2509_23043_amd import binding, inputs
    g = inputs.ea_lattice(4, 1)
    betas = 1.0 + 1e-6 * np.arange(4)
    with pytest.raises(binding.TaptError) as e:
        binding.Context(g, betas, seed=1)
    assert e.value.code == binding.PT_EUNSUPPORTED
    assert "swap table of pair (0, 1)" in str(e.value)
