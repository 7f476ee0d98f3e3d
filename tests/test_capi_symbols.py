"""The C-ABI library loads without a GPU and exports every function that
include/symhss.h declares; the binding's struct layouts match the header's
sizes.  No compute call is made here."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symhss.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(symhss_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2609_33216_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2609_33216_amd.build import build
        build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2609_33216_amd import binding
    assert sorted(binding.EXPORTS) == _declared()


def test_struct_sizes():
    from paper_2609_33216_amd import binding
    # symhss_medium: 4 doubles; symhss_opts: 2 int32 + double + 2 int32 + double
    assert ctypes.sizeof(binding.Medium) == 32
    assert ctypes.sizeof(binding.Opts) == 32
    assert binding.Opts.proxy_ratio.offset == 24
    assert ctypes.sizeof(binding.Stats) % 8 == 0


def test_null_context_is_rejected(lib):
    # argument checks on the host side of the boundary, no device work
    assert lib.symhss_compress(None) == 1
    assert lib.symhss_factor(None) == 1
    assert lib.symhss_get_stats(None, None) == 1
