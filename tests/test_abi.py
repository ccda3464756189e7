"""The C-ABI library loads and exports every entry point the header declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1905_09758_amd", "libnd.so")


def header_functions():
    text = open(os.path.join(ROOT, "include", "nd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1905_09758_amd import build
        build.build()
    import torch  # noqa: F401  (the HIP runtime torch ships)
    return ctypes.CDLL(LIB)


def test_header_declares_the_five_named_calls():
    fns = header_functions()
    for name in ("nd_build_csr", "nd_motif_filter", "nd_cheb_moments", "nd_ldos_moments", "nd_reconstruct"):
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in header_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_every_symbol(lib):
    import paper_1905_09758_amd as nd
    assert sorted(nd.EXPORTS) == header_functions()


def test_last_error_is_callable_without_device(lib):
    lib.nd_last_error.restype = ctypes.c_char_p
    assert lib.nd_last_error() == b""
