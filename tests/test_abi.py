"""The C-ABI library loads and exports every entry point its header declares (no GPU calls)."""
import ctypes as ct
import os
import re

import pytest

import paper_2009_00745_amd as lise

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lise.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lise_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_symbols():
    assert declared_symbols() == sorted(lise.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = lise.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_version_string():
    assert "gfx950" in lise.version()


class _Lat:
    def __init__(self, n, a=1.0):
        self.nx = self.ny = self.nz = n
        self.a = a


@pytest.mark.parametrize("n", [7, 11, 0, 256])
def test_unsupported_lattice_rejected_before_device_work(n):
    """Sizes with a prime factor > 5 (or out of range) fail in host validation."""
    import workloads as wl
    with pytest.raises(lise.LiseError, match="UNSUPPORTED"):
        lise.Context(_Lat(n), 4, wl.Functional(ncomp=2))


def test_bad_arguments_rejected():
    import workloads as wl
    with pytest.raises(lise.LiseError, match="ARG"):
        lise.Context(_Lat(8), 0, wl.Functional(ncomp=2))
    with pytest.raises(lise.LiseError, match="ARG"):
        lise.Context(_Lat(8), 4, wl.Functional(ncomp=3))
    with pytest.raises(lise.LiseError, match="ARG"):
        lise.Context(_Lat(8, a=-1.0), 4, wl.Functional(ncomp=2))
