"""CPU checks of the C-ABI library: it loads and exports every entry point the
public header declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")
LIB = os.path.join(ROOT, "paper_2106_07616_amd", "librbffd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def library():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rbffd_build_stencils", "rbffd_assemble", "simple_step", "poisson_solve"):
        assert required in names


def test_library_exports_every_declared_symbol(library):
    for name in declared_functions():
        assert hasattr(library, name), name


def test_binding_covers_the_header():
    from paper_2106_07616_amd import binding
    assert sorted(binding.EXPORTED) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2106_07616_amd import binding
    with pytest.raises(ImportError):
        binding.load_library(str(tmp_path / "missing.so"))


def test_driver_tolerance_rule():
    from paper_2106_07616_amd.driver import outer_tolerance
    assert outer_tolerance(0.1, None, first=True) == 1e-4
    assert outer_tolerance(0.1, 1e-2, first=False) == pytest.approx(1e-3 if 1e-3 < 1e-4 else 1e-4)
    assert outer_tolerance(0.1, 1e-6, first=False) == pytest.approx(1e-7)
