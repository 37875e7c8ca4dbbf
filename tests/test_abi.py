"""CPU-side checks of the C ABI: the library loads, exports every function
include/ddilu.h declares, and its host-only sizing rule agrees with the
oracle's statement of the same rule (no device calls)."""

import ctypes
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddilu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dd_partition", "ilu0_factor", "dd_trsv_apply", "bicgstab_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2508_04917_amd import ddilu
    lib = ctypes.CDLL(ddilu.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(ddilu.EXPORTS) == declared_functions()


@pytest.mark.parametrize("dims,bs,lds,ncu", [
    ((160, 160, 160), 3, 160 * 1024, 256), ((64, 64, 64), 3, 160 * 1024, 256),
    ((128, 128, 128), 3, 160 * 1024, 256), ((16, 16, 16), 1, 160 * 1024, 256),
    ((48, 48, 48), 3, 160 * 1024, 256), ((128, 128, 256), 1, 64 * 1024, 104),
    ((30, 12, 7), 3, 20000, 8), ((5, 5, 5), 3, 100, 4)])
def test_auto_subdims_matches_oracle(dims, bs, lds, ncu):
    from paper_2508_04917_amd import ddilu
    expect = O.auto_subdims(*dims, bs, lds, ncu)
    if expect is None:
        with pytest.raises(ddilu.DDError):
            ddilu.dd_auto_subdims(*dims, bs, lds, ncu)
    else:
        assert ddilu.dd_auto_subdims(*dims, bs, lds, ncu) == expect


def test_no_oracle_in_product_path():
    """The GPU package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2508_04917_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "liboracle" not in src and "from oracle" not in src, f
