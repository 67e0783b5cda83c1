"""CPU-side checks of the native library: it builds, loads and exports every
symbol the C header declares (no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2004_01729_amd", "libftcc.so")
HEADER = os.path.join(ROOT, "include", "ftcc.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ftcc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2004_01729_amd import build
        build.build_library()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("ftcc_set_hamiltonian", "ftcc_solve_amplitudes", "ftcc_grand_potential",
                     "ftcc_lambda", "ftcc_response"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_lists_match_header():
    from paper_2004_01729_amd import ftcc
    assert sorted(ftcc.exported_symbols()) == _declared()


def test_abi_version_and_error_string(lib):
    lib.ftcc_abi_version.restype = ctypes.c_int
    assert lib.ftcc_abi_version() == 6
    lib.ftcc_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.ftcc_last_error(), bytes)


def test_default_options(lib):
    from paper_2004_01729_amd import ftcc
    o = ftcc.default_options()
    assert (o.n_tau, o.nodes_per_panel, o.propagator, o.max_iter, o.checkpoint, o.diis_depth) == (16, 4, 0, 200, 0, 0)
    assert o.tol == 1e-12 and o.occ_thresh == 0.0 and o.mem_cap_bytes == 0 and o.spin_orbital == 0
