"""The built library exports every function include/xlbomd.h declares (no GPU
needed: nothing is called), and the binding rejects bad arguments on the host."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2303_00689_amd", "libxlbomd.so")


def _declared():
    text = open(os.path.join(ROOT, "include", "xlbomd.h")).read()
    return sorted(set(re.findall(r"\b(xlbomd_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2303_00689_amd import build
        build.build()
    return LIB


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("xlbomd_fock", "xlbomd_fermi_dm", "xlbomd_dm_response",
                     "xlbomd_krylov_kernel", "xlbomd_step"):
        assert required in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (xlbomd_[a-z_0-9]+)", out))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing


def test_binding_symbol_list_matches_header(built):
    from paper_2303_00689_amd import binding
    assert sorted(binding.SYMBOLS) == _declared()


def test_library_loads_without_gpu(built):
    from paper_2303_00689_amd import binding
    lib = binding.load()
    assert lib.xlbomd_n_orb(None) == 0
    assert lib.xlbomd_destroy(None) == -1
