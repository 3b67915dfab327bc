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


# binding struct -> C struct name
_STRUCTS = {"Model": "xlbomd_model", "System": "xlbomd_system", "Params": "xlbomd_params",
            "MDStateC": "xlbomd_md_state", "Report": "xlbomd_report", "SCFParams": "xlbomd_scf_params",
            "SCFReport": "xlbomd_scf_report", "OverlapModelC": "xlbomd_overlap_model"}


def test_binding_structs_match_header_layout(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets the C
    compiler gives the header's struct (a mismatch would pass wrong values
    through the ABI without any error)."""
    from paper_2303_00689_amd import binding
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "xlbomd.h"', 'int main(void) {']
    for py, cname in _STRUCTS.items():
        lines.append(f'  printf("{py} size %zu\\n", sizeof({cname}));')
        for field, _ in getattr(binding, py)._fields_:
            lines.append(f'  printf("{py} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-x", "c", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        py, field, value = line.split()
        cls = getattr(binding, py)
        got = C_sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), (py, field, got, value)


def C_sizeof(cls):
    import ctypes
    return ctypes.sizeof(cls)


def test_create_rejects_bad_arguments_before_any_device_call(built):
    """Argument checks of xlbomd_create come before any HIP call, so they run
    without a GPU: sizes outside 1..8191 atoms, electron counts outside
    (0, 2n), a non-positive temperature, an out-of-range rank."""
    import ctypes as C
    from paper_2303_00689_amd import binding
    lib = binding.load()
    oc = (C.c_double * 5)()
    nz = (C.c_float * 55)()

    def create(n_atoms=2, n_elec=8.0, T_e=3000.0, m=4, w0_limit=0.0, T_ion_limit=0.0):
        sysc = binding.System(n_atoms=n_atoms, n_elec=n_elec,
                              onecenter=C.cast(oc, C.POINTER(C.c_double)),
                              noise55=C.cast(nz, C.POINTER(C.c_float)))
        prm = binding.Params(prec=0, T_e=T_e, m=m, dt=0.5, kappa=1.84, alpha=0.0055, kernel_c=1.0,
                             w0_limit=w0_limit, T_ion_limit=T_ion_limit)
        h = C.c_void_p(1234)
        st = lib.xlbomd_create(C.byref(sysc), C.byref(prm), None, C.byref(h))
        return st, h.value

    for kw in (dict(n_atoms=0), dict(n_atoms=-3), dict(n_atoms=8192), dict(n_elec=0.0),
               dict(n_elec=16.0), dict(n_elec=float("nan")), dict(T_e=0.0), dict(m=-1), dict(m=33),
               dict(w0_limit=-1.0), dict(T_ion_limit=float("nan"))):
        st, h = create(**kw)
        assert st == -1, kw
        assert h is None, kw


def test_binding_refuses_noise_that_fp32_does_not_hold(built):
    """The ABI takes the two-centre noise in FP32; the binding refuses FP64
    noise that would be rounded (before any device call)."""
    import numpy as np
    from paper_2303_00689_amd import binding
    from synth import carbon_cluster
    s = carbon_cluster(3, 1)
    bad = s.noise.astype(np.float64) + 1e-12
    with pytest.raises(binding.XLBOMDError):
        binding.Handle(s.n_atoms, s.n_elec, s.onecenter, bad, s.params)
