"""xlbomd_spectral_bounds_noalloc (no handle, scratch in a static device
array) against xlbomd_spectral_bounds on a handle: the same bounds, bit for
bit, on two calls in a row, the second with a smaller input, and n beyond the
stated maximum refused before any work."""

import numpy as np
import pytest

from synth import workload
from oracle import model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2303_00689_amd import binding
    return binding


def _fock(name, seed):
    s, w = workload(name)
    n = s.n_orb
    rng = np.random.default_rng(seed)
    X = np.eye(n) * s.n_elec / n + 0.02 * rng.standard_normal((n, n))
    X = 0.5 * (X + X.T)
    return s, w, model.fock(X, s.R, s.onecenter, s.noise, s.params)


def test_noalloc_bounds_equal_the_handle_bounds(lib):
    dev = torch.device("cuda:0")
    for name in ("c100", "c10"):          # the second call is the smaller one
        s, w, F = _fock(name, 5)
        Fd = torch.tensor(F, dtype=torch.float64, device=dev)
        lo, hi = lib.spectral_bounds_noalloc(Fd)
        h = lib.handle_for(s, w)
        try:
            lo_h, hi_h = h.spectral_bounds(Fd)
        finally:
            h.close()
        eps = np.linalg.eigvalsh(F)
        print(f"{name}: noalloc [{lo!r}, {hi!r}], handle [{lo_h!r}, {hi_h!r}], spectrum [{eps[0]:.6f}, {eps[-1]:.6f}]")
        assert lo == lo_h and hi == hi_h
        assert lo <= eps[0] and hi >= eps[-1]


def test_noalloc_refuses_sizes_beyond_its_scratch(lib):
    n = lib.SPECTRAL_BOUNDS_NOALLOC_MAX_N + 4
    # the size check comes before any access to F: a 1 x 1 tensor stands in
    F = torch.zeros((1, 1), dtype=torch.float64, device="cuda:0")
    lohi = (lib.C.c_double * 2)()
    st = lib.load().xlbomd_spectral_bounds_noalloc(lib.C.c_void_p(F.data_ptr()), n, None, lohi)
    assert st == -1
    st = lib.load().xlbomd_spectral_bounds_noalloc(lib.C.c_void_p(F.data_ptr()), 0, None, lohi)
    assert st == -1
