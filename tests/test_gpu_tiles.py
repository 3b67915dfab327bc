"""The GEMM tile table (xlbomd_set_tile_table) and the timing call of the
autotuner (xlbomd_time_gemm).

Both kernel families are run through the handle's matmul with the table
forcing one or the other: in FP64 they give the same bits on and above the
diagonal (every such element sums its k terms in the same order in both
tilings; below the diagonal of a symmetric output one family mirrors where
the other computes the diagonal tiles' lower halves); in split
precision each stays within the split arithmetic's budget of
tests/test_gpu_split.py, with the FP32-accumulation term at these sizes.
Orders cover one tile, ragged last tiles (and, for the medium tiles, a ragged
last k panel: n % 32 != 0) and several tiles of each family.
"""

import numpy as np
import pytest

from synth import carbon_cluster

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MM_BOUND = {"fp64": 1e-13, "bf16x3": 5e-5, "bf16x6": 2.5e-6, "fp16x3": 1.5e-6}
PREC = {"fp64": 0, "bf16x3": 1, "bf16x6": 2, "fp16x3": 3}


@pytest.fixture(scope="module")
def binding():
    from paper_2303_00689_amd import binding as b
    yield b
    b.install_tile_table()   # back to the table the library loads with


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _product(binding, h, A, B, sym, prec, family):
    n = A.shape[0]
    binding.set_tile_table([[prec, sym, 1 << 20, family]])
    dev = torch.device("cuda:0")
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    h.matmul(torch.tensor(A, device=dev), torch.tensor(B, device=dev), C, sym_out=bool(sym))
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("mode", ["fp64", "bf16x3", "bf16x6", "fp16x3"])
@pytest.mark.parametrize("n_atoms", [32, 37, 100, 264, 840])
@pytest.mark.parametrize("sym", [0, 1])
def test_families_agree(binding, mode, n_atoms, sym):
    s = carbon_cluster(n_atoms, 3)
    n = s.n_orb        # 128, 148, 400, 1056, 3360: one tile, ragged tiles and k, several, full size
    h = binding.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, prec=mode)
    try:
        rng = np.random.default_rng(n + 5)
        A = rng.uniform(-0.5, 0.5, (n, n))
        A = 0.5 * (A + A.T)
        B = A @ A / n + np.eye(n) if sym else rng.uniform(-0.5, 0.5, (n, n))
        prec = PREC[mode]
        small = _product(binding, h, A, B, sym, prec, binding.GEMM_SMALL)
        large_runs = binding.time_gemm(n, prec, sym, binding.GEMM_LARGE, 1) is not None
        large = _product(binding, h, A, B, sym, prec, binding.GEMM_LARGE) if large_runs else None
        mid_runs = prec != 0 and binding.time_gemm(n, prec, sym, binding.GEMM_MEDIUM, 1) is not None
        mid = _product(binding, h, A, B, sym, prec, binding.GEMM_MEDIUM) if mid_runs else None
        cpt = _product(binding, h, A, B, sym, prec, binding.GEMM_COMPACT)
    finally:
        binding.set_tile_table([])
        h.close()
    if mode == "fp64":
        ref = A @ B
        assert _rel(small, ref) <= MM_BOUND[mode]
        # compact tiles sum every element's k terms in the same order as the
        # small ones: the same bits on and above the diagonal
        iu = np.triu_indices(n)
        assert np.array_equal(small[iu], cpt[iu])
        if not sym:
            assert np.array_equal(small, cpt)
        if large is not None:
            assert _rel(large, ref) <= MM_BOUND[mode]
            if sym:
                # symmetric outputs: the entries on and above the diagonal are
                # the same products; below it the small tiles compute the
                # diagonal tiles' lower halves, the large ones mirror
                iu = np.triu_indices(n)
                assert np.array_equal(small[iu], large[iu])
                assert np.array_equal(large, large.T)
            else:
                assert np.array_equal(small, large)
        return
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    ref = A32 @ B32
    S = float((np.abs(A32) @ np.abs(B32)).max())
    acc = 4.0 * np.sqrt(n) * 2.0**-24 * S / np.abs(ref).max()
    for name, C in (("small", small), ("large", large), ("medium", mid), ("compact", cpt)):
        if C is None:
            continue
        err = _rel(C, ref)
        print(f"{mode} n={n} sym={sym} {name} tiles: rel err {err:.2e}")
        assert err <= MM_BOUND[mode] + acc


def test_time_gemm_and_table_arguments(binding):
    # a family that cannot run n is refused by the timer; a timed product is positive
    assert binding.time_gemm(400, 1, 0, binding.GEMM_LARGE, 1) is None       # 400 % 32 != 0
    assert binding.time_gemm(1040, 0, 1, binding.GEMM_LARGE, 1) > 0.0        # 1040 % 16 == 0
    assert binding.time_gemm(96, 0, 0, binding.GEMM_LARGE, 1) is None        # below 128
    assert binding.time_gemm(256, 3, 0, binding.GEMM_LARGE, 1) > 0.0        # FP16x3: 160-row tiles
    assert binding.time_gemm(400, 3, 1, binding.GEMM_MEDIUM, 1) is None      # FP16x3 medium: n % 32 == 0
    assert binding.time_gemm(256, 3, 0, binding.GEMM_SMALL, 1) > 0.0
    assert binding.time_gemm(256, 0, 0, binding.GEMM_MEDIUM, 1) is None      # split only
    assert binding.time_gemm(400, 2, 1, binding.GEMM_MEDIUM, 1) > 0.0       # ragged last k panel
    assert binding.time_gemm(402, 1, 1, binding.GEMM_MEDIUM, 1) is None      # 402 % 4 != 0
    assert binding.time_gemm(416, 1, 1, binding.GEMM_MEDIUM, 1) > 0.0
    assert binding.time_gemm(148, 3, 1, binding.GEMM_COMPACT, 1) > 0.0       # ragged, FP16x3 too
    assert binding.time_gemm(60, 1, 1, binding.GEMM_COMPACT, 1) is None       # below 64
    assert binding.time_gemm(256, 0, 0, binding.GEMM_COMPACT, 1) > 0.0       # FP64 32-row tiles
    for bad in ([[4, 0, 100, 1]], [[0, 2, 100, 1]], [[0, 0, 0, 1]], [[0, 0, 100, 5]],
                [[0, 0, 100, 1]] * (binding.TILE_TABLE_MAX + 1)):
        with pytest.raises(binding.XLBOMDError):
            binding.set_tile_table(bad)
    binding.set_tile_table([])


def test_installed_table_rows_are_valid(binding):
    # the committed table (if any) is well formed and every row's family exists
    import json
    import os
    if not os.path.exists(binding.TILE_TABLE_PATH):
        pytest.skip("no tile table installed")
    with open(binding.TILE_TABLE_PATH) as f:
        rows = json.load(f)["rows"]
    assert 0 < len(rows) <= binding.TILE_TABLE_MAX
    binding.set_tile_table(rows)
    binding.set_tile_table([])
