"""Non-orthogonal basis on the GPU against the oracle (Methods section 3,
eqs. 17-21, 36, 37, 41): the overlap S(R), the Loewdin factor Z = S^(-1/2),
the density matrix through Z, its response, and the Pulay force term, at 10
and 100 atoms for the default overlap and a stronger one, and at 840 atoms.

Bars: S to 1e-14 (its entries are at most 1; the two sides' exp differ in
the last bits); Z to 1e-12 of max|Z| and Z^T S Z = I to 1e-12; P, P1 and the
Pulay forces to 1e-10 of the largest reference entry, with mu to the bound
the electron count fixes it to, as in tests/test_gpu_parity.py.  One atom
(S = I, no Pulay term) and two atoms (one pair) are the smallest cases.  The eq. 37
forces for S != I are xlbomd_forces plus the Pulay term, against the oracle's
two parts.
"""

import numpy as np
import pytest

from synth import OverlapModel, carbon_cluster, workload
from oracle import model, density, dynamics, overlap

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-10
STRONG = OverlapModel(s0=0.15, r0=1.4, lam=0.5)


def t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def lib():
    from paper_2303_00689_amd import binding
    return binding


def run_case(lib, s, T_e, ov, seed=0, m=3, check_response=True, prec="fp64", p1_bar=None):
    beta = density.beta_of(T_e)
    n = s.n_orb
    rng = np.random.default_rng(seed)
    X = np.eye(n) * s.n_elec / n + 0.02 * rng.standard_normal((n, n))
    X = 0.5 * (X + X.T)
    h = lib.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, T_e=T_e, m=m, prec=prec)
    try:
        h.set_geometry(t(s.R))
        print(f"[nonorth] {s.n_atoms} atoms, s0 {ov.s0}, T_e {T_e:.0f} K, {prec}", flush=True)
        S = torch.empty((n, n), dtype=torch.float64, device=DEV)
        h.overlap(ov, S)
        Sref = overlap.overlap(s.R, ov)
        eS = float(np.abs(S.cpu().numpy() - Sref).max())
        Z = torch.empty_like(S)
        iters = h.lowdin(S, Z)
        Zg = Z.cpu().numpy()
        Zref = overlap.lowdin(Sref)
        eZ = rel(Zg, Zref)
        ortho = float(np.abs(Zg.T @ Sref @ Zg - np.eye(n)).max())
        F = torch.empty_like(S)
        h.fock(t(X), F, include_h=True)
        Fref = model.fock(X, s.R, s.onecenter, s.noise, s.params)
        P = torch.empty_like(S)
        mu, ent = h.fermi_dm_nonorth(F, Z, P)
        dm = overlap.density_matrix(Fref, Zref, s.n_elec, beta)
        # the entropy of eq. 4 from the occupations of F_perp's levels
        assert ent == pytest.approx(density.entropy(dm["f"]), rel=1e-9, abs=1e-9)
        Pg = P.cpu().numpy()
        eP = rel(Pg, dm["P"])
        f = dm["f"]
        dmu = 1e-11 * s.n_elec / (2.0 * beta * max(np.sum(f * (1.0 - f)), 1e-300))
        bar = TOL + min(beta * dmu, 1e-6)
        trPS = float(np.sum(Pg * Sref))
        out = dict(eS=eS, eZ=eZ, ortho=ortho, eP=eP, iters=iters)
        if check_response:
            V = rng.standard_normal((n, n))
            V = V + V.T
            F1 = model.two_electron(V, s.R, s.onecenter, s.noise, s.params)
            P1 = torch.empty_like(S)
            h.dm_response_nonorth(t(F1), Z, P1)
            out["eP1"] = rel(P1.cpu().numpy(), overlap.response(Fref, F1, Zref, s.n_elec, beta, dm))
        fp = torch.empty((s.n_atoms, 3), dtype=torch.float64, device=DEV)
        h.pulay_forces(ov, F, P, Z, fp)
        fref = overlap.pulay_forces(s.R, ov, Fref, dm["P"], Zref)
        out["ePulay"] = rel(fp.cpu().numpy(), fref)
        # eq. 37 with S != I: xlbomd_forces at (P0 = P, X) plus the Pulay term
        f37 = torch.empty_like(fp)
        h.forces(P, t(X), f37)
        ref37 = dynamics.forces(s.R, dm["P"], X, s.params, s.noise) + fref
        out["e37"] = rel(f37.cpu().numpy() + fp.cpu().numpy(), ref37)
    finally:
        h.close()
    print(f"  S {eS:.1e}, Z {eZ:.1e} ({iters} Newton-Schulz iterations), Z^T S Z - I {ortho:.1e}, "
          f"P {eP:.1e}, mu {mu:.8f} / {dm['mu']:.8f}, Tr PS - N_e {trPS - s.n_elec:.1e}, "
          + ", ".join(f"{k} {v:.1e}" for k, v in out.items() if k in ("eP1", "ePulay", "e37"))
          + f"; bar {bar:.1e}")
    assert eS <= 1e-14
    assert eZ <= 1e-12 and ortho <= 1e-12
    assert abs(mu - dm["mu"]) <= dmu + 1e-12
    assert abs(trPS - s.n_elec) <= 1e-9 * s.n_elec
    assert eP <= bar
    if check_response:
        assert out["eP1"] <= (bar if p1_bar is None else p1_bar)
    assert out["ePulay"] <= bar
    assert out["e37"] <= bar
    return out


@pytest.mark.parametrize("n_atoms,seed,T_e", [(1, 1, 3000.0), (2, 4, 3000.0), (10, 1, 3000.0), (100, 2, 5000.0)])
@pytest.mark.parametrize("ov", [OverlapModel(), STRONG], ids=["default", "strong"])
def test_nonorth_calls_match_oracle(lib, n_atoms, seed, T_e, ov):
    run_case(lib, carbon_cluster(n_atoms, seed), T_e, ov, seed=n_atoms)


@pytest.mark.parametrize("prec,p1_bar", [("dm64_bf16x3", 5e-4), ("dm64_bf16x6", 2e-5)])
def test_nonorth_mixed_precision(lib, prec, p1_bar):
    # FP64 transforms and density matrix (1e-10), split response chain: the
    # response is held to about three times its measured error (1.5e-4 and
    # 4.6e-6 of max|P1|), as the split-mode bounds of tests/test_gpu_split.py
    run_case(lib, carbon_cluster(100, 2), 5000.0, OverlapModel(), seed=5, prec=prec, p1_bar=p1_bar)


def test_nonorth_allones_pattern(lib):
    # the all-ones 10 x 10 pattern J of the two-centre blocks (every G term on)
    from synth import ModelParams
    s = carbon_cluster(100, 2, params=ModelParams(j_pattern="allones"))
    run_case(lib, s, 5000.0, STRONG, seed=9)


def test_nonorth_at_840_atoms(lib):
    s, w = workload("c840")
    run_case(lib, s, w["T_e"], OverlapModel(), seed=7, m=w["m"], check_response=False)


def test_identity_overlap_reduces_to_the_orthogonal_calls(lib):
    # s0 = 0: S = I, Z = I, and every call equals its orthogonal counterpart
    s = carbon_cluster(10, 1)
    n = s.n_orb
    rng = np.random.default_rng(3)
    X = np.eye(n) * s.n_elec / n + 0.02 * rng.standard_normal((n, n))
    X = 0.5 * (X + X.T)
    h = lib.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, T_e=3000.0, m=3)
    try:
        h.set_geometry(t(s.R))
        ov = OverlapModel(s0=0.0)
        S = torch.empty((n, n), dtype=torch.float64, device=DEV)
        h.overlap(ov, S)
        assert torch.equal(S, torch.eye(n, dtype=torch.float64, device=DEV))
        Z = torch.empty_like(S)
        h.lowdin(S, Z)
        assert float((Z - torch.eye(n, dtype=torch.float64, device=DEV)).abs().max()) <= 1e-15
        F = torch.empty_like(S)
        h.fock(t(X), F, include_h=True)
        P, P0 = torch.empty_like(S), torch.empty_like(S)
        h.fermi_dm_nonorth(F, Z, P)
        h.fermi_dm(F, P0)
        assert float((P - P0).abs().max()) <= 1e-13
        fp = torch.empty((s.n_atoms, 3), dtype=torch.float64, device=DEV)
        h.pulay_forces(ov, F, P, Z, fp)
        assert float(fp.abs().max()) == 0.0
    finally:
        h.close()


def test_nonorth_arguments(lib):
    s = carbon_cluster(4, 1)
    n = s.n_orb
    h = lib.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, T_e=3000.0, m=3)
    try:
        S = torch.empty((n, n), dtype=torch.float64, device=DEV)
        with pytest.raises(lib.XLBOMDError):
            h.overlap(OverlapModel(), S)                     # positions not set
        h.set_geometry(t(s.R))
        with pytest.raises(lib.XLBOMDError):
            h.overlap(OverlapModel(lam=0.0), S)
        with pytest.raises(lib.XLBOMDError):
            h.lowdin(S, S)                                   # Z aliases S
        # an indefinite "overlap" is refused
        with pytest.raises(lib.XLBOMDError):
            h.lowdin(t(-np.eye(n)), torch.empty_like(S))
        P1 = torch.empty_like(S)
        with pytest.raises(lib.XLBOMDError):
            h.dm_response_nonorth(S, S.clone(), P1)           # no chain cached
        # a chain of the orthogonal call is not the one the response differentiates
        X = t(np.eye(n) * s.n_elec / n)
        F = torch.empty_like(S)
        h.fock(X, F, include_h=True)
        h.fermi_dm(F, torch.empty_like(S), entropy=False)
        with pytest.raises(lib.XLBOMDError):
            h.dm_response_nonorth(F, t(np.eye(n)), P1)
    finally:
        h.close()
