"""Degenerate cases of the Krylov kernel and the step on the GPU against the
oracle.

Breakdown (Methods, section 6, eq. 34): the symmetric 4 x 4 matrices of a
1-atom system span 10 dimensions, so a rank-16 request must end at the grade
of the Krylov space of J (at most 10); the oracle and the GPU stop at the same
rank, and Y there is J^-1 W0 exactly (the oracle's full-rank pin), so the
residual is at rounding level.  A 2-atom system (36 dimensions) at rank 32
stays below its grade.  A call for zero MD steps leaves the state as it was.
"""

import numpy as np
import pytest

from synth import carbon_cluster
from oracle import model, density, krylov, dynamics

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-10


def t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def lib():
    from paper_2303_00689_amd import binding
    return binding


@pytest.mark.parametrize("n_atoms,m", [(1, 16), (2, 32)])
def test_krylov_rank_at_the_grade_matches_oracle(lib, n_atoms, m):
    s = carbon_cluster(n_atoms, 21)
    T_e = 3000.0
    beta = density.beta_of(T_e)
    n = s.n_orb
    rng = np.random.default_rng(n_atoms + 40)
    X = np.eye(n) * s.n_elec / n + 0.05 * rng.standard_normal((n, n))
    X = 0.5 * (X + X.T)
    h = lib.Handle(s.n_atoms, s.n_elec, s.onecenter, s.noise, s.params, T_e=T_e, m=m)
    try:
        h.set_geometry(t(s.R))
        F = torch.empty((n, n), dtype=torch.float64, device=DEV)
        h.fock(t(X), F, include_h=True)
        P = torch.empty_like(F)
        h.fermi_dm(F, P)
        Y = torch.empty_like(F)
        rank, rel = h.krylov_kernel(t(X), P, m, Y)
    finally:
        h.close()
    Fref = model.fock(X, s.R, s.onecenter, s.noise, s.params)
    dm = density.density_matrix(Fref, s.n_elec, beta)

    def jac(V):
        F1 = model.two_electron(V, s.R, s.onecenter, s.noise, s.params)
        return density.response(Fref, F1, s.n_elec, beta, dm) - V
    Yref, rref, relref = krylov.krylov_kernel(X, dm["P"], jac, m)
    dim = n * (n + 1) // 2
    print(f"{n_atoms} atom(s), m = {m}: rank GPU {rank}, oracle {rref} (symmetric dimension {dim}); "
          f"relres GPU {rel:.2e}, oracle {relref:.2e}")
    assert rank == rref
    if dim < m:
        assert rank <= dim < m          # the basis closed before rank m
        assert rel < 1e-10 and relref < 1e-10
    err = float(np.abs(Y.cpu().numpy() - Yref).max() / np.abs(Yref).max())
    assert err <= TOL, err


def test_zero_steps_leave_the_state(lib):
    from synth import workload
    s, w = workload("c10")
    st = dynamics.Settings(T_e=w["T_e"], m=w["m"], dt=w["dt"])
    n = s.n_orb
    X0 = np.eye(n) * s.n_elec / n
    o = dynamics.init_state(s, st, X0)
    h = lib.handle_for(s, w)
    try:
        h.set_geometry(t(s.R))
        state = lib.MDState(R=t(o.R), V=t(o.V), A=t(o.A), X=torch.stack([t(x) for x in o.Xhist]), Y=t(o.Y),
                            head=0, mu=o.mu)
        before = [x.clone() for x in (state.R, state.V, state.A, state.X, state.Y)]
        reps = h.step(state, 0)
        torch.cuda.synchronize()
        assert reps == []
        for a, b in zip(before, (state.R, state.V, state.A, state.X, state.Y)):
            assert torch.equal(a, b)
        assert state.head == 0
    finally:
        h.close()
