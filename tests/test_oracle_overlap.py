"""Pins of oracle/overlap.py (non-orthogonal basis, Methods section 3,
eqs. 18-21, 36, 41) against what the mathematics fixes, not against its own
formulas:

* S(R): symmetric with unit atom blocks, equal to I when s0 = 0, invariant
  under translation and covariant under rotation (the s orbital is a scalar,
  the p orbitals a vector: rotating the geometry by Q turns each p block by
  Q), and its derivative blocks agree with central differences of S(R);
* Loewdin Z: Z^T S Z = I (eq. 21) and Z = S^(-1/2) by scipy's matrix square
  root;
* density matrix (eqs. 18-20): equal to the one built from scipy's
  generalized eigensolver F C = S C eps (C^T S C = I), and the same for
  another Z of eq. 21 (the Cholesky factor Z = L^-T); Tr P S = N_e;
* response (eq. 36): central differences of the density matrix, Tr P1 S = 0,
  and the same for the Cholesky Z;
* Pulay term (eq. 41): minus the derivative of the spin-summed grand
  potential of F C = S C eps, at fixed F and mu, through S(R), by central
  differences; a dropped factor, a sign, or F P in the wrong order fails it.
"""

import numpy as np
import pytest
import scipy.linalg

from synth import OverlapModel, carbon_cluster
from oracle import overlap, density, model

OV = OverlapModel()
STRONG = OverlapModel(s0=0.15, r0=1.4, lam=0.5)


def _system(n_atoms=6, seed=3):
    return carbon_cluster(n_atoms, seed)


def _fock(s, rng, scale=0.02):
    n = s.n_orb
    X = np.eye(n) * s.n_elec / n + scale * rng.standard_normal((n, n))
    X = 0.5 * (X + X.T)
    return model.fock(X, s.R, s.onecenter, s.noise, s.params)


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("ov", [OV, STRONG])
def test_overlap_structure_and_symmetries(ov):
    s = _system(8, 5)
    S = overlap.overlap(s.R, ov)
    N = s.n_atoms
    assert np.array_equal(S, S.T)
    Sb = S.reshape(N, 4, N, 4)
    for A in range(N):
        assert np.array_equal(Sb[A, :, A, :], np.eye(4))
    assert np.linalg.eigvalsh(S)[0] > 0.3
    assert np.array_equal(overlap.overlap(s.R, OverlapModel(0.0, 1.4, 0.4)), np.eye(4 * N))
    # translation
    assert np.allclose(overlap.overlap(s.R + np.array([0.3, -1.2, 2.0]), ov), S, rtol=0, atol=1e-15)
    # rotation: S(R Q^T) = U S(R) U^T with U = diag over atoms of [1, Q]
    Q = _rotation(7)
    U1 = np.eye(4)
    U1[1:, 1:] = Q
    U = np.kron(np.eye(N), U1)
    assert np.abs(overlap.overlap(s.R @ Q.T, ov) - U @ S @ U.T).max() <= 1e-14


def test_overlap_derivative_blocks_match_central_differences():
    s = _system(5, 9)
    N = s.n_atoms
    a, b, dS = overlap.overlap_derivative_blocks(s.R, STRONG)
    h = 1e-5
    for p in range(a.size):
        for k in range(3):
            Rp, Rm = s.R.copy(), s.R.copy()
            Rp[b[p], k] += h
            Rm[b[p], k] -= h
            fd = (overlap.overlap(Rp, STRONG) - overlap.overlap(Rm, STRONG)).reshape(N, 4, N, 4)[a[p], :, b[p], :]
            assert np.abs(fd / (2 * h) - dS[p, :, :, k]).max() <= 1e-8


@pytest.mark.parametrize("ov", [OV, STRONG])
def test_lowdin_factor(ov):
    s = _system(10, 1)
    S = overlap.overlap(s.R, ov)
    Z = overlap.lowdin(S)
    n = S.shape[0]
    assert np.abs(Z.T @ S @ Z - np.eye(n)).max() <= 1e-13
    ref = np.linalg.inv(np.real(scipy.linalg.sqrtm(S)))
    assert np.abs(Z - ref).max() <= 1e-12


def _cholesky_z(S):
    L = np.linalg.cholesky(S)
    return np.linalg.inv(L).T          # Z^T S Z = L^-1 L L^T L^-T = I


@pytest.mark.parametrize("T_e", [3000.0, 20000.0])
def test_density_matrix_matches_generalized_eigenproblem(T_e):
    s = _system(10, 1)
    rng = np.random.default_rng(4)
    F = _fock(s, rng)
    S = overlap.overlap(s.R, STRONG)
    beta = density.beta_of(T_e)
    dm = overlap.density_matrix(F, overlap.lowdin(S), s.n_elec, beta)
    eps, C = scipy.linalg.eigh(F, S)
    mu = density.solve_mu(eps, 0.5 * s.n_elec, beta)
    f = density.fermi(eps, mu, beta)
    P = 2.0 * (C * f) @ C.T
    scale = np.abs(P).max()
    assert abs(dm["mu"] - mu) <= 1e-9
    assert np.abs(dm["P"] - P).max() <= 1e-11 * scale
    assert abs(np.trace(dm["P"] @ S) - s.n_elec) <= 1e-10
    dm2 = overlap.density_matrix(F, _cholesky_z(S), s.n_elec, beta)
    assert np.abs(dm2["P"] - dm["P"]).max() <= 1e-11 * scale


def test_response_matches_central_differences_and_any_z():
    s = _system(8, 2)
    rng = np.random.default_rng(6)
    F = _fock(s, rng)
    S = overlap.overlap(s.R, STRONG)
    Z = overlap.lowdin(S)
    beta = density.beta_of(5000.0)
    F1 = rng.standard_normal(F.shape)
    F1 = 0.5 * (F1 + F1.T)
    P1 = overlap.response(F, F1, Z, s.n_elec, beta)
    h = 1e-5
    fd = (overlap.density_matrix(F + h * F1, Z, s.n_elec, beta)["P"]
          - overlap.density_matrix(F - h * F1, Z, s.n_elec, beta)["P"]) / (2 * h)
    scale = np.abs(P1).max()
    assert np.abs(P1 - fd).max() <= 1e-6 * scale
    assert abs(np.trace(P1 @ S)) <= 1e-11 * scale * F.shape[0]
    P1c = overlap.response(F, F1, _cholesky_z(S), s.n_elec, beta)
    assert np.abs(P1c - P1).max() <= 1e-10 * scale


def _grand_potential(F, S, mu, beta):
    eps = scipy.linalg.eigh(F, S, eigvals_only=True)
    return -2.0 / beta * np.sum(np.logaddexp(0.0, -beta * (eps - mu)))


@pytest.mark.parametrize("T_e", [3000.0, 10000.0])
def test_pulay_term_is_the_overlap_derivative_of_the_grand_potential(T_e):
    s = _system(6, 3)
    rng = np.random.default_rng(8)
    F = _fock(s, rng)
    beta = density.beta_of(T_e)
    S = overlap.overlap(s.R, STRONG)
    Z = overlap.lowdin(S)
    dm = overlap.density_matrix(F, Z, s.n_elec, beta)
    got = overlap.pulay_forces(s.R, STRONG, F, dm["P"], Z)
    h = 1e-5
    fd = np.zeros_like(got)
    for I in range(s.n_atoms):
        for k in range(3):
            Rp, Rm = s.R.copy(), s.R.copy()
            Rp[I, k] += h
            Rm[I, k] -= h
            fd[I, k] = -(_grand_potential(F, overlap.overlap(Rp, STRONG), dm["mu"], beta)
                         - _grand_potential(F, overlap.overlap(Rm, STRONG), dm["mu"], beta)) / (2 * h)
    print(f"T_e {T_e:.0f} K: max |Pulay| {np.abs(got).max():.3e}, max |diff| {np.abs(got - fd).max():.2e}")
    assert np.abs(got).max() > 1e-2
    assert np.abs(got - fd).max() <= 1e-6 * np.abs(got).max()
    # the identity overlap has no Pulay term
    I = np.eye(F.shape[0])
    assert np.abs(overlap.pulay_forces(s.R, OverlapModel(0.0, 1.4, 0.4), F, dm["P"], I)).max() == 0.0
