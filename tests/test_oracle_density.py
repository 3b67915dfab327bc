"""Pins of the oracle's Fermi density matrix, entropy and canonical response."""

import numpy as np
import pytest

from synth import carbon_cluster
from oracle import model, density


def _sym(rng, n, scale=1.0):
    a = rng.standard_normal((n, n)) * scale
    return a + a.T


def test_two_level_closed_form():
    # F = [[a, b], [b, a]]: eigenvalues a -+ b, eigenvectors (1, +-1)/sqrt 2.
    a, b, beta = -1.0, -0.4, 2.0
    F = np.array([[a, b], [b, a]])
    dm = density.density_matrix(F, 2.0, beta)
    # one electron pair: f1 + f2 = 1 with f = 1/(1+exp(beta(e - mu))) -> mu = a (symmetric levels)
    f1 = 1.0 / (1.0 + np.exp(beta * (a + b - a)))
    f2 = 1.0 - f1
    D = 0.5 * np.array([[f1 + f2, f1 - f2], [f1 - f2, f1 + f2]])
    np.testing.assert_allclose(dm["P"], 2.0 * D, atol=1e-15)
    assert dm["mu"] == pytest.approx(a, abs=1e-12)


def test_density_invariants():
    sys_ = carbon_cluster(8, 3)
    rng = np.random.default_rng(3)
    F = _sym(rng, sys_.n_orb, 3.0)
    beta = density.beta_of(5000.0)
    dm = density.density_matrix(F, sys_.n_elec, beta)
    P = dm["P"]
    assert np.trace(P) == pytest.approx(sys_.n_elec, abs=1e-11 * sys_.n_elec)
    np.testing.assert_allclose(P, P.T, atol=1e-14)
    np.testing.assert_allclose(P @ F, F @ P, atol=1e-12)
    w = np.linalg.eigvalsh(P)
    assert w.min() > -1e-13 and w.max() < 2.0 + 1e-13


def test_low_temperature_idempotent():
    rng = np.random.default_rng(4)
    eps = np.concatenate([np.linspace(-10, -2, 6), np.linspace(2, 9, 6)])
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    F = (Q * eps) @ Q.T
    beta = density.beta_of(100.0)
    P = density.density_matrix(F, 12.0, beta)["P"]
    D = 0.5 * P
    gap = 4.0
    assert np.abs(D @ D - D).max() <= 12 * np.exp(-beta * gap / 2) + 1e-14
    np.testing.assert_allclose(D, (Q[:, :6]) @ Q[:, :6].T, atol=1e-12)


def test_entropy_thermodynamic_identity():
    # S/k_B = beta^2 dOmega/dbeta at fixed mu, Omega = -(1/beta) sum ln(1 + exp(-beta (e - mu)))
    rng = np.random.default_rng(5)
    eps = rng.uniform(-3, 3, 20)
    mu, beta = 0.3, 1.7
    f = density.fermi(eps, mu, beta)

    def omega(b):
        return -np.sum(np.logaddexp(0.0, -b * (eps - mu))) / b

    h = 1e-5
    dO = (omega(beta + h) - omega(beta - h)) / (2 * h)
    assert density.entropy(f) == pytest.approx(beta * beta * dO, rel=1e-8)
    assert density.entropy(np.full(7, 0.5)) == pytest.approx(7 * np.log(2.0), rel=1e-15)
    assert density.entropy(np.array([0.0, 1.0])) == 0.0


def test_response_matches_finite_differences():
    sys_ = carbon_cluster(5, 6)
    rng = np.random.default_rng(6)
    F = _sym(rng, sys_.n_orb, 2.0)
    F1 = _sym(rng, sys_.n_orb, 1.0)
    beta = density.beta_of(3000.0)
    P1 = density.response(F, F1, sys_.n_elec, beta)
    h = 1e-5
    fd = (density.density_matrix(F + h * F1, sys_.n_elec, beta)["P"]
          - density.density_matrix(F - h * F1, sys_.n_elec, beta)["P"]) / (2 * h)
    np.testing.assert_allclose(P1, fd, atol=2e-8 * np.abs(fd).max())
    assert abs(np.trace(P1)) < 1e-13


def test_response_special_cases():
    rng = np.random.default_rng(7)
    n = 12
    F = _sym(rng, n, 2.0)
    beta = 2.5
    # a constant shift of F only moves mu: canonical response vanishes
    assert np.abs(density.response(F, np.eye(n), 12.0, beta)).max() < 1e-13
    # a perturbation commuting with F: closed form diag(-beta f(1-f)(eps - eps_bar))
    dm = density.density_matrix(F, 12.0, beta)
    f, eps, C = dm["f"], dm["eps"], dm["C"]
    w = f * (1 - f)
    ebar = np.sum(w * eps) / np.sum(w)
    ref = 2.0 * (C * (-beta * w * (eps - ebar))) @ C.T
    np.testing.assert_allclose(density.response(F, F, 12.0, beta, dm), ref, atol=1e-13)
