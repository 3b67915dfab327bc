"""Finite-temperature density matrix, its canonical response and the entropy.

Plain definitions by eigendecomposition (S = I, so Z = I in eqs. 18-20):
  * Fermi occupations f_i = 1 / (exp(beta (eps_i - mu0)) + 1) (eq. 7) with mu0
    fixed by sum_i f_i = N_occ (eq. 8), and D0 = sum_i f_i C_i C_i^T (eq. 2,
    eq. 19);
  * the canonical first-order response dD/dlambda of D[F0 + lambda F1] at
    lambda = 0 (eq. 36) with mu re-solved so that Tr D stays N_occ.  The paper
    defers its DMPT recipe to its ref. [16]; the quantity is the derivative of
    a matrix function, whose textbook closed form is the Daleckii-Krein
    (Loewner) formula D1 = C (Phi o C^T F1 C) C^T with
    Phi_ab = (f_a - f_b) / (eps_a - eps_b) (Phi_aa = f'(eps_a)), followed by the
    chemical-potential term (d mu/d lambda) dD/dmu with dD/dmu = beta D(I - D).
  * the electronic entropy S(f) / k_B = -sum_i [f ln f + (1 - f) ln(1 - f)]
    (eq. 4).
Spin: D is the one-spin density matrix (Tr D = N_occ = N_e / 2); the
interface returns the spin-summed P = 2 D.
"""

from __future__ import annotations

import numpy as np

KB_EV_PER_K = 8.617333262e-5  # Boltzmann constant, eV/K (CODATA 2018)


def beta_of(T_e: float) -> float:
    """Inverse electronic temperature 1 / (k_B T_e) in 1/eV."""
    return 1.0 / (KB_EV_PER_K * T_e)


def fermi(eps: np.ndarray, mu: float, beta: float) -> np.ndarray:
    """Occupations of eq. 7, evaluated without overflow."""
    x = beta * (np.asarray(eps) - mu)
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def solve_mu(eps: np.ndarray, n_occ: float, beta: float, max_iter: int = 400) -> float:
    """Chemical potential of eq. 8 by bisection (sum f is strictly monotone in mu)."""
    lo = float(np.min(eps)) - 40.0 / beta
    hi = float(np.max(eps)) + 40.0 / beta
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if np.sum(fermi(eps, mid, beta)) < n_occ:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def density_matrix(F: np.ndarray, n_elec: float, beta: float) -> dict:
    """Spin-summed P = 2 D0 with D0 = C diag(f) C^T, f from eq. 7 at the mu0 of
    eq. 8 (N_occ = n_elec / 2).  Returns P, mu, eps, C, f."""
    eps, C = np.linalg.eigh(np.asarray(F, dtype=np.float64))
    mu = solve_mu(eps, 0.5 * n_elec, beta)
    f = fermi(eps, mu, beta)
    D = (C * f) @ C.T
    return dict(P=2.0 * D, mu=mu, eps=eps, C=C, f=f)


def entropy(f: np.ndarray) -> float:
    """S(f) / k_B of eq. 4 over one-spin orbitals, with 0 ln 0 = 0."""
    f = np.asarray(f, dtype=np.float64)
    s = np.zeros_like(f)
    m = (f > 0.0) & (f < 1.0)
    s[m] = -(f[m] * np.log(f[m]) + (1.0 - f[m]) * np.log1p(-f[m]))
    return float(np.sum(s))


def loewner_matrix(eps: np.ndarray, f: np.ndarray, beta: float) -> np.ndarray:
    """Phi_ab = (f_a - f_b)/(eps_a - eps_b), Phi_aa = -beta f_a (1 - f_a).

    Evaluated as -beta f_lo (1 - f_hi) expm1(x)/x with x = beta (eps_lo - eps_hi)
    <= 0, an exact rewriting of the divided difference that neither overflows
    nor cancels."""
    ea = eps[:, None]
    eb = eps[None, :]
    lo_is_a = ea <= eb
    f_lo = np.where(lo_is_a, f[:, None], f[None, :])
    f_hi = np.where(lo_is_a, f[None, :], f[:, None])
    x = beta * (np.minimum(ea, eb) - np.maximum(ea, eb))
    ratio = np.ones_like(x)
    nz = x != 0.0
    ratio[nz] = np.expm1(x[nz]) / x[nz]
    return -beta * f_lo * (1.0 - f_hi) * ratio


def response(F: np.ndarray, F1: np.ndarray, n_elec: float, beta: float, dm: dict | None = None) -> np.ndarray:
    """Spin-summed canonical response P1 = 2 dD0/dlambda of D0[F + lambda F1]
    (eq. 36), Tr P1 = 0.

    For a symmetric F1 the response is symmetric; the result is returned as
    D1 + D1^T, so that rounding leaves it exactly symmetric.  (An
    antisymmetric residue of rounding size would otherwise be amplified by the
    Jacobian's large eigenvalues on antisymmetric matrices when a Krylov basis
    (eq. 34) is built from repeated responses, and the basis would leave the
    symmetric matrices the method works on.)"""
    if dm is None:
        dm = density_matrix(F, n_elec, beta)
    C, eps, f = dm["C"], dm["eps"], dm["f"]
    Phi = loewner_matrix(eps, f, beta)
    D1 = C @ (Phi * (C.T @ np.asarray(F1, dtype=np.float64) @ C)) @ C.T
    w = f * (1.0 - f)
    sw = np.sum(w)
    if sw > 0.0:
        D1 = D1 - (np.trace(D1) / sw) * ((C * w) @ C.T)
    return D1 + D1.T
