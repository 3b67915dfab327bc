"""Non-orthogonal basis: the overlap S(R), a congruence factor Z, the density
matrix, its response and the Pulay force term, in plain FP64.

TEST INFRASTRUCTURE: like the rest of oracle/, this module is the reference
the GPU path is checked against and is never called by the product path.

Paper, Methods section 3 and the forces of section 6:
  * the orthogonalised Fock matrix F_perp = Z^T F Z (eq. 18) with any Z that
    satisfies Z^T S Z = I (eq. 21), the symmetric (Loewdin) choice being
    Z = S^(-1/2);
  * D0_perp = Fermi function of F_perp with mu0 fixed by Tr D0_perp = N_occ
    (eq. 19), and the transform back D0 = Z D0_perp Z^T (eq. 20);
  * the response of D0 to a Fock perturbation F1 is Z times the response of
    D0_perp to Z^T F1 Z, times Z^T (eq. 36);
  * the gradient of the shadow energy gains the Pulay term
    -2 Tr[Z Z^T F D S_{R_I}] (eqs. 37, 39, 41), D the one-spin density matrix;
    the force is minus the gradient.  With the spin-summed P = 2 D the force
    term is + Tr[S^-1 F P S_{R_I}], since Z Z^T = S^-1 for every Z of eq. 21.

The paper's semiempirical models take S = I, and its NDDO integrals are not
available here, so the overlap is synthetic (a reading; the paper gives no
form): S_AA = I, and for A != B the 4 x 4 block has the angular structure of
the hopping block of oracle/model.py (s-s: s; s_A-p_B: s l; p_A-s_B: -s l;
p_A-p_B: s l l^T, l = (R_B - R_A)/R) with the radial factor
s(R) = s0 exp(-(R - r0)/lam).
"""

from __future__ import annotations

import numpy as np

from . import density, model

# ov: any object with the radial constants s0, r0, lam (synth.OverlapModel)


def _radial(r, ov):
    s = ov.s0 * np.exp(-(r - ov.r0) / ov.lam)
    return s, -s / ov.lam


def overlap(R, ov) -> np.ndarray:
    """S(R), dense (n, n), symmetric, unit atom blocks on the diagonal."""
    R = np.asarray(R, dtype=np.float64)
    N = R.shape[0]
    S = np.eye(4 * N)
    if N < 2:
        return S
    a, b = model.pair_list(N)
    d = R[b] - R[a]
    r = np.sqrt(np.sum(d * d, axis=1))
    l = d / r[:, None]
    s, _ = _radial(r, ov)
    blk = model.hopping_block(s, l)
    Sb = S.reshape(N, 4, N, 4)
    Sb[a, :, b, :] = blk
    Sb[b, :, a, :] = np.transpose(blk, (0, 2, 1))
    return S


def overlap_derivative_blocks(R, ov):
    """Per pair A < B: dS_AB / d(R_B - R_A), shape (n_pair, 4, 4, 3), with the
    pair lists.  dS_AB/dR_B is this, dS_AB/dR_A its negative."""
    R = np.asarray(R, dtype=np.float64)
    a, b = model.pair_list(R.shape[0])
    d = R[b] - R[a]
    r = np.sqrt(np.sum(d * d, axis=1))
    l = d / r[:, None]
    s, ds = _radial(r, ov)
    # d l_i / d d_k = (delta_ik - l_i l_k) / r, d r / d d_k = l_k
    dl = (np.eye(3)[None] - l[:, :, None] * l[:, None, :]) / r[:, None, None]
    out = np.empty((a.size, 4, 4, 3))
    out[:, 0, 0, :] = ds[:, None] * l
    sp = ds[:, None, None] * l[:, :, None] * l[:, None, :] + s[:, None, None] * dl   # d(s l_i)/d d_k
    out[:, 0, 1:, :] = sp
    out[:, 1:, 0, :] = -sp
    ll = l[:, :, None] * l[:, None, :]
    dll = dl[:, :, None, :] * l[:, None, :, None] + l[:, :, None, None] * dl[:, None, :, :]
    out[:, 1:, 1:, :] = ds[:, None, None, None] * ll[..., None] * l[:, None, None, :] + s[:, None, None, None] * dll
    return a, b, out


def lowdin(S) -> np.ndarray:
    """Z = S^(-1/2) by the eigendecomposition of S (the symmetric choice of
    eq. 21)."""
    w, U = np.linalg.eigh(np.asarray(S, dtype=np.float64))
    if w[0] <= 0.0:
        raise ValueError("overlap matrix is not positive definite")
    return (U / np.sqrt(w)) @ U.T


def density_matrix(F, Z, n_elec: float, beta: float) -> dict:
    """Spin-summed P = 2 Z D0_perp Z^T (eqs. 18-20).  Returns P, mu, and the
    orthogonal-basis quantities of oracle.density (eps, C, f, P_perp, F_perp)."""
    Z = np.asarray(Z, dtype=np.float64)
    Fp = Z.T @ np.asarray(F, dtype=np.float64) @ Z
    Fp = 0.5 * (Fp + Fp.T)
    dm = density.density_matrix(Fp, n_elec, beta)
    P = Z @ dm["P"] @ Z.T
    return dict(P=0.5 * (P + P.T), mu=dm["mu"], eps=dm["eps"], C=dm["C"], f=dm["f"], P_perp=dm["P"], F_perp=Fp,
                dm_perp=dm)


def response(F, F1, Z, n_elec: float, beta: float, dm: dict | None = None) -> np.ndarray:
    """Spin-summed canonical response of eq. 36: Z P1_perp Z^T with P1_perp the
    response of the orthogonal-basis density matrix to Z^T F1 Z."""
    Z = np.asarray(Z, dtype=np.float64)
    if dm is None:
        dm = density_matrix(F, Z, n_elec, beta)
    F1p = Z.T @ np.asarray(F1, dtype=np.float64) @ Z
    F1p = 0.5 * (F1p + F1p.T)
    P1p = density.response(dm["F_perp"], F1p, n_elec, beta, dm["dm_perp"])
    P1 = Z @ P1p @ Z.T
    return 0.5 * (P1 + P1.T)


def pulay_forces(R, ov, F, P, Z) -> np.ndarray:
    """Force term of eq. 41, (N, 3) eV/Angstrom: + Tr[Z Z^T F P S_{R_I}] for the
    spin-summed P (minus the gradient term -2 Tr[Z Z^T F D S_{R_I}])."""
    R = np.asarray(R, dtype=np.float64)
    N = R.shape[0]
    out = np.zeros((N, 3))
    if N < 2:
        return out
    Z = np.asarray(Z, dtype=np.float64)
    Q = Z @ Z.T @ np.asarray(F, dtype=np.float64) @ np.asarray(P, dtype=np.float64)
    # Tr[Q S_R] = sum over the two off-diagonal blocks of each pair
    M = (Q + Q.T).reshape(N, 4, N, 4)
    a, b, dS = overlap_derivative_blocks(R, ov)
    g = np.einsum("pij,pijk->pk", M[a, :, b, :], dS)   # d Tr[Q S] / d(R_B - R_A) per pair
    np.add.at(out, b, g)
    np.add.at(out, a, -g)
    return out

