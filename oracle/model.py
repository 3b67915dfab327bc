"""Synthetic NDDO-type sp Hamiltonian: h(R), G(P) and V_nn in plain FP64.

Paper: the Fock matrix is F = h + G (eq. 6, eq. 17 with S = I for NDDO,
Methods section 1), the electron-electron matrix is G(D) = 2J(D) - K(D)
(eq. 3), and under NDDO only integrals (mu nu | lambda sigma) with mu, nu on one
atom and lambda, sigma on one atom survive.  For a spin-summed density P the
two-electron part of the Fock matrix is therefore

    G(P)_{mu nu} = sum_{lambda sigma} P_{lambda sigma}
                   [ (mu nu | lambda sigma) - 1/2 (mu lambda | nu sigma) ],

which equals the paper's 2J(D) - K(D) at D = P / 2.  The integral values are
the synthetic ones of the seeded clusters (the AM1/MNDO parameter sets the
paper uses are not available):
  * one-centre: (ss|ss)=Gss, (ss|pp)=Gsp, (sp|sp)=Hsp, (pp|pp)=Gpp,
    (pp|p'p')=Gp2, (pp'|pp')=Hpp=(Gpp-Gp2)/2, all others zero;
  * two-centre: W_AB[(mu nu),(lambda sigma)] = coul_k / sqrt(R^2 + coul_a^2)
    * (1 + noise_amp * noise_AB), a symmetric 10 x 10 block per pair.
Reading of the silent points: hopping is t(R) = t0 exp(-(R - r0)/lam) times
direction cosines (s-s: t; s_A-p_B: t l; p_A-s_B: -t l; p_A-p_B: t l l^T,
l = (R_B - R_A)/R); every atom carries a core charge Z that attracts electrons
through the (ss) column of W and repels other cores as Z^2 W[ss,ss]; a
short-range repulsion a_rep exp(-(R - r0_rep)/rho_rep) keeps the cluster
bound.  Without the core terms each atom would carry a net charge of -4e.
"""

from __future__ import annotations

import numpy as np

# Packed orbital pairs of one atom, row-major upper triangle of the 4x4 block.
PAIRS10 = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
IDX10 = np.zeros((4, 4), dtype=np.int64)
for _k, (_a, _b) in enumerate(PAIRS10):
    IDX10[_a, _b] = _k
    IDX10[_b, _a] = _k
# Multiplicity of a packed pair in a symmetric contraction (off-diagonal counted twice).
MULT10 = np.array([1.0 if a == b else 2.0 for (a, b) in PAIRS10])


def pair_list(n_atoms: int):
    """Unordered atom pairs (A < B), row-major."""
    a, b = np.triu_indices(n_atoms, 1)
    return a, b


def unpack55(noise55: np.ndarray) -> np.ndarray:
    """(Np, 55) packed upper triangles -> (Np, 10, 10) symmetric blocks."""
    noise55 = np.asarray(noise55, dtype=np.float64)
    iu = np.triu_indices(10)
    out = np.zeros((noise55.shape[0], 10, 10))
    out[:, iu[0], iu[1]] = noise55
    out[:, iu[1], iu[0]] = noise55
    return out


def pair_geometry(R: np.ndarray, params):
    """Per pair: displacement, distance, unit vector B-A, gamma and t with their
    radial derivatives."""
    a, b = pair_list(R.shape[0])
    d = R[b] - R[a]
    r = np.sqrt(np.sum(d * d, axis=1))
    l = d / r[:, None]
    s2 = r * r + params.coul_a ** 2
    gamma = params.coul_k / np.sqrt(s2)
    dgamma = -params.coul_k * r / s2 ** 1.5
    t = params.t0 * np.exp(-(r - params.r0_hop) / params.lam_hop)
    dt = -t / params.lam_hop
    return dict(a=a, b=b, d=d, r=r, l=l, gamma=gamma, dgamma=dgamma, t=t, dt=dt)


def two_centre_base(noise55, params) -> np.ndarray:
    """R-independent factor J + noise_amp * noise of every W_AB block, with the
    10 x 10 pattern J taken from the model parameters (packed, 55 entries)."""
    J = unpack55(np.asarray(params.j55(), dtype=np.float64)[None, :])
    return J + params.noise_amp * unpack55(noise55)


def two_centre_blocks(R, noise55, params) -> np.ndarray:
    """W_AB for every pair, (Np, 10, 10)."""
    g = pair_geometry(R, params)
    return g["gamma"][:, None, None] * two_centre_base(noise55, params)


def onecenter_eri(oc: np.ndarray) -> np.ndarray:
    """Four-index one-centre integrals of one atom, (4,4,4,4), from
    (Gss, Gsp, Gpp, Gp2, Hsp); chemists' notation (mu nu|lambda sigma)."""
    gss, gsp, gpp, gp2, hsp = [float(x) for x in oc]
    hpp = 0.5 * (gpp - gp2)
    E = np.zeros((4, 4, 4, 4))
    E[0, 0, 0, 0] = gss
    for i in (1, 2, 3):
        E[0, 0, i, i] = E[i, i, 0, 0] = gsp
        for (p, q, r_, s) in ((0, i, 0, i), (0, i, i, 0), (i, 0, 0, i), (i, 0, i, 0)):
            E[p, q, r_, s] = hsp
        E[i, i, i, i] = gpp
        for j in (1, 2, 3):
            if j == i:
                continue
            E[i, i, j, j] = gp2
            for (p, q, r_, s) in ((i, j, i, j), (i, j, j, i), (j, i, i, j), (j, i, j, i)):
                E[p, q, r_, s] = hpp
    return E


def _pack(block4: np.ndarray) -> np.ndarray:
    """(..., 4, 4) symmetric blocks -> (..., 10) with off-diagonals doubled, so
    that W @ pack(P_B) contracts W with the full block."""
    out = np.empty(block4.shape[:-2] + (10,))
    for k, (a, b) in enumerate(PAIRS10):
        out[..., k] = block4[..., a, b] * MULT10[k]
    return out


def _unpack10(v10: np.ndarray) -> np.ndarray:
    """(..., 10) -> symmetric (..., 4, 4), no multiplicity factors."""
    out = np.empty(v10.shape[:-1] + (4, 4))
    for k, (a, b) in enumerate(PAIRS10):
        out[..., a, b] = v10[..., k]
        out[..., b, a] = v10[..., k]
    return out


def _atom_blocks(M: np.ndarray, n_atoms: int) -> np.ndarray:
    """Diagonal 4x4 blocks of an (n, n) matrix, (N, 4, 4)."""
    Mb = M.reshape(n_atoms, 4, n_atoms, 4)
    idx = np.arange(n_atoms)
    return Mb[idx, :, idx, :]


def hopping_block(t, l):
    """4x4 hopping blocks h_AB for arrays of t (Np,) and l (Np, 3)."""
    blk = np.empty(t.shape + (4, 4))
    blk[..., 0, 0] = t
    blk[..., 0, 1:] = t[..., None] * l
    blk[..., 1:, 0] = -t[..., None] * l
    blk[..., 1:, 1:] = t[..., None, None] * l[..., :, None] * l[..., None, :]
    return blk


def hcore(R, onecenter, noise55, params) -> np.ndarray:
    """One-electron matrix h(R) (eq. 6's h), dense (n, n) FP64.

    On-site energies, hopping blocks between atoms and the attraction of every
    electron on atom A to the cores of all other atoms B: h_AA -= Z_B W_AB[:, ss].
    """
    N = R.shape[0]
    n = 4 * N
    h = np.zeros((n, n))
    for A in range(N):
        h[4 * A, 4 * A] = params.eps_s
        for i in (1, 2, 3):
            h[4 * A + i, 4 * A + i] = params.eps_p
    if N < 2:
        return h
    g = pair_geometry(R, params)
    a, b = g["a"], g["b"]
    blk = hopping_block(g["t"], g["l"])
    hb = h.reshape(N, 4, N, 4)
    hb[a, :, b, :] = blk
    hb[b, :, a, :] = np.swapaxes(blk, 1, 2)
    W = g["gamma"][:, None, None] * two_centre_base(noise55, params)
    core_a = np.zeros((N, 10))
    np.add.at(core_a, a, -params.z_core * W[:, :, 0])   # electrons on A, core of B
    np.add.at(core_a, b, -params.z_core * W[:, 0, :])   # electrons on B, core of A
    for A in range(N):
        hb[A, :, A, :] += _unpack10(core_a[A])
    return h


def two_electron(P, R, onecenter, noise55, params, chunk: int = 20000) -> np.ndarray:
    """G(P) for a spin-summed density P (eq. 3 at D = P/2), dense (n, n) FP64.

    Built block by block from the NDDO integral classes:
      one-centre  G_AA += sum_{ls} P_ls [ (mn|ls) - 1/2 (ml|ns) ]   (all on A)
      Coulomb     G_AA[(mn)] += sum_B W_AB[(mn), :] . pack(P_BB)
      exchange    G_AB[m, l] = -1/2 sum_{n in A, s in B} P_ns W_AB[(mn), (ls)]
    """
    P = np.asarray(P, dtype=np.float64)
    N = R.shape[0]
    n = 4 * N
    G = np.zeros((n, n))
    Gb = G.reshape(N, 4, N, 4)
    Pb = P.reshape(N, 4, N, 4)
    PAA = _atom_blocks(P, N)
    for A in range(N):
        E = onecenter_eri(onecenter[A])
        Gb[A, :, A, :] += (np.einsum("mnls,ls->mn", E, PAA[A])
                           - 0.5 * np.einsum("mlns,ls->mn", E, PAA[A]))
    if N < 2:
        return G
    a_all, b_all = pair_list(N)
    g = pair_geometry(R, params)
    pk = _pack(PAA)                       # (N, 10)
    coul = np.zeros((N, 10))
    for s in range(0, a_all.size, chunk):
        a = a_all[s:s + chunk]
        b = b_all[s:s + chunk]
        W = g["gamma"][s:s + chunk, None, None] * two_centre_base(noise55[s:s + chunk], params)
        np.add.at(coul, a, np.einsum("pij,pj->pi", W, pk[b]))
        np.add.at(coul, b, np.einsum("pij,pi->pj", W, pk[a]))
        W4 = W[:, IDX10[:, :, None, None], IDX10[None, None, :, :]]   # (p, m, n, l, s)
        PAB = Pb[a, :, b, :]                                          # (p, n, s)
        X = -0.5 * np.einsum("pmnls,pns->pml", W4, PAB)
        Gb[a, :, b, :] += X
        Gb[b, :, a, :] += np.swapaxes(X, 1, 2)
    for A in range(N):
        Gb[A, :, A, :] += _unpack10(coul[A])
    return G


def fock(X, R, onecenter, noise55, params) -> np.ndarray:
    """F(X) = h + G(X) (eq. 17 with S = I, so P = X)."""
    return hcore(R, onecenter, noise55, params) + two_electron(X, R, onecenter, noise55, params)


def nuclear_repulsion(R, noise55, params) -> float:
    """V_nn = sum_{A<B} [ Z^2 W_AB[ss, ss] + a_rep exp(-(R - r0_rep)/rho_rep) ]."""
    if R.shape[0] < 2:
        return 0.0
    g = pair_geometry(R, params)
    wss = g["gamma"] * (params.j55()[0] + params.noise_amp * np.asarray(noise55[:, 0], dtype=np.float64))
    rep = params.a_rep * np.exp(-(g["r"] - params.r0_rep) / params.rho_rep)
    return float(np.sum(params.z_core ** 2 * wss + rep))
