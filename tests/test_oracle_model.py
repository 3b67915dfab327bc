"""Pins of the oracle's h(R), G(P) and V_nn against independent constructions.

G(P) is checked against a brute-force contraction of the full four-index
integral tensor (built entry by entry from the NDDO integral classes), against
closed forms for one atom and for two atoms, and against the symmetries every
two-electron matrix has (linearity, Tr[Q G(P)] = Tr[P G(Q)], symmetric output).
"""

import numpy as np
import pytest

from synth import carbon_cluster, ModelParams
from oracle import model


def _sym(rng, n, scale=1.0):
    a = rng.standard_normal((n, n)) * scale
    return a + a.T


def _full_eri(sys_):
    """(mu nu|lambda sigma) over all orbitals, entry by entry."""
    N = sys_.n_atoms
    n = 4 * N
    eri = np.zeros((n, n, n, n))
    gss, gsp, gpp, gp2, hsp = sys_.onecenter[0]
    hpp = 0.5 * (gpp - gp2)

    def one(m, nn, l, s):
        # classes of one-centre integrals between s(0) and p(1..3)
        if m == nn and l == s:
            if m == 0 and l == 0:
                return gss
            if (m == 0) != (l == 0):
                return gsp
            return gpp if m == l else gp2
        if {m, nn} == {l, s} and m != nn:
            return hsp if 0 in (m, nn) else hpp
        return 0.0

    for A in range(N):
        for m in range(4):
            for nn in range(4):
                for l in range(4):
                    for s in range(4):
                        eri[4 * A + m, 4 * A + nn, 4 * A + l, 4 * A + s] = one(m, nn, l, s)
    W = model.two_centre_blocks(sys_.R, sys_.noise, sys_.params)
    a, b = model.pair_list(N)
    for p, (A, B) in enumerate(zip(a, b)):
        for m in range(4):
            for nn in range(4):
                for l in range(4):
                    for s in range(4):
                        v = W[p, model.IDX10[m, nn], model.IDX10[l, s]]
                        eri[4 * A + m, 4 * A + nn, 4 * B + l, 4 * B + s] = v
                        eri[4 * B + l, 4 * B + s, 4 * A + m, 4 * A + nn] = v
    return eri


@pytest.mark.parametrize("pattern", ["monopole", "allones"])
def test_G_matches_bruteforce_eri(pattern):
    p = ModelParams(j_pattern=pattern)
    sys_ = carbon_cluster(3, 11, params=p)
    rng = np.random.default_rng(0)
    P = _sym(rng, sys_.n_orb)
    eri = _full_eri(sys_)
    ref = np.einsum("mnls,ls->mn", eri, P) - 0.5 * np.einsum("mlns,ls->mn", eri, P)
    G = model.two_electron(P, sys_.R, sys_.onecenter, sys_.noise, p)
    np.testing.assert_allclose(G, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_G_single_atom_closed_form():
    sys_ = carbon_cluster(1, 3)
    gss, gsp, gpp, gp2, hsp = sys_.onecenter[0]
    hpp = 0.5 * (gpp - gp2)
    rng = np.random.default_rng(1)
    P = _sym(rng, 4)
    G = model.two_electron(P, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    d = np.diag(P)
    # diagonal: sum over l of P_ll [(mm|ll) - 1/2 (ml|ml)]
    assert G[0, 0] == pytest.approx(0.5 * d[0] * gss + (d[1] + d[2] + d[3]) * (gsp - 0.5 * hsp), rel=1e-13)
    for i in (1, 2, 3):
        others = sum(d[j] for j in (1, 2, 3) if j != i)
        ref = d[0] * (gsp - 0.5 * hsp) + 0.5 * d[i] * gpp + others * (gp2 - 0.5 * hpp)
        assert G[i, i] == pytest.approx(ref, rel=1e-13)
    # off-diagonal: 1/2 P_mn [3 (mn|mn) - (mm|nn)]
    for i in (1, 2, 3):
        assert G[0, i] == pytest.approx(0.5 * P[0, i] * (3 * hsp - gsp), rel=1e-13)
    assert G[1, 2] == pytest.approx(0.5 * P[1, 2] * (3 * hpp - gp2), rel=1e-13)


def test_G_two_atoms_hand_case():
    sys_ = carbon_cluster(2, 5)
    W = model.two_centre_blocks(sys_.R, sys_.noise, sys_.params)[0]
    # only the s orbital of B carries density 2 -> Coulomb on A is 2 W[:, ss]
    P = np.zeros((8, 8))
    P[4, 4] = 2.0
    G = model.two_electron(P, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    assert G[0, 0] == pytest.approx(2.0 * W[0, 0], rel=1e-14)
    assert G[1, 2] == pytest.approx(2.0 * W[model.IDX10[1, 2], 0], rel=1e-14)
    assert np.all(G[:4, 4:] == 0.0)
    # a pure s_A-s_B bond order: exchange block G_AB[m, l] = -1/2 P_{s s} W[(m s), (l s)] * 2 (both orders)
    P = np.zeros((8, 8))
    P[0, 4] = P[4, 0] = 1.0
    G = model.two_electron(P, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    for m in range(4):
        for l in range(4):
            ref = -0.5 * W[model.IDX10[m, 0], model.IDX10[l, 0]]
            assert G[m, 4 + l] == pytest.approx(ref, rel=1e-14)
    assert np.all(G[:4, :4] == 0.0)


def test_G_linear_symmetric_and_reciprocal():
    sys_ = carbon_cluster(6, 2)
    rng = np.random.default_rng(2)
    P, Q = _sym(rng, 24), _sym(rng, 24)
    args = (sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    GP, GQ = model.two_electron(P, *args), model.two_electron(Q, *args)
    np.testing.assert_allclose(model.two_electron(2.0 * P - 3.0 * Q, *args), 2.0 * GP - 3.0 * GQ, atol=1e-11)
    np.testing.assert_allclose(GP, GP.T, atol=1e-12)
    assert np.sum(Q * GP) == pytest.approx(np.sum(P * GQ), rel=1e-12)


def test_hcore_dimer_along_x():
    p = ModelParams()
    sys_ = carbon_cluster(2, 4, params=p)
    r = 1.7
    R = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    h = model.hcore(R, sys_.onecenter, sys_.noise, p)
    t = p.t0 * np.exp(-(r - p.r0_hop) / p.lam_hop)
    assert h[0, 4] == pytest.approx(t, rel=1e-14)       # s-s
    assert h[0, 5] == pytest.approx(t, rel=1e-14)       # s_A - px_B
    assert h[1, 4] == pytest.approx(-t, rel=1e-14)      # px_A - s_B
    assert h[1, 5] == pytest.approx(t, rel=1e-14)       # px-px sigma
    for (i, j) in [(0, 6), (0, 7), (2, 4), (2, 6), (3, 7), (1, 6)]:
        assert h[i, j] == 0.0
    gamma = p.coul_k / np.sqrt(r * r + p.coul_a ** 2)
    base = model.two_centre_base(sys_.noise, p)[0]
    assert h[0, 0] == pytest.approx(p.eps_s - p.z_core * gamma * base[0, 0], rel=1e-14)
    assert h[5, 5] == pytest.approx(p.eps_p - p.z_core * gamma * base[0, model.IDX10[1, 1]], rel=1e-14)
    assert h[0, 1] == pytest.approx(-p.z_core * gamma * base[model.IDX10[0, 1], 0], rel=1e-14)
    np.testing.assert_array_equal(h, h.T)


def test_nuclear_repulsion_dimer():
    p = ModelParams()
    sys_ = carbon_cluster(2, 4, params=p)
    r = 2.0
    R = np.array([[0.0, 0.0, 0.0], [0.0, r, 0.0]])
    gamma = p.coul_k / np.sqrt(r * r + p.coul_a ** 2)
    wss = gamma * (1.0 + p.noise_amp * float(sys_.noise[0, 0]))
    ref = p.z_core ** 2 * wss + p.a_rep * np.exp(-(r - p.r0_rep) / p.rho_rep)
    assert model.nuclear_repulsion(R, sys_.noise, p) == pytest.approx(ref, rel=1e-14)


def test_generator_is_seeded_and_shaped():
    a = carbon_cluster(30, 9)
    b = carbon_cluster(30, 9)
    np.testing.assert_array_equal(a.R, b.R)
    np.testing.assert_array_equal(a.noise, b.noise)
    assert a.noise.dtype == np.float32 and a.noise.shape == (435, 55)
    d = np.sqrt(((a.R[:, None] - a.R[None]) ** 2).sum(-1)) + np.eye(30) * 10
    assert d.min() >= 1.3
    assert np.abs(a.V.mean(0)).max() < 1e-15
